"""Shared-timestep leapfrog step of the N-body/SPH integrator on the device.

One step follows Sec. 3.2: half kick and drift of every particle (predicting
the gas velocity and internal energy at the drifted positions), force
evaluation (tree gravity on all particles, then SPH kernel size, density and
hydro force on the gas), second half kick, and the FP64 energy audit.  Every
arithmetic step runs in libgx; this module only sequences the calls.
"""
from __future__ import annotations

import queue
import threading
from dataclasses import dataclass, field

from . import GX_QUAD, GX_TREE_ALL, GX_TREE_GAS, Engine, GasState, ParticleSet


def _slice(p: ParticleSet, a: int, b: int) -> ParticleSet:
    s = lambda t: None if t is None else t[a:b]
    return ParticleSet(x=p.x[a:b], y=p.y[a:b], z=p.z[a:b], vx=p.vx[a:b], vy=p.vy[a:b],
                       vz=p.vz[a:b], m=p.m[a:b], eps2=s(p.eps2), id=s(p.id), type=s(p.type))


@dataclass
class StepConfig:
    G: float
    dt: float
    theta: float = 0.5
    quad: bool = True
    n_leaf: int = 16
    n_group: int = 256
    sph_leaf: int = 8
    sph_group: int = 64
    n_ngb: float = 64.0
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    h_tol: float = 1e-3
    max_iter: int = 64
    u_floor: float = 0.0


@dataclass
class GalaxyStep:
    """Particles (gas as the contiguous tail [gas_offset, n)) and step buffers."""
    eng: Engine
    p: ParticleSet
    gas_offset: int
    u: object
    cfg: StepConfig
    stats: dict = field(default_factory=dict)
    # record timing events around the kick/drift calls (stats["kd_events"])
    timing: bool = False
    # optional second engine on its own stream: the gas tree, kernel sizes,
    # density and hydro force run there, issued by a worker thread, beside the
    # tree, walk and gravity of all particles; the hydro accelerations go to a
    # zeroed set that the galaxy's stream then adds to the gravity ones (and
    # clears), so the step's results are the same as on one stream
    hydro: object = None

    def __post_init__(self):
        import torch
        # callables run right after each gravity call is enqueued (the
        # asynchronous surrogate uses it to start in the shadow of the SPH
        # and tree phases rather than beside the gravity kernel)
        self.after_gravity = []
        n, o = self.p.n, self.gas_offset
        ng = n - o
        dev = self.p.x.device
        z64 = lambda k: torch.zeros(k, dtype=torch.float64, device=dev)
        self.ax, self.ay, self.az, self.pot = z64(n), z64(n), z64(n), z64(n)
        self.stars = _slice(self.p, 0, o)
        self.gas = _slice(self.p, o, n)
        self.g = GasState.zeros(ng, device=dev)
        self.g.u = self.u
        self.vpred = z64(3 * ng)
        self.upred = z64(ng)
        self.ng = ng
        self._jobs = None
        # with a hydro engine: SPH beside the gravity of all particles (True)
        # or after it, on the same engines (False, e.g. to time the gravity
        # kernel alone)
        self.concurrent = True
        if self.hydro is not None and ng > 0:
            self.hax, self.hay, self.haz = z64(ng), z64(ng), z64(ng)
            # library calls that read sizes back block their thread until
            # their own stream is done, so each stream is driven by a thread
            self._jobs = queue.Queue()
            self._worker = threading.Thread(target=self._run_jobs, daemon=True)
            self._worker.start()

    def _run_jobs(self):
        while True:
            job = self._jobs.get()
            if job is None:
                return
            fn, done = job
            try:
                fn()
            except BaseException as e:  # re-raised by the calling thread
                done["error"] = e
            done["event"].set()

    def close(self):
        """Stop the hydro worker thread (if any)."""
        if self._jobs is not None:
            self._jobs.put(None)
            self._worker.join()
            self._jobs = None

    def _acc(self, a, b):
        return self.ax[a:b], self.ay[a:b], self.az[a:b]

    def _record(self, eng):
        import torch
        e = torch.cuda.Event()
        e.record(eng.stream)
        return e

    def forces(self, predicted: bool = True):
        """Gravity on all particles, then SPH on the gas (accelerations added).

        With a hydro engine the SPH calls are issued by the worker thread on
        the hydro engine's stream once this step's drift is done: the gas
        tree, kernel sizes, density and hydro force run beside the tree, walk
        and gravity kernel of all particles, the hydro force adding into the
        zeroed set (hax, hay, haz); the galaxy's stream then waits for it and
        adds the set to the gravity accelerations (clearing it)."""
        c, s = self.cfg, self.stats
        if self._jobs is None:
            s["tree_all"] = self.eng.tree_build(self.p, GX_TREE_ALL, c.n_leaf, c.n_group)
            s["gravity"] = self.eng.gravity_forces(self.p, c.G, c.theta,
                                                   GX_QUAD if c.quad else 0, self.ax, self.ay,
                                                   self.az, self.pot)
            for f in self.after_gravity:
                f()
            if self.ng:
                self._sph(self.eng, predicted, self._acc(self.gas_offset, self.p.n))
            return
        he = self.hydro
        done = {"event": threading.Event(), "error": None}

        def submit(start):
            def job():
                he.stream.wait_event(start)
                self._sph(he, predicted, (self.hax, self.hay, self.haz))
                done["hydro_done"] = self._record(he)
            self._jobs.put((job, done))

        if self.concurrent:
            submit(self._record(self.eng))  # from the end of the drift
        s["tree_all"] = self.eng.tree_build(self.p, GX_TREE_ALL, c.n_leaf, c.n_group)
        s["gravity"] = self.eng.gravity_forces(self.p, c.G, c.theta, GX_QUAD if c.quad else 0,
                                               self.ax, self.ay, self.az, self.pot)
        if not self.concurrent:
            submit(self._record(self.eng))  # from the end of the gravity kernel
        for f in self.after_gravity:
            f()
        done["event"].wait()
        if done["error"] is not None:
            raise RuntimeError("SPH on the hydro stream failed") from done["error"]
        self.eng.stream.wait_event(done["hydro_done"])
        self.eng.add_accel(*self._acc(self.gas_offset, self.p.n), self.hax, self.hay, self.haz)

    def _sph(self, he, predicted, acc):
        """Gas tree, kernel sizes, density and hydro force (added to acc), all
        with engine he."""
        c, s, ng = self.cfg, self.stats, self.ng
        s["tree_gas"] = he.tree_build(self.gas, GX_TREE_GAS, c.sph_leaf, c.sph_group)
        if predicted:
            vel = (self.vpred[:ng], self.vpred[ng:2 * ng], self.vpred[2 * ng:])
            u = self.upred
        else:
            vel, u = None, None
        gas_view = self.gas if vel is None else ParticleSet(
            x=self.gas.x, y=self.gas.y, z=self.gas.z, vx=vel[0], vy=vel[1], vz=vel[2],
            m=self.gas.m, eps2=self.gas.eps2)
        s["density"] = he.sph_density(gas_view, self.g, c.n_ngb, c.gamma, c.h_tol, c.max_iter,
                                      u=u)
        s["hydro"] = he.sph_forces(gas_view, self.g, *acc, gamma=c.gamma, alpha=c.alpha, u=u)

    def initial_forces(self):
        self.forces(predicted=False)

    def _event(self):
        import torch
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.eng.stream or torch.cuda.current_stream())
        return e

    def step(self):
        c, o, n = self.cfg, self.gas_offset, self.p.n
        dt = c.dt
        ev = [self._event()] if self.timing else None
        # (1) half kick + (2) drift; gas also predicts v and u at the drifted positions
        if o > 0:
            self.eng.kick_drift(self.stars, dt / 2, dt, *self._acc(0, o))
        if self.ng:
            self.eng.kick_drift(self.gas, dt / 2, dt, *self._acc(o, n), u=self.g.u,
                                dudt=self.g.dudt, u_floor=c.u_floor, vpred=self.vpred,
                                upred=self.upred)
        if ev:
            ev.append(self._event())
        # (3) forces
        self.forces(predicted=True)
        if ev:
            ev.append(self._event())
        # (4) second half kick
        if o > 0:
            self.eng.kick_drift(self.stars, dt / 2, 0.0, *self._acc(0, o))
        if self.ng:
            self.eng.kick_drift(self.gas, dt / 2, 0.0, *self._acc(o, n), u=self.g.u,
                                dudt=self.g.dudt, u_floor=c.u_floor)
        if ev:
            ev.append(self._event())
            self.stats["kd_events"] = ev
        return self.stats

    def energy(self):
        m_gas = self.gas.m if self.ng else None
        return self.eng.energy(self.p, self.pot, m_gas, self.g.u if self.ng else None)
