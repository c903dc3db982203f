"""Surrogate-coupled global step (Sec. 3.2): supernova regions of the galaxy
are handed to the learned surrogate and their gas is replaced, by particle
ID, after a delay of `delay` global steps (the paper's 0.1 Myr = 50 steps of
2,000 yr), so the global step never shrinks for the explosions.

Per hand-over, for the K sites of this step (seeded uniform choice among disk
stars whose boxes do not overlap): extract the gas in the (60 pc)^3 box
around each site, pack it into the box's own frame in pc (`gx_sn_gather`),
ambient state, gas tree and voxelization in that frame, U-Net inference,
resampling of as many particles as entered, and transformation back to the
galaxy frame drifted by the box's bulk velocity over the delay
(`gx_sn_unframe`).  The result waits in a queue and is written over the
particles with the same IDs (`gx_sn_replace`) when it falls due.  A region
whose prediction leaves the range the network was trained on is not
replaced: its gas stays with the plain integrator (the fallback), and the
count is reported.

The surrogate has its own library context (its own gas-tree slot).  In the
synchronous mode it runs on the galaxy's stream in the calling thread.  In
the asynchronous mode -- the single-GPU counterpart of the paper's pool
nodes, which work while the main nodes integrate -- the galaxy's stream
copies the gas state and the positions of all particles at the hand-over
into a snapshot (device copies, no wait on the host), and a worker thread
chooses the sites from the snapshot and runs the pipeline on it on the
surrogate's own stream (default priority) while the galaxy steps on, starting after the next step's gravity
kernel (in the shadow of the latency-bound SPH and tree phases, not beside
the compute-bound gravity kernel); the galaxy's stream waits for a result's
completion event only when its replacement falls due.  Both modes
compute the same replacements bit for bit: the same kernels on the same
state, with the uniforms of the resampling drawn from a generator seeded by
the step.  Every arithmetic step runs in libgx.
"""
from __future__ import annotations

import math
import queue as _queue
import threading
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import GX_TREE_GAS, GasState, ParticleSet
from .sn import U_PER_K, SPHConfig, Surrogate

PC_PER_KPC = 1000.0
_SNAP_F64 = ("x", "y", "z", "vx", "vy", "vz", "m", "u")



def keep_in_order(draw, pos, side, kept, seen, chosen, want):
    """One draw of candidate sites, scanned in draw order: a candidate not
    seen before is kept unless its box (edge `side`, centred on its row of
    `pos`) overlaps the box of a site kept earlier, i.e. unless some kept
    site lies closer than `side` on every axis; scanning stops once `chosen`
    holds `want` sites.  `seen` and `chosen` are updated in place; returns
    `kept` (one row per kept site, in keep order) extended by this draw's.

    Only candidates inside a window of +-2 side in x around a candidate can
    overlap it, so the candidates are sorted by x once and each is tested
    exactly against the kept sites of its window (the same decisions as a
    test against every kept site, at a fraction of the host time)."""
    n = pos.shape[0]
    x = pos[:, 0]
    order = np.argsort(x, kind="stable")
    xs = x[order]
    lo = np.searchsorted(xs, x - 2 * side, "left").tolist()
    hi = np.searchsorted(xs, x + 2 * side, "right").tolist()
    ol = order.tolist()
    if kept.shape[0]:  # sites kept from earlier draws
        hit = np.zeros(n, bool)
        for k in kept:
            hit |= (np.abs(pos - k) < side).all(axis=1)
        free = (~hit).tolist()
    else:
        free = [True] * n
    dl, pl = draw.tolist(), pos.tolist()
    mine = set()
    for j in range(n):
        d = dl[j]
        if d in seen:
            continue
        seen.add(d)
        if not free[j]:
            continue
        if hi[j] - lo[j] > 1:
            pj = pl[j]
            if any(abs(pl[k][0] - pj[0]) < side and abs(pl[k][1] - pj[1]) < side
                   and abs(pl[k][2] - pj[2]) < side for k in ol[lo[j]:hi[j]] if k in mine):
                continue
        mine.add(j)
        chosen.append(d)
        if len(chosen) == want:
            break
    return np.vstack([kept, pos[sorted(mine)].reshape(-1, 3)])

@dataclass
class Pending:
    due: int
    ids: object = None      # device int64 [m] particle IDs to overwrite
    new: dict = None        # device FP64 arrays x, y, z, vx, vy, vz, u (galaxy frame)
    done: object = None     # CUDA event on the surrogate's stream (asynchronous mode)
    ready: threading.Event = field(default_factory=threading.Event)
    error: BaseException = None


class SNCoupling:
    def __init__(self, step, surrogate: Surrogate, n_sites: int = 64, delay: int = 50,
                 side_pc: float = 60.0, seed: int = 5, r_max: float = 15.0, z_max: float = 0.3,
                 valid_sigma: float = 8.0, cfg: SPHConfig = SPHConfig(), star_type: int = 1,
                 asynchronous: bool = False, start: str = "after_gravity"):
        import torch
        self.torch = torch
        self.step, self.sur = step, surrogate
        self.eng = surrogate.eng
        self.K, self.delay, self.side = n_sites, delay, side_pc
        self.seed, self.cfg = seed, cfg
        self.valid_sigma = valid_sigma
        p, o = step.p, step.gas_offset
        # candidate sites: stars (particle type star_type; the synthetic sets
        # use 0 dark matter, 1 stars, 2 gas) in the disk, R < r_max, |z| < z_max
        x = p.x[:o].cpu().numpy()
        y = p.y[:o].cpu().numpy()
        z = p.z[:o].cpu().numpy()
        ptype = p.type[:o].cpu().numpy() if p.type is not None else np.full(o, star_type, np.uint8)
        R = np.sqrt(x * x + y * y)
        self.cand = np.nonzero((ptype == star_type) & (R < r_max) & (np.abs(z) < z_max))[0]
        if self.cand.size == 0:
            raise ValueError("no star particles inside the SN site region")
        g = int(math.ceil(n_sites ** (1.0 / 3.0)))
        lat = np.array([((k % g), (k // g) % g, k // (g * g)) for k in range(n_sites)],
                       np.float64) * 1000.0
        self.lattice = torch.as_tensor(lat, device=p.x.device)
        self.queue = deque()
        self.stats = {"regions": 0, "replaced_regions": 0, "fallback_regions": 0,
                      "particles_replaced": 0, "missing_ids": 0}
        self._lock = threading.Lock()
        self.asynchronous = asynchronous
        # asynchronous mode: a hand-over's work starts after the next gravity
        # call's kernel ("after_gravity") or as soon as its snapshot is taken
        # ("now")
        if start not in ("after_gravity", "now"):
            raise ValueError("start must be 'after_gravity' or 'now'")
        self.start = start
        self.sur_ms = []          # surrogate pipeline time on its stream, per hand-over
        if asynchronous:
            self.main_stream = torch.cuda.current_stream(p.x.device)
            self.sur_stream = surrogate.eng.stream
            if self.sur_stream is None or self.sur_stream.cuda_stream == self.main_stream.cuda_stream:
                raise ValueError("the asynchronous mode needs the surrogate engine on its own stream")
            dev = p.x.device
            ng = step.ng
            # two snapshot slots: the galaxy writes one while the worker may
            # still read the other
            self._slots = [dict({a: torch.empty(ng, dtype=torch.float64, device=dev)
                                 for a in _SNAP_F64},
                                **{a: torch.empty(p.n, dtype=torch.float64, device=dev)
                                   for a in ("px", "py", "pz")},
                                H=torch.empty(ng, dtype=torch.float32, device=dev),
                                id=torch.empty(ng, dtype=torch.int64, device=dev),
                                released=None, released_flag=threading.Event())
                           for _ in range(2)]
            for s in self._slots:
                s["released_flag"].set()
            self._next_slot = 0
            # start gates: an event after each later gravity call; the work of
            # a hand-over waits for the next one, so that it overlaps the
            # latency-bound SPH and tree phases instead of the compute-bound
            # gravity kernel
            self._gates = []
            self._gate_cv = threading.Condition()
            step.after_gravity.append(self._publish_gate)
            self._jobs = _queue.Queue()
            self._worker = threading.Thread(target=self._work, name="sn-surrogate", daemon=True)
            self._worker.start()

    # ---- sites ----------------------------------------------------------------
    def sites(self, step_index: int, pos=None):
        """This step's SN sites: candidate stars in a seeded random order,
        each kept unless its box would overlap the box of a site already kept
        (so every gas particle belongs to at most one region), until K.
        `pos` = (x, y, z) of all particles (default: the galaxy's own
        arrays; the asynchronous hand-over passes its snapshot of them)."""
        rng = np.random.default_rng(self.seed + step_index)
        torch = self.torch
        x, y, z = (self.step.p.x, self.step.p.y, self.step.p.z) if pos is None else pos
        side = self.side / PC_PER_KPC
        kept = np.zeros((0, 3))
        chosen, seen = [], set()
        want = min(self.K, self.cand.size)
        for _ in range(64):  # draws of 4K distinct candidates until K are kept
            draw = rng.choice(self.cand, size=min(4 * self.K, self.cand.size), replace=False)
            idx = torch.as_tensor(draw, device=x.device)
            at = torch.stack([x[idx], y[idx], z[idx]], dim=1).cpu().numpy()
            kept = keep_in_order(draw, at, side, kept, seen, chosen, want)
            if len(chosen) == want:
                break
        s = torch.as_tensor(np.sort(np.asarray(chosen, np.int64)), device=x.device)
        return torch.stack([x[s], y[s], z[s]], dim=1).contiguous()

    def _valid(self, pred, K):
        """Per-region check (gx_sn_check) that every predicted channel stays
        within valid_sigma standard deviations of the training targets."""
        lo, hi = self.sur.check_bounds(self.valid_sigma)
        return self.eng.sn_check(pred, K, self.sur.grid, lo, hi)

    # ---- the surrogate pipeline ----------------------------------------------------
    def _pipeline(self, snap, centers, step_index, item, on_gathered=None):
        """Regions of one hand-over from the gas state `snap` (dict of device
        arrays x .. u, H, id over the gas), on the surrogate engine's stream;
        fills item.ids / item.new.  on_gathered() is called once the snapshot
        has been read for the last time (after the gather)."""
        torch, eng, st = self.torch, self.eng, self.step
        dev = centers.device
        K = int(centers.shape[0])
        gas = ParticleSet(x=snap["x"], y=snap["y"], z=snap["z"], vx=snap["vx"], vy=snap["vy"],
                          vz=snap["vz"], m=snap["m"])
        half_kpc = 0.5 * self.side / PC_PER_KPC
        off, idx, tot = eng.sn_extract(gas, centers, half_kpc, gas.n)
        f64 = dict(dtype=torch.float64, device=dev)
        delta = {"regions": K, "replaced_regions": 0, "fallback_regions": 0}
        if tot == 0:
            if on_gathered:
                on_gathered()
            item.ids = torch.zeros(0, dtype=torch.int64, device=dev)
            item.new = {a: torch.zeros(0, **f64) for a in ("x", "y", "z", "vx", "vy", "vz", "u")}
            return delta
        offh = off.cpu().numpy()
        n_max = int((offh[1:] - offh[:-1]).max())
        box = {a: torch.empty(tot, **f64) for a in ("x", "y", "z", "vx", "vy", "vz", "m", "u")}
        box["H"] = torch.empty(tot, dtype=torch.float32, device=dev)
        lat = self.lattice[:K].contiguous()
        eng.sn_gather(gas, snap["u"], snap["H"], off, idx, n_max, centers, lat, PC_PER_KPC, box)
        ids = snap["id"].index_select(0, idx.long())
        if on_gathered:
            on_gathered()
        q = ParticleSet(x=box["x"], y=box["y"], z=box["z"], vx=box["vx"], vy=box["vy"],
                        vz=box["vz"], m=box["m"],
                        eps2=torch.zeros(tot, dtype=torch.float32, device=dev))
        ident = torch.arange(tot, dtype=torch.int32, device=dev)
        amb = eng.sn_ambient(q, box["u"], off, ident, self.side, 1.0 / U_PER_K)
        g = GasState.zeros(tot, u=box["u"], device=dev)
        g.H.copy_(box["H"])
        eng.tree_build(q, GX_TREE_GAS, self.cfg.n_leaf, self.cfg.n_group)
        xin = self.sur.inputs(q, g, lat, self.side, amb, K)
        pred = torch.empty(K * self.sur.V * 5, dtype=torch.float32, device=dev)
        self.sur.infer(xin, K, pred)
        ok = self._valid(pred, K)
        new = {a: torch.empty(tot, **f64) for a in ("x", "y", "z", "vx", "vy", "vz", "u")}
        gen = torch.Generator(device=dev)
        gen.manual_seed(1_000_003 * self.seed + step_index)
        uni = torch.rand(tot * self.sur.n_uniforms, dtype=torch.float32, device=dev,
                         generator=gen)
        self.sur.resample(pred, lat, self.side, off, n_max, uni, (box["x"], box["y"], box["z"]),
                          new)
        delay_time = self.delay * st.cfg.dt
        eng.sn_unframe(off, n_max, lat, centers, amb, delay_time, PC_PER_KPC,
                       new["x"], new["y"], new["z"])
        if not ok.all():
            # fallback: drop the regions the network cannot be trusted on
            keep = np.concatenate([np.arange(offh[c], offh[c + 1]) for c in range(K) if ok[c]]
                                  or [np.zeros(0, np.int64)])
            kt = torch.as_tensor(keep, dtype=torch.long, device=dev)
            ids = ids.index_select(0, kt)
            new = {a: v.index_select(0, kt) for a, v in new.items()}
        item.ids, item.new = ids.contiguous(), new
        delta["fallback_regions"] = int((~ok).sum())
        delta["replaced_regions"] = int(ok.sum())
        return delta

    def _count(self, delta):
        with self._lock:
            for k, v in delta.items():
                self.stats[k] += v

    # ---- hand-over and replacement ------------------------------------------
    def launch(self, step_index: int):
        """Hand this step's regions to the surrogate; queue their replacement."""
        st = self.step
        item = Pending(step_index + self.delay)
        if not self.asynchronous:
            centers = self.sites(step_index)
            snap = {a: getattr(st.gas, a) for a in ("x", "y", "z", "vx", "vy", "vz", "m")}
            snap.update(u=st.g.u, H=st.g.H, id=st.p.id[st.gas_offset:])
            self._count(self._pipeline(snap, centers, step_index, item))
            item.ready.set()
        else:
            torch = self.torch
            slot = self._slots[self._next_slot]
            self._next_slot ^= 1
            # the worker must be done reading this slot (two hand-overs ago)
            slot["released_flag"].wait()
            if slot["released"] is not None:
                self.main_stream.wait_event(slot["released"])
            for a in ("x", "y", "z", "vx", "vy", "vz", "m"):
                slot[a].copy_(getattr(st.gas, a))
            slot["u"].copy_(st.g.u)
            slot["H"].copy_(st.g.H)
            slot["id"].copy_(st.p.id[st.gas_offset:])
            # the sites are chosen by the worker from this copy of the
            # positions, so the galaxy's thread neither reads back nor waits
            for a, b in (("px", st.p.x), ("py", st.p.y), ("pz", st.p.z)):
                slot[a].copy_(b)
            taken = torch.cuda.Event()
            taken.record(self.main_stream)
            slot["released_flag"].clear()
            with self._gate_cv:
                need = len(self._gates) + 1
            self._jobs.put((slot, taken, need, step_index, item))
        self.queue.append(item)

    def _publish_gate(self):
        ev = self.torch.cuda.Event()
        ev.record(self.main_stream)
        with self._gate_cv:
            self._gates.append(ev)
            self._gate_cv.notify_all()

    def _gate(self, need):
        with self._gate_cv:
            while len(self._gates) < need:
                self._gate_cv.wait()
            return self._gates[need - 1]

    def _work(self):
        torch = self.torch
        while True:
            job = self._jobs.get()
            if job is None:
                return
            slot, taken, need, step_index, item = job
            try:
                with torch.cuda.stream(self.sur_stream):
                    self.sur_stream.wait_event(taken)
                    centers = self.sites(step_index, (slot["px"], slot["py"], slot["pz"]))
                    gate = self._gate(need) if self.start == "after_gravity" else None
                    if gate is not None:
                        self.sur_stream.wait_event(gate)
                    t0 = torch.cuda.Event(enable_timing=True)
                    t0.record(self.sur_stream)

                    def gathered():
                        ev = torch.cuda.Event()
                        ev.record(self.sur_stream)
                        slot["released"] = ev
                        slot["released_flag"].set()

                    delta = self._pipeline(slot, centers, step_index, item, on_gathered=gathered)
                    t1 = torch.cuda.Event(enable_timing=True)
                    t1.record(self.sur_stream)
                    item.done = t1
                    t1.synchronize()
                    self.sur_ms.append(t0.elapsed_time(t1))
                    self._count(delta)
            except BaseException as e:  # handed to the main thread at apply time
                item.error = e
                slot["released"] = None
                slot["released_flag"].set()
            item.ready.set()

    def apply_due(self, step_index: int):
        """Write every queued result that is due at this step (on the galaxy's
        stream, with the galaxy's engine)."""
        st = self.step
        while self.queue and self.queue[0].due <= step_index:
            item = self.queue.popleft()
            item.ready.wait()
            if item.error is not None:
                raise RuntimeError("surrogate hand-over failed") from item.error
            if self.asynchronous and item.done is not None:
                self.main_stream.wait_event(item.done)
                for t in [item.ids, *item.new.values()]:
                    t.record_stream(self.main_stream)
            m = int(item.ids.shape[0])
            if m == 0:
                continue
            n = item.new
            miss = st.eng.sn_replace(st.p.id, st.p.n, st.p.x, st.p.y, st.p.z, st.p.vx, st.p.vy,
                                     st.p.vz, st.g.u, st.gas_offset, st.g.H64, item.ids,
                                     n["x"], n["y"], n["z"], n["vx"], n["vy"], n["vz"], n["u"])
            with self._lock:
                self.stats["particles_replaced"] += m - miss
                self.stats["missing_ids"] += miss

    def drain(self):
        """Wait until every hand-over made so far has its result (opening the
        start gate now for work still waiting for the next gravity call)."""
        if self.asynchronous:
            self._publish_gate()
        for item in list(self.queue):
            item.ready.wait()

    def close(self):
        if self.asynchronous and self._worker.is_alive():
            self._publish_gate()
            self._jobs.put(None)
            self._worker.join()
            self.step.after_gravity.remove(self._publish_gate)
