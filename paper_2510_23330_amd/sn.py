"""Supernova regions: plain small-timestep SPH of many independent cubes (the
surrogate's training-data generator, fallback and judge) and the surrogate
pipeline that replaces it (voxelize -> U-Net -> resample), Secs. 3.2-3.3.

Units: pc, km/s, Msun (time unit 0.97779 Myr).  Cubes are placed far apart
in one particle set so a single gas tree serves all of them; every
arithmetic step runs in libgx.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import GX_TREE_GAS, Engine, GasState, ParticleSet

MYR = 1.0 / 0.97779          # 1 Myr in pc/(km/s)
U_PER_K = 1.0 / 48.46
E_SN = 5.028e7               # 1e51 erg in Msun (km/s)^2
SIDE = 60.0
GRID = 64


@dataclass
class SPHConfig:
    n_ngb: float = 64.0
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    c_cfl: float = 0.3
    h_tol: float = 1e-3
    max_iter: int = 64
    n_leaf: int = 8
    n_group: int = 64
    t_floor: float = 10.0


class SNBatch:
    """K cubes in one gas set (dict from ics.sn_batch) on the device."""

    def __init__(self, eng: Engine, b: dict, cfg: SPHConfig = SPHConfig(), device="cuda"):
        import torch
        self.torch = torch
        self.eng, self.cfg, self.b = eng, cfg, b
        self.p = ParticleSet.from_numpy(b, device=device)
        self.n = self.p.n
        self.g = GasState.zeros(self.n, u=b["u"], device=device)
        self.centers = torch.as_tensor(b["centres"], dtype=torch.float64, device=device)
        self.off = b["offsets"]
        self.K = len(self.off) - 1
        z = lambda: torch.zeros(self.n, dtype=torch.float64, device=device)
        self.ax, self.ay, self.az = z(), z(), z()
        self.vpred = torch.zeros(3 * self.n, dtype=torch.float64, device=device)
        self.upred = z()
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.t = 0.0
        self.steps = 0
        self.u_floor = cfg.t_floor * U_PER_K

    def ambient(self):
        """Per-cube ambient (log10 rho, log10 T, 0, 0, 0) for empty voxels."""
        K = self.K
        counts = np.diff(self.off)
        rho = counts * self.b["m"][self.off[:-1]] / SIDE ** 3
        amb = np.zeros((K, 5), np.float32)
        amb[:, 0] = np.log10(rho)
        amb[:, 1] = np.log10(self.b["T_amb"])
        return self.torch.as_tensor(amb, device=self.p.x.device)

    def inject(self, k_inj: int = 32, energy: float = E_SN):
        """1e51 erg of thermal energy into the k_inj particles nearest each centre."""
        off, idx, tot = self.eng.sn_extract(self.p, self.centers, SIDE / 2, self.n)
        self.eng.sn_inject(self.p, off, idx, self.centers, k_inj, energy, self.g.u)

    def _forces(self, predicted):
        c = self.cfg
        self.eng.tree_build(self.p, GX_TREE_GAS, c.n_leaf, c.n_group)
        n = self.n
        for a in (self.ax, self.ay, self.az):
            a.zero_()
        if predicted:
            vel = (self.vpred[:n], self.vpred[n:2 * n], self.vpred[2 * n:])
            view = ParticleSet(x=self.p.x, y=self.p.y, z=self.p.z, vx=vel[0], vy=vel[1],
                               vz=vel[2], m=self.p.m, eps2=self.p.eps2)
            u = self.upred
        else:
            view, u = self.p, None
        self.eng.sph_density(view, self.g, c.n_ngb, c.gamma, c.h_tol, c.max_iter, u=u)
        self.eng.sph_forces(view, self.g, self.ax, self.ay, self.az, gamma=c.gamma, alpha=c.alpha,
                            u=u)

    def timestep(self):
        self.eng.sph_timestep(self.g, self.cfg.c_cfl, self.dt)
        return float(self.dt.item())

    def run(self, t_end: float, max_steps: int = 100000, dt_fixed: float = None, log=None):
        """Shared-timestep KDK to t_end (Courant dt unless dt_fixed).  Returns steps."""
        if self.steps == 0:
            self._forces(predicted=False)
        while self.t < t_end * (1 - 1e-12) and self.steps < max_steps:
            dt = dt_fixed if dt_fixed else self.timestep()
            dt = min(dt, t_end - self.t)
            self.eng.kick_drift(self.p, dt / 2, dt, self.ax, self.ay, self.az, u=self.g.u,
                                dudt=self.g.dudt, u_floor=self.u_floor, vpred=self.vpred,
                                upred=self.upred)
            self._forces(predicted=True)
            self.eng.kick_drift(self.p, dt / 2, 0.0, self.ax, self.ay, self.az, u=self.g.u,
                                dudt=self.g.dudt, u_floor=self.u_floor)
            self.t += dt
            self.steps += 1
            if log and self.steps % 50 == 0:
                log(f"[sn] step {self.steps} t = {self.t / MYR * 1e3:.2f} kyr dt = {dt / MYR * 1e6:.1f} yr")
        return self.steps

    def energy(self):
        """(kinetic, thermal) totals; no gravity inside cubes."""
        p, g = self.p, self.g
        K, _, U = self.eng.energy(p, self.ax * 0, p.m, g.u)
        return K, U

    def voxelize(self, out_f32=None, grid: int = GRID):
        """Physical voxel channels [K, grid^3, 5] of the current state."""
        torch = self.torch
        if out_f32 is None:
            out_f32 = torch.zeros(self.K * grid ** 3 * 5, dtype=torch.float32, device=self.p.x.device)
        self.eng.tree_build(self.p, GX_TREE_GAS, self.cfg.n_leaf, self.cfg.n_group)
        if not bool((self.g.H > 0).all()):
            self.eng.sph_density(self.p, self.g, self.cfg.n_ngb, self.cfg.gamma, self.cfg.h_tol,
                                 self.cfg.max_iter)
        self.eng.sn_voxelize(self.p, self.g.u, self.g.H, self.centers, SIDE, grid, 1.0 / U_PER_K,
                             self.ambient(), out_f32=out_f32)
        return out_f32


def generate(eng: Engine, seeds, t_end_myr: float = 0.1, log=None, cfg: SPHConfig = SPHConfig()):
    """One batch of training pairs: voxel grids just before the explosion and
    t_end after it, from plain small-dt SPH.  Returns (x, y, info) with x, y
    device float [K, 64^3, 5]."""
    import ics
    b = ics.sn_batch(seeds)
    sb = SNBatch(eng, b, cfg)
    x = sb.voxelize()
    sb.inject()
    t0 = time.perf_counter()
    steps = sb.run(t_end_myr * MYR, log=log)
    sb.torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    y = sb.voxelize()
    info = {"steps": steps, "seconds": wall, "n_particles": sb.n, "K": sb.K,
            "n_cm3": b["n_cm3"].tolist(), "T": b["T_amb"].tolist()}
    return x, y, info
