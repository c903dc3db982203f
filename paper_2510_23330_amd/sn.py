"""Supernova regions: plain small-timestep SPH of many independent cubes (the
surrogate's training-data generator, fallback and error reference) and the surrogate
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
        self.noconv = 0          # kernel-size solves that hit the iteration cap
        self.u_floor = cfg.t_floor * U_PER_K
        # ambient state of each cube before the explosion (mean density, mass-
        # weighted temperature and bulk velocity of its gas): the value of
        # voxels no particle kernel reaches, at every later voxelization too
        off, idx, _ = eng.sn_extract(self.p, self.centers, SIDE / 2, self.n)
        self._amb = eng.sn_ambient(self.p, self.g.u, off, idx, SIDE, 1.0 / U_PER_K)

    def ambient(self):
        """Per-cube ambient (log10 rho, log10 T, vx, vy, vz), device float [K * 5]."""
        return self._amb

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
        d = self.eng.sph_density(view, self.g, c.n_ngb, c.gamma, c.h_tol, c.max_iter, u=u,
                                 allow_noconv=True)
        self.noconv += int(d.get("n_noconv", 0))
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
            self._guard()
            if log and self.steps % 50 == 0:
                log(f"[sn] step {self.steps} t = {self.t / MYR * 1e3:.2f} kyr dt = {dt / MYR * 1e6:.1f} yr")
        return self.steps

    # fields carried by the working set of run_cubes
    _P_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "eps2")
    _G_FIELDS = ("u", "dudt", "H64", "H", "rho", "P", "cs", "vsig")

    def run_cubes(self, t_end: float, max_steps: int = 100000, log=None):
        """KDK to t_end in which every cube takes its own Courant step: the
        step of cube c is c_cfl min over its particles of H / v_sig
        (gx_sph_timestep per cube), applied by gx_kick_drift_cubes, so a cube
        is not held to the smallest step of the batch.  Cubes are independent
        (no forces between them), so they share the force evaluations of one
        working set; a cube that reaches t_end leaves it, its final state
        written back to the batch's arrays.  Returns the per-cube step counts
        (numpy int [K])."""
        torch = self.torch
        dev = self.p.x.device
        K = self.K
        off = np.asarray(self.off, np.int64)
        t_c = np.zeros(K)
        steps = np.zeros(K, np.int64)
        if self.steps == 0:
            self._forces(predicted=False)
        full_p, full_g = self.p, self.g
        full_a = (self.ax, self.ay, self.az)
        active = np.arange(K)
        keep = None           # particle indices of the working set in the full arrays
        cid = torch.as_tensor(np.asarray(self.b["cube_id"], np.int32), device=dev)
        dt_dev = torch.zeros(K, dtype=torch.float64, device=dev)
        it = 0
        while active.size and it < max_steps:
            ka = active.size
            self.eng.sph_timestep(self.g, self.cfg.c_cfl, dt_dev[:ka], cube_id=cid, n_cubes=ka)
            dt = np.minimum(dt_dev[:ka].cpu().numpy(), t_end - t_c[active])
            dt_dev[:ka].copy_(torch.as_tensor(dt, device=dev))
            self.eng.kick_drift_cubes(self.p, cid, dt_dev[:ka], 0.5, 1.0, self.ax, self.ay, self.az,
                                      u=self.g.u, dudt=self.g.dudt, u_floor=self.u_floor,
                                      vpred=self.vpred, upred=self.upred)
            self._forces(predicted=True)
            self.eng.kick_drift_cubes(self.p, cid, dt_dev[:ka], 0.5, 0.0, self.ax, self.ay, self.az,
                                      u=self.g.u, dudt=self.g.dudt, u_floor=self.u_floor)
            t_c[active] += dt
            steps[active] += 1
            it += 1
            self._guard()
            done = t_c[active] >= t_end * (1 - 1e-12)
            if done.any():
                # write the working set back, then keep the unfinished cubes only
                if keep is not None:
                    for f in self._P_FIELDS:
                        getattr(full_p, f).index_copy_(0, keep, getattr(self.p, f))
                    for f in self._G_FIELDS:
                        getattr(full_g, f).index_copy_(0, keep, getattr(self.g, f))
                    for a, b in zip(full_a, (self.ax, self.ay, self.az)):
                        a.index_copy_(0, keep, b)
                active = active[~done]
                if active.size == 0:
                    break
                idx = np.concatenate([np.arange(off[c], off[c + 1]) for c in active])
                keep = torch.as_tensor(idx, device=dev)
                self.p = ParticleSet(**{f: getattr(full_p, f).index_select(0, keep)
                                        for f in self._P_FIELDS})
                self.g = GasState(**{f: getattr(full_g, f).index_select(0, keep)
                                     for f in self._G_FIELDS})
                self.ax, self.ay, self.az = (a.index_select(0, keep) for a in full_a)
                n = int(idx.size)
                self.n = n
                self.vpred = torch.zeros(3 * n, dtype=torch.float64, device=dev)
                self.upred = torch.zeros(n, dtype=torch.float64, device=dev)
                counts = off[active + 1] - off[active]
                cid = torch.as_tensor(np.repeat(np.arange(active.size, dtype=np.int32), counts),
                                      device=dev)
            if log and it % 50 == 0:
                log(f"[sn] iteration {it}: {active.size} cubes left")
        self.p, self.g = full_p, full_g
        self.ax, self.ay, self.az = full_a
        self.n = full_p.n
        self.vpred = torch.zeros(3 * self.n, dtype=torch.float64, device=dev)
        self.upred = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self.t = t_end
        self.steps += int(steps.max()) if K else 0
        return steps

    def _guard(self, x_max: float = 1e7, u_max: float = 1e12):
        """Stop a run whose state left the representable range (a forced
        timestep far above the Courant limit can do that) before the next tree
        build or kernel-size solve sees it."""
        torch = self.torch
        p = self.p
        m = torch.stack([p.x.abs().max(), p.y.abs().max(), p.z.abs().max(), self.g.u.max()])
        m = m.cpu().numpy()
        if not (np.all(np.isfinite(m)) and m[:3].max() < x_max and m[3] < u_max):
            raise FloatingPointError(f"SPH state diverged at step {self.steps} "
                                     f"(max |x| {m[:3].max():.3g}, max u {m[3]:.3g})")

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


def generate(eng: Engine, seeds, t_end_myr: float = 0.1, log=None, cfg: SPHConfig = SPHConfig(),
             dt_fixed_myr: float = None, keep=False, grid: int = GRID, per_cube: bool = False):
    """One batch of training pairs: voxel grids just before the explosion and
    t_end after it, from plain small-dt SPH (or fixed steps of dt_fixed_myr).
    Returns (x, y, info) with x, y device float [K * 64^3 * 5] physical
    channels; info["batch"] is the SNBatch at t = 0 voxelization state when
    keep is set (its particles then hold the final state)."""
    import ics
    b = ics.sn_batch(seeds)
    sb = SNBatch(eng, b, cfg)
    x = sb.voxelize(grid=grid)
    sb.torch.cuda.synchronize()
    t0 = time.perf_counter()
    sb.inject()
    cube_steps = None
    if per_cube and dt_fixed_myr is None:
        cube_steps = sb.run_cubes(t_end_myr * MYR, log=log)
        steps = int(cube_steps.max())
    else:
        steps = sb.run(t_end_myr * MYR, log=log,
                       dt_fixed=None if dt_fixed_myr is None else dt_fixed_myr * MYR)
    sb.torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    y = sb.voxelize(grid=grid)
    info = {"steps": steps, "seconds": wall, "n_particles": sb.n, "K": sb.K, "noconv": sb.noconv,
            "n_cm3": b["n_cm3"].tolist(), "T": b["T_amb"].tolist()}
    if cube_steps is not None:
        info["cube_steps"] = cube_steps.tolist()
    if keep:
        info["batch"] = sb
    return x, y, info


ENCODINGS = ("5ch", "8cube")
RESAMPLERS = ("cdf", "gibbs")
V0_KMS = 1.0                 # offset inside the eight-cube velocity logarithms


class Surrogate:
    """The learned replacement of a supernova region's plain SPH (Sec. 3.3):
    U-Net weights plus the channel statistics that standardise its inputs and
    targets.  Inputs are the voxelized state just before the explosion,
    outputs the state 0.1 Myr after it.

    encoding "5ch": the network sees and predicts the five physical channels
    (log10 rho, log10 T, vx, vy, vz); "8cube": the paper's eight cubes (log10
    rho, log10 T, and per velocity component a positive and a negative cube
    of log10(v0 + |v|)), decoded back to the five physical channels after the
    network.  resampler "cdf": exact inverse-CDF draws of the voxels; "gibbs":
    Gibbs chains of `sweeps` sweeps started at the entering particles' voxels."""

    def __init__(self, eng: Engine, batch: int = 4, base: int = 32, levels: int = 4,
                 grid: int = GRID, seed: int = 0, device="cuda", train: bool = True,
                 encoding: str = "5ch", resampler: str = "cdf", sweeps: int = 4):
        import torch
        from .unet import UNet
        if encoding not in ENCODINGS or resampler not in RESAMPLERS:
            raise ValueError(f"encoding in {ENCODINGS}, resampler in {RESAMPLERS}")
        self.torch, self.eng, self.grid, self.device = torch, eng, grid, device
        self.encoding, self.resampler, self.sweeps = encoding, resampler, int(sweeps)
        self.nc = 5 if encoding == "5ch" else 8
        self.net = UNet(eng, S=grid, batch=batch, base=base, levels=levels, seed=seed, device=device,
                        train=train, nc_in=self.nc, nc_out=self.nc)
        self._alloc_stats()
        self.V = grid ** 3

    STATS = ("mean_in", "std_in", "scale_in", "shift_in", "mean_out", "std_out", "scale_out",
             "shift_out", "mean_phys", "std_phys")

    def _alloc_stats(self):
        torch = self.torch
        f = dict(dtype=torch.float32, device=self.device)
        nc = self.nc
        # channel mean and standard deviation of the network's training inputs
        # and targets (in its encoding), the standardising maps x -> x * scale
        # + shift, and the physical targets' mean and deviation (trust check)
        self.mean_in, self.std_in = torch.zeros(nc, **f), torch.ones(nc, **f)
        self.mean_out, self.std_out = torch.zeros(nc, **f), torch.ones(nc, **f)
        self.scale_in, self.shift_in = torch.ones(nc, **f), torch.zeros(nc, **f)
        self.scale_out, self.shift_out = torch.ones(nc, **f), torch.zeros(nc, **f)
        self.mean_phys, self.std_phys = torch.zeros(5, **f), torch.ones(5, **f)

    @property
    def n_uniforms(self):
        """Uniform numbers the resampler takes per particle."""
        return 4 if self.resampler == "cdf" else 3 * self.sweeps + 3

    # ---- statistics -----------------------------------------------------------
    def encode(self, x_phys, V, out):
        """Physical rows [V, 5] -> the network's channels [V, nc] (unstandardized)."""
        if self.nc == 5:
            out.copy_(x_phys[:V * 5])
        else:
            self.eng.sn_encode8(x_phys, V, V0_KMS, out)
        return out

    def channel_sums(self, X, sums, chunk: int = 64):
        """Add FP64 channel sums of the network's encoding of physical rows
        X (device float [n, V * 5]) into sums (device double [2 nc])."""
        torch, V = self.torch, self.V
        if self.nc == 5:
            self.eng.chan_stats(X.reshape(-1), 5, 5, sums)
            return sums
        tmp = torch.empty(min(chunk, X.shape[0]) * V * self.nc, dtype=torch.float32,
                          device=X.device)
        for a in range(0, X.shape[0], chunk):
            b = min(chunk, X.shape[0] - a)
            enc = self.encode(X[a:a + b].reshape(-1), b * V, tmp[:b * V * self.nc])
            self.eng.chan_stats(enc, self.nc, self.nc, sums)
        return sums

    def set_stats(self, sums_in, sums_out, count, sums_phys=None, min_std: float = 1e-3):
        """Channel moments from FP64 sums (gx_chan_stats over count rows) of
        the encoded inputs and targets and of the physical targets (the same
        as the targets' for the five-channel encoding)."""
        nc = self.nc
        self.eng.chan_moments(sums_in, nc, count, min_std, self.mean_in, self.std_in,
                              self.scale_in, self.shift_in)
        self.eng.chan_moments(sums_out, nc, count, min_std, self.mean_out, self.std_out,
                              self.scale_out, self.shift_out)
        if sums_phys is None:
            if nc != 5:
                raise ValueError("the eight-cube encoding needs the physical target sums")
            self.mean_phys.copy_(self.mean_out)
            self.std_phys.copy_(self.std_out)
        else:
            sc = self.torch.empty(5, dtype=self.torch.float32, device=self.device)
            sh = self.torch.empty_like(sc)
            self.eng.chan_moments(sums_phys, 5, count, min_std, self.mean_phys, self.std_phys,
                                  sc, sh)

    def standardize(self, x_f32, which="in", out_f32=None, out_bf16=None):
        """Physical [.., 5] rows -> the network's standardized channels:
        out_f32 rows of nc floats, out_bf16 rows of 8 (channels nc.. zero)."""
        scale, shift = (self.scale_in, self.shift_in) if which == "in" else \
            (self.scale_out, self.shift_out)
        nc = self.nc
        V = x_f32.numel() // 5
        src = x_f32
        if nc != 5:
            src = self.encode(x_f32, V, self.torch.empty(V * nc, dtype=self.torch.float32,
                                                         device=x_f32.device))
        self.eng.chan_affine(src, nc, nc, scale, shift, out=out_f32, out_stride=nc,
                             out_bf16=out_bf16, bf_stride=8)

    def check_bounds(self, sigma: float):
        """Per physical channel [lo, hi] = mean +- sigma std of the training
        targets (host FP64), for gx_sn_check."""
        mo = self.mean_phys.cpu().numpy().astype(np.float64)
        so = self.std_phys.cpu().numpy().astype(np.float64)
        return mo - sigma * so, mo + sigma * so

    # ---- inference ------------------------------------------------------------
    def inputs(self, p: ParticleSet, g: GasState, centers, side, amb, K):
        """Standardized network input bf16 [K * V * 8] of K regions (gas tree
        of p built by the caller)."""
        torch = self.torch
        dev = centers.device
        xin = torch.empty(K * self.V * 8, dtype=torch.bfloat16, device=dev)
        if self.nc == 5:
            self.eng.sn_voxelize(p, g.u, g.H, centers, side, self.grid, 1.0 / U_PER_K, amb,
                                 mean=self.mean_in, std=self.std_in, out_bf16=xin, cpad=8)
        else:
            phys = torch.empty(K * self.V * 5, dtype=torch.float32, device=dev)
            self.eng.sn_voxelize(p, g.u, g.H, centers, side, self.grid, 1.0 / U_PER_K, amb,
                                 out_f32=phys)
            self.standardize(phys, "in", out_bf16=xin)
        return xin

    def infer(self, x_bf16, K: int, out_f32):
        """x_bf16 [K * V * 8] standardized inputs -> out_f32 [K * V * 5] physical."""
        net, V, B, nc = self.net, self.V, self.net.B, self.nc
        tmp = None if nc == 5 else self.torch.empty(min(B, K) * V * nc, dtype=self.torch.float32,
                                                    device=out_f32.device)
        for a in range(0, K, B):
            b = min(B, K - a)
            net.Bcur = b
            dst = out_f32[a * V * 5:(a + b) * V * 5] if nc == 5 else tmp[:b * V * nc]
            net.forward(x_bf16[a * V * 8:(a + b) * V * 8], out_phys=dst,
                        scale=self.std_out, shift=self.mean_out)
            if nc != 5:
                self.eng.sn_decode8(dst, b * V, out_f32[a * V * 5:(a + b) * V * 5])
        net.Bcur = B
        return out_f32

    def resample(self, pred, centers, side, off, n_max, uniforms, start, out):
        """Particles drawn from the predicted grids (CSR off by region): the
        chosen resampler; start = (x, y, z) device FP64 positions of the
        particles that entered (frame of centers; used by the Gibbs chains)."""
        o = [out[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u")]
        if self.resampler == "cdf":
            self.eng.sn_resample(pred, centers, self.grid, side, off, n_max, uniforms, U_PER_K, *o)
        else:
            self.eng.sn_resample_gibbs(pred, centers, self.grid, side, off, n_max, *start,
                                       self.sweeps, uniforms, U_PER_K, *o)

    def regions(self, p: ParticleSet, g: GasState, centers, side: float = SIDE, cap: int = None,
                cfg: SPHConfig = SPHConfig(), uniforms=None, build_tree=True):
        """Extract -> voxelize -> infer -> resample for K regions (Sec. 3.2
        steps 2-4).  Returns (offsets, idx, new) with new = dict of device FP64
        arrays x, y, z, vx, vy, vz, u of the replacement particles (CSR by
        region, same count as the members idx it replaces)."""
        torch, eng = self.torch, self.eng
        K = int(centers.shape[0])
        dev = centers.device
        off, idx, tot = eng.sn_extract(p, centers, side / 2, cap or p.n)
        amb = eng.sn_ambient(p, g.u, off, idx, side, 1.0 / U_PER_K)
        if build_tree:
            eng.tree_build(p, GX_TREE_GAS, cfg.n_leaf, cfg.n_group)
        xin = self.inputs(p, g, centers, side, amb, K)
        pred = torch.empty(K * self.V * 5, dtype=torch.float32, device=dev)
        self.infer(xin, K, pred)
        new = {k: torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
               for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
        if tot > 0:
            n_max = int((off[1:] - off[:-1]).max().item())
            if uniforms is None:
                uniforms = torch.rand(tot * self.n_uniforms, dtype=torch.float32, device=dev)
            li = idx.long()
            start = tuple(a.index_select(0, li).contiguous() for a in (p.x, p.y, p.z))
            self.resample(pred, centers, side, off, n_max, uniforms, start, new)
        return off, idx, {k: v[:tot] for k, v in new.items()}, pred

    # ---- persistence ----------------------------------------------------------
    def save(self, path, moments: bool = False):
        """Weights (FP32 master copy), channel statistics and encoding; Adam
        moments only when asked (they triple the file)."""
        d = self.net.state_dict()
        extra = {"m": d["m"], "v": d["v"]} if moments else {}
        np.savez(path, w32=d["w32"], t=d["t"], encoding=np.str_(self.encoding), **extra,
                 **{k: getattr(self, k).cpu().numpy() for k in self.STATS})

    def export(self, path):
        """Inference weights: BF16 bits of every parameter (what the network
        computes with) plus the FP32 biases, the channel statistics and the
        encoding."""
        w = self.net.w32.cpu().numpy()
        b0 = min(ly.b_off for ly in self.net.L)
        bits = self.net.wbf.view(self.torch.int16).cpu().numpy().view(np.uint16)
        np.savez_compressed(path, w_bf16=bits, bias_f32=w[b0:], b_off=np.int64(b0),
                            levels=np.int64(self.net.levels), base=np.int64(self.net.base),
                            encoding=np.str_(self.encoding),
                            **{k: getattr(self, k).cpu().numpy() for k in self.STATS})

    @staticmethod
    def file_encoding(path):
        d = np.load(path)
        return str(d["encoding"]) if "encoding" in d else "5ch"

    def load(self, path):
        d = np.load(path)
        enc = str(d["encoding"]) if "encoding" in d else "5ch"
        if enc != self.encoding:
            raise ValueError(f"{path}: encoding {enc}, this surrogate uses {self.encoding}")
        if "w_bf16" in d:  # an exported inference file
            if int(d["levels"]) != self.net.levels or int(d["base"]) != self.net.base:
                raise ValueError(f"{path}: network shape differs")
            w = (d["w_bf16"].astype(np.uint32) << 16).view(np.float32).copy()
            w[int(d["b_off"]):] = d["bias_f32"]
            d = dict(d, w32=w)
        z = np.zeros_like(d["w32"])
        self.net.load_state_dict({"w32": d["w32"], "m": d["m"] if "m" in d else z,
                                  "v": d["v"] if "v" in d else z,
                                  "t": int(d["t"]) if "m" in d else 0})
        for k in self.STATS:
            if k in d:
                getattr(self, k).copy_(self.torch.as_tensor(d[k]))
            elif k in ("mean_phys", "std_phys") and self.nc == 5:
                # files written before the physical statistics were kept
                getattr(self, k).copy_(self.torch.as_tensor(d[k.replace("phys", "out")]))
            else:
                raise ValueError(f"{path}: no {k}")
