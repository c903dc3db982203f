"""Surrogate-coupled global step (Sec. 3.2): supernova regions of the galaxy
are handed to the learned surrogate and their gas is replaced, by particle
ID, after a delay of `delay` global steps (the paper's 0.1 Myr = 50 steps of
2,000 yr), so the global step never shrinks for the explosions.

Per call, for the K sites of this step (seeded uniform choice among disk
stars): extract the gas in the (60 pc)^3 box around each site, pack it into
the box's own frame in pc (`gx_sn_gather`), ambient state, gas tree and
voxelization in that frame, U-Net inference, resampling of as many particles
as entered, and transformation back to the galaxy frame drifted by the box's
bulk velocity over the delay (`gx_sn_unframe`).  The result waits in a queue
and is written over the particles with the same IDs (`gx_sn_replace`) when it
falls due.  A region whose prediction leaves the range the network was
trained on is not replaced: its gas stays with the plain integrator (the
fallback), and the count is reported.

The surrogate runs on its own library context (its own gas-tree slot) on the
same stream as the galaxy step; every arithmetic step runs in libgx.
"""
from __future__ import annotations

import math
from collections import deque
from dataclasses import dataclass

import numpy as np

from . import GX_TREE_GAS, Engine, GasState, ParticleSet
from .sn import U_PER_K, SPHConfig, Surrogate

PC_PER_KPC = 1000.0


@dataclass
class Pending:
    due: int
    ids: object        # device int64 [m] particle IDs to overwrite
    new: dict          # device FP64 arrays x, y, z, vx, vy, vz, u (galaxy frame)


class SNCoupling:
    def __init__(self, step, surrogate: Surrogate, n_sites: int = 64, delay: int = 50,
                 side_pc: float = 60.0, seed: int = 5, r_max: float = 15.0, z_max: float = 0.3,
                 valid_sigma: float = 8.0, cfg: SPHConfig = SPHConfig(), star_type: int = 1):
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

    def sites(self, step_index: int):
        """This step's SN sites: candidate stars in a seeded random order,
        each kept unless its box would overlap the box of a site already kept
        (so every gas particle belongs to at most one region), until K."""
        rng = np.random.default_rng(self.seed + step_index)
        torch, p = self.torch, self.step.p
        side = self.side / PC_PER_KPC
        kept = np.zeros((0, 3))
        chosen, seen = [], set()
        want = min(self.K, self.cand.size)
        for _ in range(64):  # draws of 4K distinct candidates until K are kept
            draw = rng.choice(self.cand, size=min(4 * self.K, self.cand.size), replace=False)
            idx = torch.as_tensor(draw, device=p.x.device)
            pos = torch.stack([p.x[idx], p.y[idx], p.z[idx]], dim=1).cpu().numpy()
            for j in range(pos.shape[0]):
                if draw[j] in seen:
                    continue
                seen.add(int(draw[j]))
                if kept.shape[0] and np.any(np.all(np.abs(kept - pos[j]) < side, axis=1)):
                    continue
                kept = np.vstack([kept, pos[j]])
                chosen.append(draw[j])
                if len(chosen) == want:
                    break
            if len(chosen) == want:
                break
        s = torch.as_tensor(np.sort(np.asarray(chosen, np.int64)), device=p.x.device)
        return torch.stack([p.x[s], p.y[s], p.z[s]], dim=1).contiguous()

    def _valid(self, pred, K):
        """Per-region check (gx_sn_check) that every predicted channel stays
        within valid_sigma standard deviations of the training targets."""
        sur = self.sur
        mo = sur.mean_out.cpu().numpy().astype(np.float64)
        so = sur.std_out.cpu().numpy().astype(np.float64)
        return self.eng.sn_check(pred, K, sur.grid, mo - self.valid_sigma * so,
                                 mo + self.valid_sigma * so)

    def launch(self, step_index: int):
        """Hand this step's regions to the surrogate; queue their replacement."""
        torch, eng, st = self.torch, self.eng, self.step
        gas, dev = st.gas, st.p.x.device
        centers = self.sites(step_index)
        K = int(centers.shape[0])
        half_kpc = 0.5 * self.side / PC_PER_KPC
        off, idx, tot = eng.sn_extract(gas, centers, half_kpc, gas.n)
        self.stats["regions"] += K
        if tot == 0:
            return
        offh = off.cpu().numpy()
        n_max = int((offh[1:] - offh[:-1]).max())
        f64 = dict(dtype=torch.float64, device=dev)
        box = {a: torch.empty(tot, **f64) for a in ("x", "y", "z", "vx", "vy", "vz", "m", "u")}
        box["H"] = torch.empty(tot, dtype=torch.float32, device=dev)
        lat = self.lattice[:K].contiguous()
        eng.sn_gather(gas, st.g.u, st.g.H, off, idx, n_max, centers, lat, PC_PER_KPC, box)
        q = ParticleSet(x=box["x"], y=box["y"], z=box["z"], vx=box["vx"], vy=box["vy"],
                        vz=box["vz"], m=box["m"],
                        eps2=torch.zeros(tot, dtype=torch.float32, device=dev))
        ident = torch.arange(tot, dtype=torch.int32, device=dev)
        amb = eng.sn_ambient(q, box["u"], off, ident, self.side, 1.0 / U_PER_K)
        g = GasState.zeros(tot, u=box["u"], device=dev)
        g.H.copy_(box["H"])
        eng.tree_build(q, GX_TREE_GAS, self.cfg.n_leaf, self.cfg.n_group)
        xin = torch.empty(K * self.sur.V * 8, dtype=torch.bfloat16, device=dev)
        eng.sn_voxelize(q, g.u, g.H, lat, self.side, self.sur.grid, 1.0 / U_PER_K, amb,
                        mean=self.sur.mean_in, std=self.sur.std_in, out_bf16=xin, cpad=8)
        pred = torch.empty(K * self.sur.V * 5, dtype=torch.float32, device=dev)
        self.sur.infer(xin, K, pred)
        ok = self._valid(pred, K)
        new = {a: torch.empty(tot, **f64) for a in ("x", "y", "z", "vx", "vy", "vz", "u")}
        uni = torch.rand(tot * 4, dtype=torch.float32, device=dev)
        eng.sn_resample(pred, lat, self.sur.grid, self.side, off, n_max, uni, U_PER_K,
                        *(new[a] for a in ("x", "y", "z", "vx", "vy", "vz", "u")))
        delay_time = self.delay * st.cfg.dt
        eng.sn_unframe(off, n_max, lat, centers, amb, delay_time, PC_PER_KPC,
                       new["x"], new["y"], new["z"])
        ids = st.p.id[st.gas_offset:].index_select(0, idx.long())
        if not ok.all():
            # fallback: drop the regions the network cannot be trusted on
            keep = np.concatenate([np.arange(offh[c], offh[c + 1]) for c in range(K) if ok[c]]
                                  or [np.zeros(0, np.int64)])
            kt = torch.as_tensor(keep, dtype=torch.long, device=dev)
            ids = ids.index_select(0, kt)
            new = {a: v.index_select(0, kt) for a, v in new.items()}
        self.stats["fallback_regions"] += int((~ok).sum())
        self.stats["replaced_regions"] += int(ok.sum())
        self.queue.append(Pending(step_index + self.delay, ids.contiguous(), new))

    def apply_due(self, step_index: int):
        """Write every queued result that is due at this step."""
        st = self.step
        while self.queue and self.queue[0].due <= step_index:
            item = self.queue.popleft()
            m = int(item.ids.shape[0])
            if m == 0:
                continue
            n = item.new
            miss = self.eng.sn_replace(st.p.id, st.p.n, st.p.x, st.p.y, st.p.z, st.p.vx, st.p.vy,
                                       st.p.vz, st.g.u, st.gas_offset, st.g.H64, item.ids,
                                       n["x"], n["y"], n["z"], n["vx"], n["vy"], n["vz"], n["u"])
            self.stats["particles_replaced"] += m - miss
            self.stats["missing_ids"] += miss
