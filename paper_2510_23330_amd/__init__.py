"""paper_2510_23330_amd -- Python binding of libgx, the MI355X interaction
engine for the N-body/SPH galaxy integrator of arXiv 2510.23330.

Everything here is argument marshalling: PyTorch provides device memory and
the current HIP stream, and every step of the path runs in libgx's HIP
kernels.  Function names follow the C ABI in include/gx.h without the
``gx_`` prefix.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import (GX_DIRECT, GX_PREC_FP64, GX_QUAD, GX_TREE_ALL, GX_TREE_GAS, GxGas,
                   GxParticles, GxStats)

__all__ = ["Engine", "ParticleSet", "GasState", "GxError", "GX_QUAD", "GX_DIRECT",
           "GX_PREC_FP64", "GX_TREE_ALL", "GX_TREE_GAS"]


class GxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _ptr(t, dtype=None):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("libgx takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libgx takes contiguous tensors")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


@dataclass
class ParticleSet:
    """Device structure-of-arrays particle view (torch tensors)."""
    x: object
    y: object
    z: object
    vx: object
    vy: object
    vz: object
    m: object
    eps2: object = None
    id: object = None
    type: object = None

    @property
    def n(self):
        return int(self.x.shape[0])

    @classmethod
    def from_numpy(cls, d: dict, device="cuda", sl=slice(None)):
        torch = _torch()
        f64 = lambda k: torch.as_tensor(np.ascontiguousarray(d[k][sl], np.float64), device=device)
        eps2 = d.get("eps2")
        return cls(x=f64("x"), y=f64("y"), z=f64("z"), vx=f64("vx"), vy=f64("vy"), vz=f64("vz"),
                   m=f64("m"),
                   eps2=None if eps2 is None else torch.as_tensor(
                       np.ascontiguousarray(eps2[sl], np.float32), device=device),
                   id=None if "id" not in d else torch.as_tensor(
                       np.ascontiguousarray(d["id"][sl], np.int64), device=device),
                   type=None if "type" not in d else torch.as_tensor(
                       np.ascontiguousarray(d["type"][sl], np.uint8), device=device))

    def view(self, vel=None):
        """ctypes gx_particles; ``vel`` optionally replaces (vx, vy, vz)."""
        torch = _torch()
        vx, vy, vz = vel if vel is not None else (self.vx, self.vy, self.vz)
        s = GxParticles()
        s.x, s.y, s.z = _ptr(self.x, torch.float64), _ptr(self.y, torch.float64), _ptr(self.z, torch.float64)
        s.vx, s.vy, s.vz = _ptr(vx, torch.float64), _ptr(vy, torch.float64), _ptr(vz, torch.float64)
        s.m = _ptr(self.m, torch.float64)
        s.eps2 = _ptr(self.eps2, torch.float32)
        s.id = _ptr(self.id, torch.int64)
        s.type = _ptr(self.type, torch.uint8)
        s.n = self.n
        for t in (self.y, self.z, vx, vy, vz, self.m):
            if t.shape[0] != s.n:
                raise ValueError("particle arrays differ in length")
        return s


@dataclass
class GasState:
    """Device gas state (torch tensors), same order as the gas ParticleSet."""
    u: object
    dudt: object
    H64: object
    H: object
    rho: object
    P: object
    cs: object
    vsig: object

    @classmethod
    def zeros(cls, n, u=None, device="cuda"):
        torch = _torch()
        z64 = lambda: torch.zeros(n, dtype=torch.float64, device=device)
        z32 = lambda: torch.zeros(n, dtype=torch.float32, device=device)
        if u is None:
            uu = z64()
        elif isinstance(u, torch.Tensor):
            uu = u.to(device=device, dtype=torch.float64).contiguous()
        else:
            uu = torch.as_tensor(np.ascontiguousarray(u, np.float64), device=device)
        return cls(u=uu, dudt=z64(), H64=z64(), H=z32(), rho=z32(), P=z32(), cs=z32(), vsig=z32())

    def view(self, u=None):
        torch = _torch()
        g = GxGas()
        g.u = _ptr(self.u if u is None else u, torch.float64)
        g.dudt = _ptr(self.dudt, torch.float64)
        g.H64 = _ptr(self.H64, torch.float64)
        g.H, g.rho, g.P = (_ptr(t, torch.float32) for t in (self.H, self.rho, self.P))
        g.cs, g.vsig = _ptr(self.cs, torch.float32), _ptr(self.vsig, torch.float32)
        g.n = int(self.u.shape[0])
        return g


class Engine:
    """One libgx context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = _lib.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = C.c_void_p()
        self._check(self.lib.gx_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)), None)
        self.ctx = h

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.gx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ctx="self", allow=()):
        if rc != 0 and rc not in allow:
            c = self.ctx if ctx == "self" else None
            msg = self.lib.gx_last_error(c).decode() if c else ""
            raise GxError(rc, msg)
        return rc

    def set_walk_stack_limit(self, entries: int):
        """Test hook: limit the gravity walk's small stack (0 restores it)."""
        self._check(self.lib.gx_set_walk_stack_limit(self.ctx, int(entries)))

    @property
    def stream(self):
        """The torch stream this context enqueues on."""
        return self._stream

    def set_stream(self, stream):
        self._stream = stream
        self._check(self.lib.gx_set_stream(self.ctx, C.c_void_p(stream.cuda_stream)))

    # ---- hot path ----------------------------------------------------------
    def tree_build(self, p: ParticleSet, which=GX_TREE_ALL, n_leaf=16, n_group=256, perm_out=None,
                   vel=None):
        st = GxStats()
        v = p.view(vel)
        self._check(self.lib.gx_tree_build(self.ctx, C.byref(v), which, n_leaf, n_group,
                                           _ptr(perm_out), C.byref(st)))
        return st.as_dict()

    def gravity_forces(self, p: ParticleSet, G, theta, flags, ax, ay, az, pot, stats=True):
        st = GxStats()
        v = p.view()
        self._check(self.lib.gx_gravity_forces(self.ctx, C.byref(v), float(G), float(theta),
                                               int(flags), _ptr(ax), _ptr(ay), _ptr(az),
                                               _ptr(pot), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def sph_density(self, gas: ParticleSet, g: GasState, n_ngb=64.0, gamma=5.0 / 3.0, tol=1e-3,
                    max_iter=64, stats=True, allow_noconv=False, u=None):
        st = GxStats()
        v = gas.view()
        gv = g.view(u)
        rc = self._check(self.lib.gx_sph_density(self.ctx, C.byref(v), C.byref(gv), float(n_ngb),
                                                 float(gamma), float(tol), int(max_iter),
                                                 C.byref(st) if stats else None),
                         allow=(_lib.GX_ENOCONV,) if allow_noconv else ())
        d = st.as_dict() if stats else {}
        d["status"] = rc
        return d

    def sph_forces(self, gas: ParticleSet, g: GasState, ax, ay, az, gamma=5.0 / 3.0, alpha=1.0,
                   vel=None, u=None, stats=True):
        st = GxStats()
        v = gas.view(vel)
        gv = g.view(u)
        self._check(self.lib.gx_sph_forces(self.ctx, C.byref(v), C.byref(gv), float(gamma),
                                           float(alpha), _ptr(ax), _ptr(ay), _ptr(az),
                                           C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def kick_drift(self, p: ParticleSet, dt_kick, dt_drift, ax, ay, az, u=None, dudt=None,
                   u_floor=0.0, vpred=None, upred=None):
        n_u = 0 if u is None else int(u.shape[0])
        self._check(self.lib.gx_kick_drift(self.ctx, p.n, float(dt_kick), float(dt_drift),
                                           _ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx),
                                           _ptr(p.vy), _ptr(p.vz), _ptr(ax), _ptr(ay), _ptr(az),
                                           n_u, _ptr(u), _ptr(dudt), float(u_floor), _ptr(vpred),
                                           _ptr(upred)))

    def add_accel(self, ax, ay, az, bx, by, bz):
        """a += b, then b = 0 (device double [n] each)."""
        n = int(ax.shape[0])
        for t in (ay, az, bx, by, bz):
            if int(t.shape[0]) != n:
                raise ValueError("add_accel: arrays of different lengths")
        f64 = _torch().float64
        self._check(self.lib.gx_add_accel(self.ctx, n, *(_ptr(t, f64) for t in (ax, ay, az, bx, by,
                                                                               bz))))

    def kick_drift_cubes(self, p: ParticleSet, cube_id, dt_cube, f_kick, f_drift, ax, ay, az,
                         u=None, dudt=None, u_floor=0.0, vpred=None, upred=None):
        """Half step of independent cubes, each with its own dt (device double [K])."""
        torch = _torch()
        self._check(self.lib.gx_kick_drift_cubes(
            self.ctx, p.n, _ptr(cube_id, torch.int32), _ptr(dt_cube, torch.float64), float(f_kick),
            float(f_drift), _ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx), _ptr(p.vy), _ptr(p.vz),
            _ptr(ax), _ptr(ay), _ptr(az), _ptr(u), _ptr(dudt), float(u_floor), _ptr(vpred),
            _ptr(upred)))

    def energy(self, p: ParticleSet, pot, m_gas=None, u=None):
        out = (C.c_double * 3)()
        n_gas = 0 if u is None else int(u.shape[0])
        self._check(self.lib.gx_energy(self.ctx, C.byref(p.view()), _ptr(pot), n_gas,
                                       _ptr(m_gas), _ptr(u), out))
        return tuple(out)

    def sph_timestep(self, g: GasState, c_cfl, dt_out, cube_id=None, n_cubes=1):
        gv = g.view()
        self._check(self.lib.gx_sph_timestep(self.ctx, C.byref(gv), float(c_cfl), _ptr(cube_id),
                                             int(n_cubes), _ptr(dt_out)))

    # ---- inspection ----------------------------------------------------------
    def tree_counts(self, which=GX_TREE_ALL):
        nn, ng = C.c_int64(), C.c_int64()
        self._check(self.lib.gx_tree_counts(self.ctx, which, C.byref(nn), C.byref(ng)))
        return nn.value, ng.value

    def tree_export(self, which=GX_TREE_ALL, n=None):
        nn, ng = self.tree_counts(which)
        if n is None:
            raise ValueError("pass n (particle count)")
        o = dict(keys=np.zeros(n, np.uint64), perm=np.zeros(n, np.int32), box=np.zeros(4),
                 begin=np.zeros(nn, np.int32), end=np.zeros(nn, np.int32),
                 next=np.zeros(nn, np.int32), level=np.zeros(nn, np.int32),
                 leaf=np.zeros(nn, np.int8), mass=np.zeros(nn), com=np.zeros((nn, 3)),
                 quad=np.zeros((nn, 6), np.float32), eps2bar=np.zeros(nn, np.float32),
                 lo=np.zeros((nn, 3)), hi=np.zeros((nn, 3)), groups=np.zeros(ng, np.int32))
        pp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(self.lib.gx_tree_export(self.ctx, which, *(pp(o[k]) for k in (
            "keys", "perm", "box", "begin", "end", "next", "level", "leaf", "mass", "com", "quad",
            "eps2bar", "lo", "hi", "groups"))))
        return o

    def gravity_list_sizes(self):
        """(groups, pc entries, pp ranges) of the last gravity call's lists
        (host values kept by the context; no device access)."""
        ng, npc, npr = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.gx_gravity_list_sizes(self.ctx, C.byref(ng), C.byref(npc), C.byref(npr)))
        return ng.value, npc.value, npr.value

    def gravity_lists(self):
        ng, npc, npr = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.gx_gravity_list_sizes(self.ctx, C.byref(ng), C.byref(npc), C.byref(npr)))
        o = dict(pc_off=np.zeros(ng.value + 1, np.int64), pc=np.zeros(max(1, npc.value), np.int32),
                 pp_off=np.zeros(ng.value + 1, np.int64),
                 pp_begin=np.zeros(max(1, npr.value), np.int32),
                 pp_end=np.zeros(max(1, npr.value), np.int32))
        pp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(self.lib.gx_gravity_list_export(self.ctx, pp(o["pc_off"]), pp(o["pc"]),
                                                    pp(o["pp_off"]), pp(o["pp_begin"]),
                                                    pp(o["pp_end"])))
        o["pc"] = o["pc"][:npc.value]
        o["pp_begin"] = o["pp_begin"][:npr.value]
        o["pp_end"] = o["pp_end"][:npr.value]
        return o

    # ---- supernova surrogate: SN regions -------------------------------------
    def sn_extract(self, gas: ParticleSet, centers, half_side, cap):
        """Members of the boxes around each site: (offsets[k+1], idx[total], total)."""
        torch = _torch()
        k = int(centers.shape[0])
        offsets = torch.zeros(k + 1, dtype=torch.int32, device=centers.device)
        idx = torch.zeros(max(1, int(cap)), dtype=torch.int32, device=centers.device)
        tot = C.c_int64()
        self._check(self.lib.gx_sn_extract(self.ctx, C.byref(gas.view()), _ptr(centers, torch.float64),
                                           k, float(half_side), _ptr(offsets), _ptr(idx), int(cap),
                                           C.byref(tot)))
        return offsets, idx[:tot.value], tot.value

    def sn_inject(self, gas: ParticleSet, offsets, idx, centers, k_inj, energy, u):
        torch = _torch()
        self._check(self.lib.gx_sn_inject(self.ctx, C.byref(gas.view()), _ptr(offsets, torch.int32),
                                          _ptr(idx, torch.int32), _ptr(centers, torch.float64),
                                          int(centers.shape[0]), int(k_inj), float(energy),
                                          _ptr(u, torch.float64)))

    def sn_ambient(self, gas: ParticleSet, u, offsets, idx, side, u_to_T, amb=None):
        """Per-box ambient (log10 rho, log10 T, vx, vy, vz) from the extracted members."""
        torch = _torch()
        k = int(offsets.shape[0]) - 1
        if amb is None:
            amb = torch.zeros(k * 5, dtype=torch.float32, device=u.device)
        self._check(self.lib.gx_sn_ambient(self.ctx, C.byref(gas.view()), _ptr(u, torch.float64),
                                           _ptr(offsets, torch.int32), _ptr(idx, torch.int32), k,
                                           float(side), float(u_to_T), _ptr(amb, torch.float32)))
        return amb

    def sn_gather(self, gas: ParticleSet, u, H, offsets, idx, n_max, centers, dst, scale, out: dict):
        """Pack box members into `out` (x, y, z, vx, vy, vz, m, u FP64; H FP32 or absent)."""
        torch = _torch()
        k = int(offsets.shape[0]) - 1
        f = [_ptr(out[a], torch.float64) for a in ("x", "y", "z", "vx", "vy", "vz", "m", "u")]
        self._check(self.lib.gx_sn_gather(self.ctx, C.byref(gas.view()), _ptr(u, torch.float64),
                                          _ptr(H, torch.float32), _ptr(offsets, torch.int32),
                                          _ptr(idx, torch.int32), k, int(n_max),
                                          _ptr(centers, torch.float64), _ptr(dst, torch.float64),
                                          float(scale), *f, _ptr(out.get("H"), torch.float32)))

    def sn_unframe(self, offsets, n_max, src, centers, amb, dt, scale, x, y, z):
        torch = _torch()
        k = int(offsets.shape[0]) - 1
        self._check(self.lib.gx_sn_unframe(self.ctx, _ptr(offsets, torch.int32), k, int(n_max),
                                           _ptr(src, torch.float64), _ptr(centers, torch.float64),
                                           _ptr(amb, torch.float32), float(dt), float(scale),
                                           _ptr(x, torch.float64), _ptr(y, torch.float64),
                                           _ptr(z, torch.float64)))

    def sn_voxelize(self, gas: ParticleSet, u, H, centers, side, grid, u_to_T, amb, mean=None,
                    std=None, out_bf16=None, cpad=8, out_f32=None):
        torch = _torch()
        self._check(self.lib.gx_sn_voxelize(
            self.ctx, C.byref(gas.view()), _ptr(u, torch.float64), _ptr(H, torch.float32),
            _ptr(centers, torch.float64), int(centers.shape[0]), float(side), int(grid),
            float(u_to_T), _ptr(amb, torch.float32), _ptr(mean, torch.float32),
            _ptr(std, torch.float32), _ptr(out_bf16, torch.bfloat16), int(cpad),
            _ptr(out_f32, torch.float32)))

    def sn_resample(self, pred, centers, grid, side, out_off, n_out_max, uniforms, T_to_u, x, y, z,
                    vx, vy, vz, u):
        torch = _torch()
        self._check(self.lib.gx_sn_resample(
            self.ctx, _ptr(pred, torch.float32), int(centers.shape[0]), int(grid), float(side),
            _ptr(centers, torch.float64), _ptr(out_off, torch.int32), int(n_out_max),
            _ptr(uniforms, torch.float32), float(T_to_u), *(_ptr(t, torch.float64) for t in
                                                              (x, y, z, vx, vy, vz, u))))

    def sn_resample_gibbs(self, pred, centers, grid, side, out_off, n_out_max, x0, y0, z0,
                          sweeps, uniforms, T_to_u, x, y, z, vx, vy, vz, u):
        """Gibbs resampling: chains start in the voxels of (x0, y0, z0);
        uniforms float [total * (3 * sweeps + 3)]."""
        torch = _torch()
        self._check(self.lib.gx_sn_resample_gibbs(
            self.ctx, _ptr(pred, torch.float32), int(centers.shape[0]), int(grid), float(side),
            _ptr(centers, torch.float64), _ptr(out_off, torch.int32), int(n_out_max),
            _ptr(x0, torch.float64), _ptr(y0, torch.float64), _ptr(z0, torch.float64),
            int(sweeps), _ptr(uniforms, torch.float32), float(T_to_u),
            *(_ptr(t, torch.float64) for t in (x, y, z, vx, vy, vz, u))))

    def sn_encode8(self, in5, V, v0, out8, in_stride=5):
        """Eight-cube encoding of V physical rows into out8 float [V * 8]."""
        torch = _torch()
        self._check(self.lib.gx_sn_encode8(self.ctx, int(V), _ptr(in5, torch.float32),
                                           int(in_stride), float(v0), _ptr(out8, torch.float32)))
        return out8

    def sn_decode8(self, in8, V, out5, in_stride=8):
        """Physical rows (log10 rho, log10 T, v) from eight-cube rows."""
        torch = _torch()
        self._check(self.lib.gx_sn_decode8(self.ctx, int(V), _ptr(in8, torch.float32),
                                           int(in_stride), _ptr(out5, torch.float32)))
        return out5

    def sn_check(self, pred, k, grid, lo, hi):
        """Per-cube trust flags (numpy bool [k]) of a prediction: every value
        finite and inside [lo, hi] of its channel (lo, hi: 5 floats)."""
        torch = _torch()
        lo_h = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(5))
        hi_h = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).reshape(5))
        ok = np.zeros(max(int(k), 1), dtype=np.uint8)
        self._check(self.lib.gx_sn_check(
            self.ctx, _ptr(pred, torch.float32), int(k), int(grid),
            lo_h.ctypes.data_as(C.c_void_p), hi_h.ctypes.data_as(C.c_void_p),
            ok.ctypes.data_as(C.c_void_p)))
        return ok[:int(k)].astype(bool)

    def sn_check_noalloc(self, pred, k, grid, lo, hi, ok_dev):
        """gx_sn_check without allocation or synchronisation: flags written to
        the device uint8 tensor ok_dev [k] (1 = trusted)."""
        torch = _torch()
        lo_h = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(5))
        hi_h = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).reshape(5))
        self._check(self.lib.gx_sn_check_noalloc(
            self.ctx, _ptr(pred, torch.float32), int(k), int(grid),
            lo_h.ctypes.data_as(C.c_void_p), hi_h.ctypes.data_as(C.c_void_p),
            _ptr(ok_dev, torch.uint8)))
        return ok_dev

    def sn_replace(self, id, id_cap, x, y, z, vx, vy, vz, u, u_offset, H64, new_id, nx, ny, nz, nvx,
                   nvy, nvz, nu):
        torch = _torch()
        miss = C.c_int64()
        self._check(self.lib.gx_sn_replace(
            self.ctx, int(id.shape[0]), _ptr(id, torch.int64), int(id_cap),
            *(_ptr(t, torch.float64) for t in (x, y, z, vx, vy, vz, u)), int(u_offset),
            _ptr(H64, torch.float64), int(new_id.shape[0]), _ptr(new_id, torch.int64),
            *(_ptr(t, torch.float64) for t in (nx, ny, nz, nvx, nvy, nvz, nu)), C.byref(miss)))
        return miss.value

    # ---- supernova surrogate: network blocks ------------------------------------
    def conv3d_fwd(self, x, B, S, Cin, w, bias, ksize, Cout, act, out_bf16=None, out_f32=None):
        torch = _torch()
        self._check(self.lib.gx_conv3d_fwd(self.ctx, _ptr(x, torch.bfloat16), B, S, Cin,
                                           _ptr(w, torch.bfloat16), _ptr(bias, torch.float32),
                                           ksize, Cout, int(act), _ptr(out_bf16, torch.bfloat16),
                                           _ptr(out_f32, torch.float32)))

    def conv3d_fwd_fused(self, x, c1, x2, upsample, B, S, Cin, w, bias, Cout, act, out_bf16=None,
                         out_f32=None):
        torch = _torch()
        self._check(self.lib.gx_conv3d_fwd_fused(
            self.ctx, _ptr(x, torch.bfloat16), int(c1), _ptr(x2, torch.bfloat16), int(upsample), B,
            S, Cin, _ptr(w, torch.bfloat16), _ptr(bias, torch.float32), Cout, int(act),
            _ptr(out_bf16, torch.bfloat16), _ptr(out_f32, torch.float32)))

    def conv_head(self, x, B, S, Cin, w, bias, Cout, nc, scale, shift, out, out_stride):
        torch = _torch()
        self._check(self.lib.gx_conv_head(
            self.ctx, _ptr(x, torch.bfloat16), B, S, Cin, _ptr(w, torch.bfloat16),
            _ptr(bias, torch.float32), Cout, int(nc), _ptr(scale, torch.float32),
            _ptr(shift, torch.float32), _ptr(out, torch.float32), int(out_stride)))

    def conv3d_fwd_pool(self, x, B, S, Cin, w, bias, Cout, act, out_bf16, pool_bf16):
        torch = _torch()
        self._check(self.lib.gx_conv3d_fwd_pool(
            self.ctx, _ptr(x, torch.bfloat16), B, S, Cin, _ptr(w, torch.bfloat16),
            _ptr(bias, torch.float32), Cout, int(act), _ptr(out_bf16, torch.bfloat16),
            _ptr(pool_bf16, torch.bfloat16)))

    def conv3d_bwd_data(self, dout, B, S, Cin, w, ksize, Cout, y_in, din):
        torch = _torch()
        self._check(self.lib.gx_conv3d_bwd_data(self.ctx, _ptr(dout, torch.bfloat16), B, S, Cin,
                                                _ptr(w, torch.bfloat16), ksize, Cout,
                                                _ptr(y_in, torch.bfloat16),
                                                _ptr(din, torch.bfloat16)))

    def conv3d_bwd_weight(self, x, dout, B, S, Cin, ksize, Cout, dw, dbias=None):
        torch = _torch()
        self._check(self.lib.gx_conv3d_bwd_weight(self.ctx, _ptr(x, torch.bfloat16),
                                                  _ptr(dout, torch.bfloat16), B, S, Cin, ksize,
                                                  Cout, _ptr(dw, torch.float32),
                                                  _ptr(dbias, torch.float32)))

    def conv3d_bwd_weight_fused(self, x, c1, x2, upsample, dout, B, S, Cin, ksize, Cout, dw,
                                dbias=None):
        torch = _torch()
        self._check(self.lib.gx_conv3d_bwd_weight_fused(
            self.ctx, _ptr(x, torch.bfloat16), int(c1), _ptr(x2, torch.bfloat16), int(upsample),
            _ptr(dout, torch.bfloat16), B, S, Cin, ksize, Cout, _ptr(dw, torch.float32),
            _ptr(dbias, torch.float32)))

    def avgpool2(self, x, B, S, Cc, out, backward=False):
        torch = _torch()
        self._check(self.lib.gx_avgpool2(self.ctx, _ptr(x, torch.bfloat16), B, S, Cc,
                                         _ptr(out, torch.bfloat16), int(backward)))

    def upsample2(self, x, B, S, Cc, out, backward=False):
        torch = _torch()
        self._check(self.lib.gx_upsample2(self.ctx, _ptr(x, torch.bfloat16), B, S, Cc,
                                          _ptr(out, torch.bfloat16), int(backward)))

    def concat(self, a, Ca, b, Cb, V, out, split=False):
        torch = _torch()
        self._check(self.lib.gx_concat(self.ctx, _ptr(a, torch.bfloat16), Ca,
                                       _ptr(b, torch.bfloat16), Cb, int(V),
                                       _ptr(out, torch.bfloat16), int(split)))

    def mse(self, pred, Cp, target, nc, V, dpred=None):
        torch = _torch()
        loss = C.c_double()
        self._check(self.lib.gx_mse(self.ctx, _ptr(pred, torch.float32), Cp,
                                    _ptr(target, torch.float32), nc, int(V),
                                    _ptr(dpred, torch.bfloat16), C.byref(loss)))
        return loss.value

    def adam_step(self, w, grad, m, v, lr, b1, b2, eps, t, w_bf16=None):
        torch = _torch()
        self._check(self.lib.gx_adam_step(self.ctx, int(w.numel()), _ptr(w, torch.float32),
                                          _ptr(grad, torch.float32), _ptr(m, torch.float32),
                                          _ptr(v, torch.float32), float(lr), float(b1), float(b2),
                                          float(eps), int(t), _ptr(w_bf16, torch.bfloat16)))

    def grad_combine(self, a, b, y, out):
        torch = _torch()
        self._check(self.lib.gx_grad_combine(self.ctx, int(a.numel()), _ptr(a, torch.bfloat16),
                                             _ptr(b, torch.bfloat16), _ptr(y, torch.bfloat16),
                                             _ptr(out, torch.bfloat16)))

    def cube_sym(self, x, B, S, C, vc, sym, out):
        """Cube symmetry sym[b] (perm * 8 + flips) of each sample of x -> out."""
        torch = _torch()
        self._check(self.lib.gx_cube_sym(self.ctx, _ptr(x, torch.float32), int(B), int(S), int(C),
                                         int(vc), _ptr(sym, torch.int32), _ptr(out, torch.float32)))

    def chan_stats(self, x, stride, nc, sums):
        """sums (device float64 [2 nc]) += per-channel sum and sum of squares."""
        torch = _torch()
        V = int(x.numel()) // int(stride)
        self._check(self.lib.gx_chan_stats(self.ctx, V, _ptr(x, torch.float32), int(stride), int(nc),
                                           _ptr(sums, torch.float64)))

    def chan_affine(self, x, in_stride, nc, scale, shift, out=None, out_stride=None, out_bf16=None,
                    bf_stride=None):
        torch = _torch()
        V = int(x.numel()) // int(in_stride)
        self._check(self.lib.gx_chan_affine(
            self.ctx, V, _ptr(x, torch.float32), int(in_stride), int(nc), _ptr(scale, torch.float32),
            _ptr(shift, torch.float32), _ptr(out, torch.float32), int(out_stride or nc),
            _ptr(out_bf16, torch.bfloat16), int(bf_stride or nc)))

    def chan_moments(self, sums, nc, count, min_std, mean=None, std=None, scale=None,
                     shift=None):
        """Mean, floored standard deviation and the standardising affine map
        (scale = 1/std, shift = -mean/std) from FP64 channel sums."""
        torch = _torch()
        f = lambda t: _ptr(t, torch.float32)
        self._check(self.lib.gx_chan_moments(self.ctx, _ptr(sums, torch.float64), int(nc),
                                             float(count), float(min_std), f(mean), f(std),
                                             f(scale), f(shift)))

    # ---- whole network -------------------------------------------------------
    def _unet_desc(self, levels, base, cin, cout, w_bf16, w_f32):
        torch = _torch()
        return _lib.GxUNet(int(levels), int(base), int(cin), int(cout),
                           _ptr(w_bf16, torch.bfloat16), _ptr(w_f32, torch.float32))

    def unet_forward(self, desc, x, B, S, save, out_f32=None, nc=0, scale=None, shift=None,
                     out_phys=None):
        torch = _torch()
        self._check(self.lib.gx_unet_forward(
            self.ctx, C.byref(desc), _ptr(x, torch.bfloat16), int(B), int(S), int(bool(save)),
            _ptr(out_f32, torch.float32), int(nc), _ptr(scale, torch.float32),
            _ptr(shift, torch.float32), _ptr(out_phys, torch.float32)))

    def unet_backward(self, desc, x, B, S, dout, grad):
        torch = _torch()
        self._check(self.lib.gx_unet_backward(self.ctx, C.byref(desc), _ptr(x, torch.bfloat16),
                                              int(B), int(S), _ptr(dout, torch.bfloat16),
                                              _ptr(grad, torch.float32)))

    def unet_saved(self, name: str, gradient: bool = False):
        """Copy of a tensor kept by the last saving forward pass (bf16, flat)."""
        torch = _torch()
        cnt = C.c_int64(0)
        self._check(self.lib.gx_unet_saved(self.ctx, name.encode(), int(gradient), None, 0,
                                           C.byref(cnt)))
        out = torch.empty(cnt.value, dtype=torch.bfloat16, device=f"cuda:{self.device}")
        self._check(self.lib.gx_unet_saved(self.ctx, name.encode(), int(gradient),
                                           _ptr(out, torch.bfloat16), cnt.value, C.byref(cnt)))
        return out

    def f32_to_bf16(self, x, y):
        torch = _torch()
        self._check(self.lib.gx_f32_to_bf16(self.ctx, _ptr(x, torch.float32), int(x.numel()),
                                            _ptr(y, torch.bfloat16)))


def unet_sizes(levels, base, cin, cout):
    """(n_params, n_layers) of a network description."""
    lib = _lib.load()
    n, k = C.c_int64(0), C.c_int64(0)
    rc = lib.gx_unet_sizes(int(levels), int(base), int(cin), int(cout), C.byref(n), C.byref(k))
    if rc:
        raise GxError(rc, "bad network description")
    return n.value, k.value


def unet_layers(levels, base, cin, cout):
    """Per layer: (name, cin, cout, ksize, w_off, b_off), in the library's order."""
    lib = _lib.load()
    _, nl = unet_sizes(levels, base, cin, cout)
    out = []
    for i in range(nl):
        name = C.create_string_buffer(16)
        ci, co, ks = C.c_int(0), C.c_int(0), C.c_int(0)
        wo, bo = C.c_int64(0), C.c_int64(0)
        rc = lib.gx_unet_layer(int(levels), int(base), int(cin), int(cout), i, name, 16,
                               C.byref(ci), C.byref(co), C.byref(ks), C.byref(wo), C.byref(bo))
        if rc:
            raise GxError(rc, "bad layer index")
        out.append((name.value.decode(), ci.value, co.value, ks.value, wo.value, bo.value))
    return out


def version() -> str:
    return _lib.load().gx_version().decode()
