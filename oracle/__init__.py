"""FP64 CPU oracle for the interaction path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never does.

The arithmetic lives in ``gx_oracle.c`` (plain C, FP64, OpenMP over
receivers) and in the small NumPy functions below; this file only marshals
arguments.  It shares no code with the HIP path.

Functions and the passages they follow
--------------------------------------
direct_gravity     Eq. 1 (Sec. 3.5), direct sum, self pair excluded.
Tree               Barnes-Hut octree (Sec. 3.4) over Morton-sorted particles,
                   groups sharing one interaction list (Sec. 5.2.2, 5.2.4).
sph_density        kernel size + density/pressure (Sec. 5.2.5; Table 3/4).
sph_force          hydro force (Table 3/4).
kick_drift         second-order leapfrog, half kick / drift / half kick
                   (Sec. 3.2), positions and velocities in FP64 (Sec. 4.3).
energy             total energy audit in FP64.
eos                ideal-gas pressure and sound speed.
conv3d*, voxelize  the surrogate's convolutions and particle-to-grid mapping
                   (Sec. 3.3); the network composition is in ``oracle.unet``.
sn                 (module) the supernova-region steps of Sec. 3.2: box
                   extraction, injection, ambient state, inverse-CDF
                   resampling, trust check, replacement by ID.

Every function is pinned by the CPU tests to something other than itself:
closed forms, brute force, invariants, hand-computed cases (the opening
criterion at its boundary, the cell softening through its expansion, a
head-on viscous pair), finite differences and statistical tests.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

P = C.c_void_p
I64 = C.c_int64
D = C.c_double


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp",
                               "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_direct_gravity.argtypes = [I64, P, P, P, P, P, D, I64, P, P, P, P, P]
        L.orc_root_box.argtypes = [I64, P, P, P, P]
        L.orc_morton_keys.argtypes = [I64, P, P, P, P, P]
        L.orc_tree_build.argtypes = [I64, P, P, P, P, P, C.c_int, C.c_int]
        L.orc_tree_build.restype = P
        L.orc_tree_free.argtypes = [P]
        L.orc_tree_nnodes.argtypes = [P]
        L.orc_tree_nnodes.restype = I64
        L.orc_tree_ngroups.argtypes = [P]
        L.orc_tree_ngroups.restype = I64
        L.orc_tree_box.argtypes = [P, P]
        L.orc_tree_get_sorted.argtypes = [P, P, P]
        L.orc_tree_get_nodes.argtypes = [P] + [P] * 11
        L.orc_tree_get_groups.argtypes = [P, P]
        L.orc_tree_list_counts.argtypes = [P, D, P, P, P]
        L.orc_tree_list_fill.argtypes = [P, D, P, P, P, P]
        L.orc_tree_gravity.argtypes = [P, D, D, C.c_int, P, P, P, P, P, P]
        L.orc_tree_gravity_groups.argtypes = [P, D, D, C.c_int, I64, P, P, P, P, P, P, P]
        L.orc_node_field.argtypes = [P, I64, C.c_int, P, P]
        L.orc_wendland_c4.argtypes = [D, D]
        L.orc_wendland_c4.restype = D
        L.orc_wendland_c4_dr.argtypes = [D, D]
        L.orc_wendland_c4_dr.restype = D
        L.orc_sph_density.argtypes = [I64, P, P, P, P, D, D, C.c_int, I64, P, P, P, P, P, P]
        L.orc_sph_density.restype = I64
        L.orc_sph_force.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, D, D, I64, P,
                                    P, P, P, P, P]
        ci = C.c_int
        L.orc_conv3d_fwd.argtypes = [ci, ci, ci, ci, ci, P, P, P, P]
        L.orc_conv3d_bwd_data.argtypes = [ci, ci, ci, ci, ci, P, P, P]
        L.orc_conv3d_bwd_weight.argtypes = [ci, ci, ci, ci, ci, P, P, P, P]
        L.orc_voxelize.argtypes = [I64] + [P] * 10 + [D, ci, P, D, D, P]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def direct_gravity(p: dict, G: float = 1.0, idx=None):
    """FP64 direct sum of Eq. 1.  Returns (ax, ay, az, pot) for receivers idx (or all)."""
    x, y, z, m = (_f64(p[k]) for k in ("x", "y", "z", "m"))
    e2 = _f64(p["eps2"])
    n = x.size
    if idx is not None:
        idx = np.ascontiguousarray(idx, np.int64)
    k = n if idx is None else idx.size
    out = [np.zeros(k) for _ in range(4)]
    lib().orc_direct_gravity(n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(e2), G,
                             k, _ptr(idx), *(_ptr(o) for o in out))
    return tuple(out)


def root_box(p: dict):
    x, y, z = (_f64(p[k]) for k in ("x", "y", "z"))
    out = np.zeros(4)
    lib().orc_root_box(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(out))
    return out


def morton_keys(p: dict, box=None):
    x, y, z = (_f64(p[k]) for k in ("x", "y", "z"))
    box = root_box(p) if box is None else _f64(box)
    keys = np.zeros(x.size, np.uint64)
    lib().orc_morton_keys(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(box), _ptr(keys))
    return keys


class Tree:
    """Octree over Morton-sorted particles (nodes in depth-first pre-order)."""

    def __init__(self, p: dict, n_leaf: int = 16, n_group: int = 256):
        self._keep = [_f64(p[k]) for k in ("x", "y", "z", "m", "eps2")]
        x, y, z, m, e2 = self._keep
        self.n = x.size
        self._h = lib().orc_tree_build(self.n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(e2),
                                       n_leaf, n_group)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_tree_free(self._h)
            self._h = None

    @property
    def n_nodes(self):
        return int(lib().orc_tree_nnodes(self._h))

    @property
    def n_groups(self):
        return int(lib().orc_tree_ngroups(self._h))

    def box(self):
        out = np.zeros(4)
        lib().orc_tree_box(self._h, _ptr(out))
        return out

    def sorted(self):
        key = np.zeros(self.n, np.uint64)
        perm = np.zeros(self.n, np.int64)
        lib().orc_tree_get_sorted(self._h, _ptr(key), _ptr(perm))
        return key, perm

    def nodes(self):
        nn = self.n_nodes
        o = dict(begin=np.zeros(nn, np.int64), end=np.zeros(nn, np.int64),
                 next=np.zeros(nn, np.int64), level=np.zeros(nn, np.int32),
                 leaf=np.zeros(nn, np.int8), mass=np.zeros(nn), com=np.zeros((nn, 3)),
                 quad=np.zeros((nn, 6)), eps2bar=np.zeros(nn), lo=np.zeros((nn, 3)),
                 hi=np.zeros((nn, 3)))
        lib().orc_tree_get_nodes(self._h, *(_ptr(o[k]) for k in (
            "begin", "end", "next", "level", "leaf", "mass", "com", "quad", "eps2bar",
            "lo", "hi")))
        return o

    def groups(self):
        g = np.zeros(self.n_groups, np.int64)
        lib().orc_tree_get_groups(self._h, _ptr(g))
        return g

    def lists(self, theta: float):
        """Per-group interaction lists: (pp_off, pp_leaf_nodes, pc_off, pc_nodes, npp_particles)."""
        ng = self.n_groups
        a, c, p = (np.zeros(ng, np.int64) for _ in range(3))
        lib().orc_tree_list_counts(self._h, theta, _ptr(a), _ptr(c), _ptr(p))
        pp_off = np.concatenate([[0], np.cumsum(a)]).astype(np.int64)
        pc_off = np.concatenate([[0], np.cumsum(c)]).astype(np.int64)
        pp = np.zeros(max(1, pp_off[-1]), np.int64)
        pc = np.zeros(max(1, pc_off[-1]), np.int64)
        lib().orc_tree_list_fill(self._h, theta, _ptr(pp_off), _ptr(pc_off), _ptr(pp), _ptr(pc))
        return pp_off, pp[:pp_off[-1]], pc_off, pc[:pc_off[-1]], p

    def gravity(self, G: float = 1.0, theta: float = 0.5, quad: bool = True):
        """FP64 tree force at original indices: (ax, ay, az, pot, n_pp, n_pc)."""
        out = [np.zeros(self.n) for _ in range(4)]
        npp = C.c_int64(0)
        npc = C.c_int64(0)
        lib().orc_tree_gravity(self._h, G, theta, int(quad), *(_ptr(o) for o in out),
                               C.byref(npp), C.byref(npc))
        return (*out, npp.value, npc.value)

    def gravity_groups(self, groups, G: float = 1.0, theta: float = 0.5, quad: bool = True):
        """FP64 tree force for the receivers of the given groups only (original indices;
        other entries stay zero): (ax, ay, az, pot, n_pp, n_pc)."""
        gsel = np.ascontiguousarray(groups, np.int64)
        out = [np.zeros(self.n) for _ in range(4)]
        npp = C.c_int64(0)
        npc = C.c_int64(0)
        lib().orc_tree_gravity_groups(self._h, G, theta, int(quad), gsel.size, _ptr(gsel),
                                      *(_ptr(o) for o in out), C.byref(npp), C.byref(npc))
        return (*out, npp.value, npc.value)

    def node_field(self, node: int, r, quad: bool = True):
        out = np.zeros(4)
        r = _f64(r)
        lib().orc_node_field(self._h, node, int(quad), _ptr(r), _ptr(out))
        return out


def wendland_c4(r: float, H: float) -> float:
    return lib().orc_wendland_c4(float(r), float(H))


def wendland_c4_dr(r: float, H: float) -> float:
    return lib().orc_wendland_c4_dr(float(r), float(H))


def sph_density(gas: dict, n_ngb: float = 64.0, tol: float = 1e-10, max_iter: int = 200,
                idx=None, H_guess=None, with_slope=False):
    """Kernel size and density by safeguarded Newton.

    Returns (H, rho, iters, n_fail), plus dN_eff/dln H at the solution when
    ``with_slope``."""
    x, y, z, m = (_f64(gas[k]) for k in ("x", "y", "z", "m"))
    n = x.size
    if idx is not None:
        idx = np.ascontiguousarray(idx, np.int64)
    k = n if idx is None else idx.size
    H = np.zeros(k)
    rho = np.zeros(k)
    it = np.zeros(k, np.int32)
    hg = None if H_guess is None else _f64(H_guess)
    slope = np.zeros(k)
    nfail = lib().orc_sph_density(n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), n_ngb, tol, max_iter,
                                  k, _ptr(idx), _ptr(hg), _ptr(H), _ptr(rho), _ptr(it),
                                  _ptr(slope))
    if with_slope:
        return H, rho, it, int(nfail), slope
    return H, rho, it, int(nfail)


def sph_force(gas: dict, H, rho, gamma: float = 5.0 / 3.0, alpha: float = 1.0, idx=None,
              vel=None, u=None):
    """Hydro acceleration, du/dt, signal speed.  Returns (ax, ay, az, dudt, vsig)."""
    x, y, z, m = (_f64(gas[k]) for k in ("x", "y", "z", "m"))
    if vel is None:
        vel = (gas["vx"], gas["vy"], gas["vz"])
    vx, vy, vz = (_f64(v) for v in vel)
    uu = _f64(gas["u"] if u is None else u)
    H = _f64(H)
    rho = _f64(rho)
    n = x.size
    if idx is not None:
        idx = np.ascontiguousarray(idx, np.int64)
    k = n if idx is None else idx.size
    out = [np.zeros(k) for _ in range(5)]
    lib().orc_sph_force(n, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m),
                        _ptr(uu), _ptr(H), _ptr(rho), gamma, alpha, k, _ptr(idx),
                        *(_ptr(o) for o in out))
    return tuple(out)


def eos(rho, u, gamma: float = 5.0 / 3.0):
    """Ideal gas: P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u)."""
    rho = _f64(rho)
    u = _f64(u)
    return (gamma - 1.0) * rho * u, np.sqrt(gamma * (gamma - 1.0) * u)


def kick_drift(x, v, a, dt_kick, dt_drift, u=None, dudt=None):
    """One half of the leapfrog of Sec. 3.2 in FP64, on (3, n) arrays.

    v <- v + a dt_kick; u <- u + du/dt dt_kick; x <- x + v dt_drift.
    Returns new (x, v, u) plus the predicted (v + a dt_kick, u + du/dt dt_kick)
    that the hydro force of the next evaluation uses.
    """
    x = _f64(x).copy()
    v = _f64(v).copy()
    v = v + _f64(a) * dt_kick
    un = None
    upred = None
    if u is not None:
        un = _f64(u) + _f64(dudt) * dt_kick
        upred = un + _f64(dudt) * dt_kick
    x = x + v * dt_drift
    vpred = v + _f64(a) * dt_kick
    return x, v, un, vpred, upred


def energy(m, v, pot, u_gas=None, m_gas=None):
    """(kinetic, potential, thermal) in FP64: sum m v^2/2, sum m phi / 2, sum m u."""
    m = _f64(m)
    v = _f64(v)
    K = 0.5 * float(np.sum(m * np.sum(v * v, axis=0)))
    W = 0.5 * float(np.sum(m * _f64(pot)))
    U = 0.0 if u_gas is None else float(np.sum(_f64(m_gas) * _f64(u_gas)))
    return K, W, U


# ---------------------------------------------------------------------------
# Surrogate network (Sec. 3.3): convolution blocks and U-Net composition
# ---------------------------------------------------------------------------
def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3d(x, w, bias=None, ksize=3):
    """x [B,S,S,S,Cin], w [Cout,kvol,Cin] -> [B,S,S,S,Cout] (FP64)."""
    x = _f64(x)
    w = _f64(w)
    B, S, _, _, Cin = x.shape
    Cout = w.shape[0]
    out = np.zeros((B, S, S, S, Cout))
    b = None if bias is None else _f64(bias)
    lib().orc_conv3d_fwd(B, S, Cin, Cout, ksize, _ptr(x), _ptr(w), _ptr(b), _ptr(out))
    return out


def conv3d_bwd_data(dout, w, Cin, ksize=3):
    dout = _f64(dout)
    w = _f64(w)
    B, S, _, _, Cout = dout.shape
    din = np.zeros((B, S, S, S, Cin))
    lib().orc_conv3d_bwd_data(B, S, Cin, Cout, ksize, _ptr(dout), _ptr(w), _ptr(din))
    return din


def conv3d_bwd_weight(x, dout, ksize=3):
    x = _f64(x)
    dout = _f64(dout)
    B, S, _, _, Cin = x.shape
    Cout = dout.shape[-1]
    kv = 27 if ksize == 3 else 1
    dw = np.zeros((Cout, kv, Cin))
    db = np.zeros(Cout)
    lib().orc_conv3d_bwd_weight(B, S, Cin, Cout, ksize, _ptr(x), _ptr(dout), _ptr(dw), _ptr(db))
    return dw, db


def lrelu(x, a=0.1):
    return np.where(x > 0, x, a * x)


def avgpool2(x):
    B, S, _, _, C = x.shape
    return x.reshape(B, S // 2, 2, S // 2, 2, S // 2, 2, C).mean(axis=(2, 4, 6))


def upsample2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def voxelize(p, u_to_T, center, side, grid, amb, rho_floor_frac=1e-6, t_floor=10.0, H=None):
    """Brute-force particle-to-voxel mapping; returns [grid, grid, grid, 5]."""
    Hh = _f64(p["H"] if H is None else H)
    T = _f64(p["u"]) * u_to_T
    out = np.zeros((grid ** 3, 5))
    amb = _f64(amb)
    lib().orc_voxelize(len(p["x"]), *(_ptr(_f64(p[k])) for k in ("x", "y", "z", "m")), _ptr(Hh),
                       _ptr(T), *(_ptr(_f64(p[k])) for k in ("vx", "vy", "vz")),
                       _ptr(_f64(center)), float(side), int(grid), _ptr(amb),
                       float(rho_floor_frac * 10.0 ** amb[0]), float(t_floor), _ptr(out))
    return out.reshape(grid, grid, grid, 5)
