"""Supernova-region steps in plain FP64 NumPy -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.  Nothing here is shared with
the HIP path.

Each function writes out the definition it follows, as plainly as possible:

extract    Sec. 3.2 step 2: the gas inside the box of side 2h around each
           SN site, membership c - h <= x < c + h on every axis, original
           indices ascending within each box.
inject     the thermal energy of one SN (10^51 erg, Sec. 1) given to the
           k_inj members nearest the box centre (ties by index), as the same
           specific energy E / (their total mass).
ambient    the box's mean state (mean density, mass-weighted temperature and
           bulk velocity): the value of voxels no particle kernel reaches in
           the particle-to-grid mapping of Sec. 3.3.
resample   the grid-to-particle mapping of Sec. 3.3 read as exact sampling of
           the piecewise-constant density: the voxel by inverse CDF of
           10^(log10 rho_v), the position uniform inside it, T and v of that
           voxel, as many particles as entered (mass conserved).
resample_gibbs
           the same mapping by Gibbs sampling (the Markov-chain method Sec.
           3.3 names): each particle's chain starts in the voxel of the
           particle that entered, and each sweep redraws the x index from the
           density along the line through the current (y, z), then y given
           (x, z), then z given (x, y), each by the inverse CDF of the line's
           weights 10^(log10 rho); then the position uniform inside the final
           voxel and its T and v.
encode8    the eight-cube input encoding of Sec. 3.3: log10 rho, log10 T, and
           per velocity component a positive and a negative cube holding the
           logarithm of the magnitude, log10(v0 + max(+-v, 0)) (the offset v0
           keeps the logarithm finite where a cube is empty).
decode8    its inverse, v = 10^(c+) - 10^(c-) (v0 cancels).
check      trust flags of a prediction: every value finite and inside its
           channel's [lo, hi] (compared in FP32).
replace    Sec. 3.2 step 4: the new state written over the particles with the
           same IDs; when an ID appears more than once among the new
           particles the last one in the list wins.
"""
from __future__ import annotations

import numpy as np


def extract(x, y, z, centers, half):
    """CSR (offsets [K+1], idx) of the particles inside each half-open box."""
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    off = [0]
    idx = []
    for c in centers:
        inside = ((x >= c[0] - half) & (x < c[0] + half) &
                  (y >= c[1] - half) & (y < c[1] + half) &
                  (z >= c[2] - half) & (z < c[2] + half))
        members = np.nonzero(inside)[0]
        idx.append(members)
        off.append(off[-1] + members.size)
    idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    return np.asarray(off, np.int64), idx.astype(np.int64)


def inject_selection(x, y, z, members, center, k_inj):
    """The k_inj members nearest the centre: squared distances in FP64 as
    dx*dx + dy*dy + dz*dz, ascending, ties kept in member (index) order."""
    members = np.asarray(members, np.int64)
    dx = x[members] - center[0]
    dy = y[members] - center[1]
    dz = z[members] - center[2]
    d2 = dx * dx + dy * dy + dz * dz
    order = np.lexsort((members, d2))
    return members[order[:min(k_inj, members.size)]]


def inject(x, y, z, m, off, idx, centers, k_inj, energy, u):
    """Returns u with each box's injection added (boxes processed in order)."""
    u = np.array(u, np.float64, copy=True)
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    for c in range(len(off) - 1):
        members = idx[off[c]:off[c + 1]]
        if members.size == 0:
            continue
        sel = inject_selection(x, y, z, members, centers[c], k_inj)
        u[sel] += energy / np.sum(m[sel])
    return u


def ambient(m, u, vx, vy, vz, off, idx, side, u_to_T, t_floor=10.0):
    """[K, 5]: log10(total member mass / side^3), log10(max(mass-weighted
    u * u_to_T, t_floor)), mass-weighted vx, vy, vz; a box without members
    gets (-30, log10 t_floor, 0, 0, 0)."""
    K = len(off) - 1
    out = np.zeros((K, 5))
    for c in range(K):
        mem = idx[off[c]:off[c + 1]]
        M = float(np.sum(m[mem]))
        if M > 0:
            out[c, 0] = np.log10(M / side ** 3)
            out[c, 1] = np.log10(max(np.sum(m[mem] * u[mem]) / M * u_to_T, t_floor))
            out[c, 2] = np.sum(m[mem] * vx[mem]) / M
            out[c, 3] = np.sum(m[mem] * vy[mem]) / M
            out[c, 4] = np.sum(m[mem] * vz[mem]) / M
        else:
            out[c] = (-30.0, np.log10(t_floor), 0.0, 0.0, 0.0)
    return out


def resample(pred, centers, grid, side, counts, uniforms, T_to_u):
    """pred [K, grid^3, 5] physical channels (log10 rho, log10 T, vx, vy, vz),
    voxel order z-major with x fastest; uniforms [total, 4] in [0, 1).
    Particle j of cube c takes the first voxel v whose inclusive prefix sum
    C[v] of 10^(log10 rho) exceeds uniforms[j, 0] * C[last], a position
    uniform inside v from uniforms[j, 1:4], and T, v of that voxel.
    Returns dict of x, y, z, vx, vy, vz, u and the chosen voxel per particle."""
    pred = np.asarray(pred, np.float64)
    K = pred.shape[0]
    nvox = grid ** 3
    uniforms = np.asarray(uniforms, np.float64).reshape(-1, 4)
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    dv = side / grid
    out = {k: [] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "voxel")}
    j = 0
    for c in range(K):
        C = np.cumsum(10.0 ** pred[c, :, 0])
        for _ in range(int(counts[c])):
            target = uniforms[j, 0] * C[-1]
            v = int(np.searchsorted(C, target, side="right"))
            v = min(v, nvox - 1)
            X, Y, Z = v % grid, (v // grid) % grid, v // (grid * grid)
            out["x"].append(centers[c, 0] - side / 2 + (X + uniforms[j, 1]) * dv)
            out["y"].append(centers[c, 1] - side / 2 + (Y + uniforms[j, 2]) * dv)
            out["z"].append(centers[c, 2] - side / 2 + (Z + uniforms[j, 3]) * dv)
            out["vx"].append(pred[c, v, 2])
            out["vy"].append(pred[c, v, 3])
            out["vz"].append(pred[c, v, 4])
            out["u"].append(10.0 ** pred[c, v, 1] * T_to_u)
            out["voxel"].append(v)
            j += 1
    return {k: np.asarray(v) for k, v in out.items()}


def line_draw(w, u):
    """Inverse-CDF draw along one line of voxel weights w (FP64): the first
    index whose inclusive prefix sum exceeds u * (the line's total), the
    prefix sums taken in index order; the last index if none does."""
    C = np.cumsum(np.asarray(w, np.float64))
    k = int(np.searchsorted(C, float(u) * C[-1], side="right"))
    return min(k, len(C) - 1)


def resample_gibbs(pred, centers, grid, side, counts, start, sweeps, uniforms, T_to_u,
                   sel=None):
    """pred [K, grid^3, 5] physical channels (voxel order z-major, x fastest);
    start [total, 3] positions of the particles that entered, in the frame of
    `centers`; uniforms [total, 3 * sweeps + 3] in [0, 1): uniforms[j, 3s],
    [3s + 1], [3s + 2] drive the x, y and z draws of sweep s, the last three
    the position inside the final voxel.  The chain of particle j starts at
    the voxel holding start[j] (indices clamped to the grid).  sel: the
    particles to compute (default all).  Returns dict of x, y, z, vx, vy, vz,
    u and the final voxel, for the particles of sel in order."""
    pred = np.asarray(pred, np.float64)
    K = pred.shape[0]
    start = np.asarray(start, np.float64).reshape(-1, 3)
    nu = 3 * sweeps + 3
    uniforms = np.asarray(uniforms, np.float64).reshape(-1, nu)
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    counts = np.asarray(counts, np.int64)
    off = np.concatenate([[0], np.cumsum(counts)])
    total = int(off[-1])
    sel = np.arange(total) if sel is None else np.asarray(sel, np.int64)
    cube_of = np.searchsorted(off, sel, side="right") - 1
    half = 0.5 * side
    dv = side / grid
    # weights rho_v per cube as [z, y, x] arrays
    rho = [(10.0 ** pred[c, :, 0]).reshape(grid, grid, grid) for c in range(K)]
    out = {k: [] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "voxel")}
    for j, c in zip(sel, cube_of):
        lo = centers[c] - half
        ijk = [min(max(int(np.floor((start[j, a] - lo[a]) / dv)), 0), grid - 1)
               for a in range(3)]
        X, Y, Z = ijk
        r = rho[c]
        for s in range(sweeps):
            X = line_draw(r[Z, Y, :], uniforms[j, 3 * s])
            Y = line_draw(r[Z, :, X], uniforms[j, 3 * s + 1])
            Z = line_draw(r[:, Y, X], uniforms[j, 3 * s + 2])
        v = (Z * grid + Y) * grid + X
        ub = uniforms[j, 3 * sweeps:]
        out["x"].append(lo[0] + (X + ub[0]) * dv)
        out["y"].append(lo[1] + (Y + ub[1]) * dv)
        out["z"].append(lo[2] + (Z + ub[2]) * dv)
        out["vx"].append(pred[c, v, 2])
        out["vy"].append(pred[c, v, 3])
        out["vz"].append(pred[c, v, 4])
        out["u"].append(10.0 ** pred[c, v, 1] * T_to_u)
        out["voxel"].append(v)
    return {k: np.asarray(v) for k, v in out.items()}


def encode8(phys, v0):
    """phys [..., 5] = (log10 rho, log10 T, vx, vy, vz) -> [..., 8] =
    (log10 rho, log10 T, log10(v0 + max(vx, 0)), log10(v0 + max(-vx, 0)),
    the same for vy, then vz)."""
    phys = np.asarray(phys, np.float64)
    out = np.empty(phys.shape[:-1] + (8,))
    out[..., 0] = phys[..., 0]
    out[..., 1] = phys[..., 1]
    for a in range(3):
        v = phys[..., 2 + a]
        out[..., 2 + 2 * a] = np.log10(v0 + np.maximum(v, 0.0))
        out[..., 3 + 2 * a] = np.log10(v0 + np.maximum(-v, 0.0))
    return out


def decode8(enc):
    """[..., 8] -> [..., 5]: log10 rho, log10 T kept; v = 10^(c+) - 10^(c-)."""
    enc = np.asarray(enc, np.float64)
    out = np.empty(enc.shape[:-1] + (5,))
    out[..., 0] = enc[..., 0]
    out[..., 1] = enc[..., 1]
    for a in range(3):
        out[..., 2 + a] = 10.0 ** enc[..., 2 + 2 * a] - 10.0 ** enc[..., 3 + 2 * a]
    return out


def check(pred, lo, hi):
    """ok[c] = every value of cube c finite and lo[ch] <= value <= hi[ch]."""
    pred = np.asarray(pred, np.float32)
    lo32 = np.asarray(lo, np.float64).astype(np.float32)
    hi32 = np.asarray(hi, np.float64).astype(np.float32)
    return np.array([bool(np.all(np.isfinite(p) & (p >= lo32) & (p <= hi32))) for p in pred])


def replace(ids, fields, new_ids, new_fields):
    """fields: dict of arrays indexed like ids; new_fields (a subset of the
    field names) indexed like new_ids.  Fields without new values (the
    masses) are kept.  Returns (updated copies, number of new ids not found)."""
    pos = {int(i): k for k, i in enumerate(np.asarray(ids))}
    out = {k: np.array(v, copy=True) for k, v in fields.items()}
    missing = 0
    for k, i in enumerate(np.asarray(new_ids)):
        if int(i) not in pos:
            missing += 1
            continue
        for f in new_fields:
            out[f][pos[int(i)]] = new_fields[f][k]
    return out, missing
