"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module draws particle sets only; it holds none of the method's
arithmetic (no forces, densities, trees or integrators).  Every generator
uses NumPy's PCG64 stream, so a (function, arguments, seed) triple gives the
same bytes on every machine.

The sets stand in for the paper's AGAMA Milky-Way model (Sec. 4.2: an NFW-like
dark halo with a thin exponential stellar and gas disk whose scale height is
about 10 % of its scale length) and for its 1 Msun supernova training cubes
(Sec. 3.3), neither of which is available.

Units
-----
* ``plummer`` / ``gas_sphere`` / ``lattice``: N-body units, G = M = 1.
* ``disk_galaxy``: kpc, km/s, Msun; G = 4.30091e-6 kpc (km/s)^2 / Msun.
* ``sn_cube``: pc, km/s, Msun; G unused (no self-gravity in cubes).

Every generator returns a dict of contiguous NumPy arrays (structure of
arrays): x, y, z, vx, vy, vz, m (float64), eps2 (float32, per-particle
squared softening), id (int64), type (uint8: 0 dark matter, 1 star, 2 gas),
and for gas u (float64, specific internal energy).  Gas particles always form
the contiguous tail of the arrays so that a gas-only view is an offset.
"""
from __future__ import annotations

import math

import numpy as np

G_KPC = 4.30091e-6          # kpc (km/s)^2 / Msun
G_PC = 4.30091e-3           # pc (km/s)^2 / Msun
KPC_TIME_GYR = 0.97779      # one kpc/(km/s) in Gyr
PC_TIME_MYR = 0.97779       # one pc/(km/s) in Myr
U_PER_K = 1.0 / 48.46       # (km/s)^2 per kelvin, gamma = 5/3, mu = 0.6
MSUN_PC3_PER_CM3 = 0.03459  # 1 hydrogen atom / cm^3 (rho = 1.4 m_H n) in Msun/pc^3
E_SN = 5.028e7              # 1e51 erg in Msun (km/s)^2

T_DM, T_STAR, T_GAS = 0, 1, 2


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _pack(x, y, z, vx, vy, vz, m, eps2, ptype, u=None, id0=0):
    n = len(x)
    out = {
        "x": np.ascontiguousarray(x, np.float64),
        "y": np.ascontiguousarray(y, np.float64),
        "z": np.ascontiguousarray(z, np.float64),
        "vx": np.ascontiguousarray(vx, np.float64),
        "vy": np.ascontiguousarray(vy, np.float64),
        "vz": np.ascontiguousarray(vz, np.float64),
        "m": np.ascontiguousarray(m, np.float64),
        "eps2": np.ascontiguousarray(eps2, np.float32),
        "id": np.arange(id0, id0 + n, dtype=np.int64),
        "type": np.ascontiguousarray(ptype, np.uint8),
    }
    if u is not None:
        out["u"] = np.ascontiguousarray(u, np.float64)
    return out


def _iso_dirs(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(1.0 - cz * cz)
    return s * np.cos(ph), s * np.sin(ph), cz


def plummer(n: int = 8192, seed: int = 1, eps_pair: float = 0.01):
    """Equal-mass Plummer sphere, G = M = a = 1.

    Radii from the inverse cumulative mass r = (X^(-2/3) - 1)^(-1/2); speeds
    q * v_esc(r) with q drawn by rejection from q^2 (1 - q^2)^(7/2) (the
    Aarseth-Henon-Wielen recipe); isotropic directions.  ``eps_pair`` is the
    softening of a pair, so each particle carries eps_i^2 = eps_pair^2 / 2.
    """
    rng = _rng(seed)
    X = rng.uniform(0.0, 1.0, n)
    X = np.clip(X, 1e-12, 1.0 - 1e-12)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    ux, uy, uz = _iso_dirs(rng, n)
    q = np.empty(n)
    filled = 0
    while filled < n:
        k = 2 * (n - filled) + 64
        q1 = rng.uniform(0.0, 1.0, k)
        q2 = rng.uniform(0.0, 0.1, k)
        ok = q1[q2 < q1 * q1 * (1.0 - q1 * q1) ** 3.5]
        take = min(len(ok), n - filled)
        q[filled:filled + take] = ok[:take]
        filled += take
    vesc = math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    v = q * vesc
    wx, wy, wz = _iso_dirs(rng, n)
    m = np.full(n, 1.0 / n)
    eps2 = np.full(n, eps_pair * eps_pair / 2.0)
    return _pack(r * ux, r * uy, r * uz, v * wx, v * wy, v * wz, m, eps2,
                 np.full(n, T_STAR))


def gas_sphere(n: int = 8192, seed: int = 2, sigma: float = 0.1, u: float = 1.0,
               eps: float = 0.01):
    """Uniform-density gas sphere of unit radius and unit mass.

    Positions uniform in the ball (r = U^(1/3), isotropic direction); each
    velocity component Gaussian with standard deviation ``sigma``; specific
    internal energy ``u`` everywhere.
    """
    rng = _rng(seed)
    r = rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    ux, uy, uz = _iso_dirs(rng, n)
    v = rng.normal(0.0, sigma, (3, n))
    m = np.full(n, 1.0 / n)
    return _pack(r * ux, r * uy, r * uz, v[0], v[1], v[2], m,
                 np.full(n, eps * eps / 2.0), np.full(n, T_GAS), u=np.full(n, u))


def lattice(nside: int = 24, spacing: float = 1.0, jitter: float = 0.0,
            seed: int = 7, u: float = 1.0, m: float = 1.0):
    """Simple cubic lattice of nside^3 gas particles at rest (optionally jittered)."""
    rng = _rng(seed)
    g = np.arange(nside, dtype=np.float64) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    n = x.size
    if jitter > 0.0:
        d = rng.uniform(-jitter, jitter, (3, n)) * spacing
        x, y, z = x + d[0], y + d[1], z + d[2]
    zero = np.zeros(n)
    return _pack(x, y, z, zero, zero, zero, np.full(n, m),
                 np.full(n, (0.1 * spacing) ** 2), np.full(n, T_GAS),
                 u=np.full(n, u))


def slab_and_sparse(n_slab: int = 12000, n_sparse: int = 24, seed: int = 11,
                    height: float = 0.5, thickness: float = 0.02, sigma: float = 0.05):
    """Dense gas slab with a few sparse particles above and below it.

    n_slab particles uniform in [0, 1]^2 x [-thickness/2, thickness/2];
    n_sparse particles uniform in [0, 1]^2 at z = +-height (half on each
    side).  The sparse particles' kernels reach into the slab, so the
    candidate lists of their groups cover most of it.  Equal masses,
    Gaussian velocities of standard deviation sigma, unit internal energy.
    """
    rng = _rng(seed)
    xs = rng.uniform(0.0, 1.0, (2, n_slab))
    zs = rng.uniform(-0.5 * thickness, 0.5 * thickness, n_slab)
    xp = rng.uniform(0.0, 1.0, (2, n_sparse))
    zp = np.where(np.arange(n_sparse) % 2 == 0, height, -height)
    x = np.concatenate([xs[0], xp[0]])
    y = np.concatenate([xs[1], xp[1]])
    z = np.concatenate([zs, zp])
    n = x.size
    v = rng.normal(0.0, sigma, (3, n))
    return _pack(x, y, z, v[0], v[1], v[2], np.full(n, 1.0 / n),
                 np.full(n, 1e-6), np.full(n, T_GAS), u=np.full(n, 1.0))


def _cyl_disk(rng, n, rd, zd, rmax):
    R = rng.gamma(2.0, rd, n)
    bad = R > rmax
    while bad.any():
        R[bad] = rng.gamma(2.0, rd, int(bad.sum()))
        bad = R > rmax
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    z = rng.exponential(zd, n) * np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0)
    return R, ph, z


def _nfw_radii(rng, n, rs, rcut):
    mu = lambda x: np.log1p(x) - x / (1.0 + x)
    xc = rcut / rs
    grid = np.concatenate([[0.0], np.geomspace(1e-6, xc, 20000)])
    cdf = mu(grid) / mu(xc)
    return np.interp(rng.uniform(0.0, 1.0, n), cdf, grid) * rs


def disk_galaxy(n_total: int = 1_000_000, seed: int = 3, frac_star: float = 0.5,
                frac_dm: float = 0.4, m_star: float = 5e10, m_dm: float = 1e12,
                m_gas: float = 1.1e10, rd_star: float = 2.6, zd_star: float = 0.3,
                rd_gas: float = 5.0, zd_gas: float = 0.15, rs_dm: float = 20.0,
                rcut_dm: float = 200.0, t_gas: float = 1e4):
    """Synthetic Milky-Way-like disk galaxy (kpc, km/s, Msun).

    Stars: exponential disk, R ~ Gamma(2, Rd) (surface density exp(-R/Rd)),
    |z| ~ Exp(zd); NFW halo with scale radius rs cut at rcut (inverse
    cumulative mass); gas: exponential disk at 1e4 K.  Disks are truncated at
    R <= 10 Rd.  Circular speed v_c = sqrt(G M(<r) / r) from the sampled,
    spherically averaged mass.  Stars rotate at v_c with isotropic Gaussian
    dispersion 0.1 v_c; halo particles are isotropic Gaussian with 1-D
    dispersion v_c/sqrt(3); gas rotates at v_c with no random motion.
    Softening: 0.05 kpc (stars, gas) and 0.15 kpc (halo) at one million
    particles, scaled as N^(-1/3).  Order: stars, halo, gas.
    """
    rng = _rng(seed)
    ns = int(round(n_total * frac_star))
    nd = int(round(n_total * frac_dm))
    ng = n_total - ns - nd
    Rs, phs, zs = _cyl_disk(rng, ns, rd_star, zd_star, 10.0 * rd_star)
    rd = _nfw_radii(rng, nd, rs_dm, rcut_dm)
    dx, dy, dz = _iso_dirs(rng, nd)
    Rg, phg, zg = _cyl_disk(rng, ng, rd_gas, zd_gas, 10.0 * rd_gas)

    x = np.concatenate([Rs * np.cos(phs), rd * dx, Rg * np.cos(phg)])
    y = np.concatenate([Rs * np.sin(phs), rd * dy, Rg * np.sin(phg)])
    z = np.concatenate([zs, rd * dz, zg])
    m = np.concatenate([np.full(ns, m_star / ns), np.full(nd, m_dm / nd),
                        np.full(ng, m_gas / ng)])
    r = np.sqrt(x * x + y * y + z * z)
    order = np.argsort(r, kind="stable")
    menc = np.empty(n_total)
    menc[order] = np.cumsum(m[order])
    vc = np.sqrt(G_KPC * menc / np.maximum(r, 1e-3))
    Rcyl = np.sqrt(x * x + y * y)
    ex = np.where(Rcyl > 0, -y / np.maximum(Rcyl, 1e-12), 0.0)
    ey = np.where(Rcyl > 0, x / np.maximum(Rcyl, 1e-12), 0.0)

    vx = np.zeros(n_total)
    vy = np.zeros(n_total)
    vz = np.zeros(n_total)
    s = slice(0, ns)
    g = rng.normal(0.0, 1.0, (3, ns)) * (0.1 * vc[s])
    vx[s] = vc[s] * ex[s] + g[0]
    vy[s] = vc[s] * ey[s] + g[1]
    vz[s] = g[2]
    d = slice(ns, ns + nd)
    g = rng.normal(0.0, 1.0, (3, nd)) * (vc[d] / math.sqrt(3.0))
    vx[d], vy[d], vz[d] = g[0], g[1], g[2]
    gs = slice(ns + nd, n_total)
    vx[gs] = vc[gs] * ex[gs]
    vy[gs] = vc[gs] * ey[gs]

    scale = (n_total / 1e6) ** (-1.0 / 3.0)
    e_star, e_dm = 0.05 * scale, 0.15 * scale
    eps = np.concatenate([np.full(ns, e_star), np.full(nd, e_dm), np.full(ng, e_star)])
    ptype = np.concatenate([np.full(ns, T_STAR), np.full(nd, T_DM), np.full(ng, T_GAS)])
    u = np.full(ng, t_gas * U_PER_K)
    out = _pack(x, y, z, vx, vy, vz, m, eps * eps, ptype)
    out["u_gas"] = u
    out["n_gas"] = ng
    out["gas_offset"] = ns + nd
    return out


def spatial_order(d: dict) -> dict:
    """Reorder the particle arrays of a ``disk_galaxy`` dict, in place, along
    a space-filling curve: the Morton order of a 1024^3 grid over the
    bounding box, separately for the collisionless block and the gas block
    (which stays last).  N-body codes keep their arrays in such an order; it
    is an input layout (ids travel with the particles) and takes no part in
    any tree: the library sorts by its own keys whatever the input order."""
    n, go = len(d["x"]), int(d["gas_offset"])
    q = []
    for c in ("x", "y", "z"):
        a = d[c]
        lo, hi = a.min(), a.max()
        v = np.clip(((a - lo) * (1024.0 / max(hi - lo, 1e-300))).astype(np.int64), 0, 1023)
        w = np.zeros(n, np.int64)
        for b in range(10):  # spread the 10 bits three apart
            w |= ((v >> b) & 1) << (3 * b)
        q.append(w)
    key = (q[0] << 2) | (q[1] << 1) | q[2]
    idx = np.concatenate([np.argsort(key[:go], kind="stable"),
                          go + np.argsort(key[go:], kind="stable")])
    for k, v in list(d.items()):
        if isinstance(v, np.ndarray) and len(v) == n:
            d[k] = v[idx]
    d["u_gas"] = d["u_gas"][idx[go:] - go]
    return d


def gas_view(p: dict) -> dict:
    """Gas-only slice (contiguous tail) of a ``disk_galaxy`` dict."""
    o = int(p["gas_offset"])
    v = {k: p[k][o:] for k in ("x", "y", "z", "vx", "vy", "vz", "m", "eps2", "id", "type")}
    v["u"] = p["u_gas"]
    return v


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices in [0, n), sorted, drawn with PCG64."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def _kolmogorov_field(rng, ngrid, slope, rms3d):
    """Three independent Gaussian random velocity components on an ngrid^3
    periodic grid with power |v_k|^2 ~ k^slope (slope = -11/3 for Kolmogorov),
    scaled to a 3-D rms of rms3d."""
    k = np.fft.fftfreq(ngrid) * ngrid
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (slope / 2.0)
    comps = []
    for _ in range(3):
        noise = rng.normal(size=(ngrid, ngrid, ngrid)) + 1j * rng.normal(size=(ngrid, ngrid, ngrid))
        comps.append(np.real(np.fft.ifftn(noise * amp)))
    v = np.stack(comps)
    v *= rms3d / np.sqrt(np.mean(np.sum(v * v, axis=0)))
    return v


def _trilinear(field, pos, side):
    """Periodic trilinear interpolation of field[c, n, n, n] (cell-centred on a
    cube of the given side starting at 0) at pos[3, m]."""
    n = field.shape[1]
    g = pos / side * n - 0.5
    i0 = np.floor(g).astype(np.int64)
    f = g - i0
    out = np.zeros((field.shape[0], pos.shape[1]))
    for dx in (0, 1):
        wx = f[0] if dx else 1 - f[0]
        for dy in (0, 1):
            wy = f[1] if dy else 1 - f[1]
            for dz in (0, 1):
                wz = f[2] if dz else 1 - f[2]
                ix = (i0[0] + dx) % n
                iy = (i0[1] + dy) % n
                iz = (i0[2] + dz) % n
                out += field[:, ix, iy, iz] * (wx * wy * wz)
    return out


def sn_cube(seed: int, n_min: int = 2000, n_max: int = 32000, side: float = 60.0,
            t_min: float = 100.0, t_max: float = 1e4, m_part: float = 1.0,
            turb_rms: float = 5.0, turb_slope: float = -11.0 / 3.0, n_fixed: int = None):
    """Gas cube around a supernova site (pc, km/s, Msun), centred on the origin.

    N log-uniform in [n_min, n_max] (unless n_fixed), particle mass m_part, so
    the number density follows from N (1 Msun in a (60 pc)^3 cube: n = N/7471
    cm^-3).  Positions Poisson-uniform in the cube; temperature log-uniform in
    [t_min, t_max], uniform across the cube; velocities from a Kolmogorov
    Gaussian random field (64^3, 3-D rms turb_rms) interpolated trilinearly.
    The explosion itself is not applied here.
    """
    rng = _rng(seed)
    if n_fixed is None:
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
    else:
        n = int(n_fixed)
    T = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
    pos = rng.uniform(0.0, side, (3, n))
    vel = _trilinear(_kolmogorov_field(rng, 64, turb_slope, turb_rms), pos, side)
    pos -= side / 2.0
    m = np.full(n, m_part)
    out = _pack(pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], m,
                np.full(n, 0.01, np.float32), np.full(n, T_GAS), u=np.full(n, T * U_PER_K))
    out["T"] = T
    out["n_cm3"] = n * m_part / side ** 3 / MSUN_PC3_PER_CM3
    return out


def sn_cube_n(seed: int, n_min: int = 2000, n_max: int = 32000) -> int:
    """Particle count sn_cube(seed) will draw (its first random number)."""
    rng = _rng(seed)
    return int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))


def sn_batch(seeds, spacing: float = 1000.0, **kw):
    """Several SN cubes in one particle set, cube k centred at a point of a
    cubic lattice of the given spacing (far enough apart that they never
    interact).  Returns the packed set plus per-particle cube ids, per-cube
    offsets [K+1] and centres [K, 3]."""
    cubes = [sn_cube(s, **kw) for s in seeds]
    K = len(cubes)
    g = int(math.ceil(K ** (1.0 / 3.0)))
    centres = np.array([((k % g), (k // g) % g, k // (g * g)) for k in range(K)],
                       dtype=np.float64) * spacing
    parts = {k: [] for k in ("x", "y", "z", "vx", "vy", "vz", "m", "eps2", "u")}
    cube_id = []
    for k, c in enumerate(cubes):
        for a, d in zip(("x", "y", "z"), range(3)):
            parts[a].append(c[a] + centres[k, d])
        for a in ("vx", "vy", "vz", "m", "eps2", "u"):
            parts[a].append(c[a])
        cube_id.append(np.full(c["x"].size, k, np.int32))
    out = _pack(*(np.concatenate(parts[a]) for a in ("x", "y", "z", "vx", "vy", "vz", "m")),
                np.concatenate(parts["eps2"]), np.full(sum(c["x"].size for c in cubes), T_GAS),
                u=np.concatenate(parts["u"]))
    out["cube_id"] = np.concatenate(cube_id)
    out["offsets"] = np.concatenate([[0], np.cumsum([c["x"].size for c in cubes])]).astype(np.int64)
    out["centres"] = centres
    out["T_amb"] = np.array([c["T"] for c in cubes])
    out["n_cm3"] = np.array([c["n_cm3"] for c in cubes])
    return out
