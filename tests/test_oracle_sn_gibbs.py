"""Pins of the oracle's Gibbs resampler and eight-cube encoding (Sec. 3.3)
against what the definitions fix: hand-computed line draws (including the
boundary rule), one sweep over a product density giving exact draws of each
marginal whatever the start, invariance of the target density under a sweep
of a non-separable density, convergence from a single start voxel, and the
encoding's values, symmetry and inverse."""
import math

import numpy as np
from scipy import stats

from oracle import sn as osn


def _chi2_p(obs, expect):
    keep = expect >= 5          # chi-square validity; the rest pooled
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(expect[keep], expect[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    return stats.chisquare(o, e * o.sum() / e.sum())[1]


def _voxels(out, grid, side=60.0):
    dv = side / grid
    X = np.floor((out["x"] + side / 2) / dv).astype(int)
    Y = np.floor((out["y"] + side / 2) / dv).astype(int)
    Z = np.floor((out["z"] + side / 2) / dv).astype(int)
    return X, Y, Z


def _pred_from_rho(rho):
    """[1, grid^3, 5] physical channels with log10 rho from rho[z, y, x]."""
    g = rho.shape[0]
    p = np.zeros((1, g ** 3, 5))
    p[0, :, 0] = np.log10(rho.reshape(-1))
    p[0, :, 1] = 3.0
    return p


def test_line_draw_by_hand():
    w = [1.0, 2.0, 3.0, 4.0]           # prefix sums 1, 3, 6, 10
    assert [osn.line_draw(w, u) for u in (0.0, 0.0625, 0.25, 0.5, 0.625, 0.96875)] == \
        [0, 0, 1, 2, 3, 3]
    # a target equal to a prefix sum goes to the next index
    assert osn.line_draw([1.0] * 4, 0.25) == 1 and osn.line_draw([1.0] * 4, 0.75) == 3
    # empty voxels are never drawn
    assert [osn.line_draw([0.0, 0.0, 5.0, 0.0], u) for u in (0.0, 0.5, 0.99)] == [2, 2, 2]


def test_one_sweep_over_a_product_density_draws_each_marginal_exactly():
    # rho = f(x) g(y) h(z): every line conditional is a marginal, so one sweep
    # gives exact draws whatever the start; a line read along the wrong axis
    # would give the wrong marginal
    grid, n = 6, 60_000
    f = np.array([1.0, 2.0, 4.0, 8.0, 16.0, 32.0])
    g = np.array([5.0, 1.0, 1.0, 1.0, 1.0, 5.0])
    h = np.array([1.0, 3.0, 9.0, 3.0, 1.0, 0.5])
    rho = h[:, None, None] * g[None, :, None] * f[None, None, :]
    pred = _pred_from_rho(rho)
    rng = np.random.default_rng(21)
    uni = rng.uniform(0, 1, (n, 6))
    start_a = rng.uniform(-30, 30, (n, 3))
    start_b = np.full((n, 3), -29.0)                # every chain in voxel (0, 0, 0)
    out_a = osn.resample_gibbs(pred, np.zeros((1, 3)), grid, 60.0, [n], start_a, 1, uni, 1.0)
    out_b = osn.resample_gibbs(pred, np.zeros((1, 3)), grid, 60.0, [n], start_b, 1, uni, 1.0)
    assert out_a["x"].size == n
    # the same uniforms give the same voxel from any start (up to the rounding
    # of the line sums, which scale with the other two factors)
    assert np.mean(out_a["voxel"] == out_b["voxel"]) > 0.999
    X, Y, Z = _voxels(out_a, grid)
    for I, m in ((X, f), (Y, g), (Z, h)):
        assert _chi2_p(np.bincount(I, minlength=grid), n * m / m.sum()) > 0.01
    assert _chi2_p(np.bincount(out_a["voxel"], minlength=grid ** 3),
                   n * rho.reshape(-1) / rho.sum()) > 0.01
    # the x marginal is not the z marginal: a transposed line would fail
    assert _chi2_p(np.bincount(X, minlength=grid), n * h / h.sum()) < 1e-6


def _ridge(grid):
    i = np.arange(grid)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    return np.exp(-((X - Y) ** 2 + (Y - Z) ** 2) / 2.0) + 0.02


def test_a_sweep_leaves_the_target_density_invariant():
    # chains started from exact draws of rho are still distributed as rho
    # after one sweep (non-separable ridge along the diagonal)
    grid, n = 5, 40_000
    rho = _ridge(grid)
    pred = _pred_from_rho(rho)
    rng = np.random.default_rng(22)
    p = rho.reshape(-1) / rho.sum()
    v0 = rng.choice(grid ** 3, size=n, p=p)
    dv = 60.0 / grid
    X0, Y0, Z0 = v0 % grid, (v0 // grid) % grid, v0 // (grid * grid)
    start = np.stack([X0, Y0, Z0], 1) * dv - 30.0 + rng.uniform(0, dv, (n, 3))
    uni = rng.uniform(0, 1, (n, 6))
    out = osn.resample_gibbs(pred, np.zeros((1, 3)), grid, 60.0, [n], start, 1, uni, 1.0)
    assert _chi2_p(np.bincount(out["voxel"], minlength=grid ** 3), n * p) > 0.01
    # a chain that drew y from the line through the old x would not keep it:
    # the same test rejects draws from the product of the marginals
    mx = rho.sum(axis=(0, 1)); my = rho.sum(axis=(0, 2)); mz = rho.sum(axis=(1, 2))
    prod = (mz[:, None, None] * my[None, :, None] * mx[None, None, :]).reshape(-1)
    vp = rng.choice(grid ** 3, size=n, p=prod / prod.sum())
    assert _chi2_p(np.bincount(vp, minlength=grid ** 3), n * p) < 1e-6


def test_chains_from_one_voxel_converge_and_zero_sweeps_stay():
    grid, n = 4, 20_000
    rho = _ridge(grid)
    pred = _pred_from_rho(rho)
    rng = np.random.default_rng(23)
    start = np.tile([[-29.0, 29.0, -29.0]], (n, 1))       # voxel (0, 3, 0): off the ridge
    sweeps = 30
    uni = rng.uniform(0, 1, (n, 3 * sweeps + 3))
    out = osn.resample_gibbs(pred, np.zeros((1, 3)), grid, 60.0, [n], start, sweeps, uni, 1.0)
    p = rho.reshape(-1) / rho.sum()
    assert _chi2_p(np.bincount(out["voxel"], minlength=grid ** 3), n * p) > 0.01
    out0 = osn.resample_gibbs(pred, np.zeros((1, 3)), grid, 60.0, [n], start, 0, uni[:, :3], 1.0)
    assert np.all(out0["voxel"] == (0 * grid + 3) * grid + 0)


def test_gibbs_outputs_counts_voxel_values_and_subsets():
    rng = np.random.default_rng(24)
    grid, K = 6, 3
    pred = np.zeros((K, grid ** 3, 5))
    pred[..., 0] = rng.normal(size=(K, grid ** 3)) - 1.0
    pred[..., 1] = rng.uniform(2.0, 6.0, (K, grid ** 3))
    pred[..., 2:] = rng.normal(size=(K, grid ** 3, 3))
    counts = np.array([50, 0, 70])
    centers = np.array([[0.0, 0.0, 0.0], [500.0, 0.0, 0.0], [0.0, 100.0, -40.0]])
    cc = np.repeat(centers, counts, axis=0)
    start = cc + rng.uniform(-35, 35, (counts.sum(), 3))   # some outside: clamped
    sweeps = 3
    uni = rng.uniform(0, 1, (counts.sum(), 3 * sweeps + 3))
    out = osn.resample_gibbs(pred, centers, grid, 60.0, counts, start, sweeps, uni, 0.25)
    assert out["x"].size == counts.sum()                   # N_out = N_in
    v = out["voxel"]
    cube = np.repeat(np.arange(K), counts)
    dv = 60.0 / grid
    X, Y, Z = v % grid, (v // grid) % grid, v // (grid * grid)
    for a, I in ((0, X), (1, Y), (2, Z)):
        pos = out["xyz"[a]] - (cc[:, a] - 30.0)
        assert np.all(pos >= I * dv - 1e-12) and np.all(pos < (I + 1) * dv + 1e-12)
        # the in-voxel offset is the last uniforms'
        assert np.allclose(pos - I * dv, uni[:, 3 * sweeps + a] * dv, atol=1e-12)
    assert np.allclose(out["u"], 10.0 ** pred[cube, v, 1] * 0.25, rtol=1e-14)
    assert np.array_equal(out["vy"], pred[cube, v, 3])
    sel = np.array([0, 49, 50, 119, 7])
    sub = osn.resample_gibbs(pred, centers, grid, 60.0, counts, start, sweeps, uni, 0.25, sel=sel)
    for k in ("x", "y", "z", "vx", "u", "voxel"):
        assert np.array_equal(sub[k], out[k][sel])


def test_encode8_by_hand_symmetry_and_inverse():
    phys = np.array([[-1.5, 3.25, 3.0, -9.0, 0.0]])
    e = osn.encode8(phys, 1.0)
    assert e.shape == (1, 8)
    assert e[0, :2].tolist() == [-1.5, 3.25]
    assert e[0, 2] == math.log10(4.0) and e[0, 3] == 0.0       # vx = +3
    assert e[0, 4] == 0.0 and e[0, 5] == 1.0                   # vy = -9
    assert e[0, 6] == 0.0 and e[0, 7] == 0.0                   # vz = 0
    rng = np.random.default_rng(25)
    p = rng.normal(size=(200, 5)) * [1, 1, 300, 30, 3]
    e = osn.encode8(p, 2.0)
    # a sign change of a component swaps its two cubes
    q = p.copy()
    q[:, 3] = -q[:, 3]
    eq = osn.encode8(q, 2.0)
    assert np.array_equal(eq[:, 4], e[:, 5]) and np.array_equal(eq[:, 5], e[:, 4])
    assert np.array_equal(eq[:, [0, 1, 2, 3, 6, 7]], e[:, [0, 1, 2, 3, 6, 7]])
    # one cube of each pair holds log10(v0): the other carries the magnitude
    for a in range(3):
        assert np.all(np.minimum(e[:, 2 + 2 * a], e[:, 3 + 2 * a]) == math.log10(2.0))
    d = osn.decode8(e)
    assert np.allclose(d, p, rtol=1e-12, atol=1e-12)
