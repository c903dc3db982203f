"""Pins of the oracle's supernova-region steps (Sec. 3.2 steps 2 and 4, the
grid-to-particle mapping of Sec. 3.3) against properties their definitions
fix: boxes that tile space partition the particles, the injected energy and
the nearest-first selection, the ambient state of a hand-computed box, and
for the resampler the particle count, the mass, the stratified inverse-CDF
counts and a chi-square test of the drawn positions against rho_v."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sn as osn


def test_extract_boxes_that_tile_space_partition_the_particles():
    h = 4.0
    g = np.array([-2.0, 0.0, 2.0]) * h       # 3^3 boxes of side 2h tiling [-3h, 3h)^3
    centers = np.array([(a, b, c) for a in g for b in g for c in g])
    rng = np.random.default_rng(1)
    pts = rng.uniform(-3.5 * h, 3.5 * h, (3, 4000))
    # particles exactly on inner faces and on the outer faces of the tiling
    face = np.array([-h, h, -3 * h, 3 * h, 0.5])
    pts[:, :len(face)] = face[None, :]
    pts[0, 10:20] = -h
    x, y, z = pts
    off, idx = osn.extract(x, y, z, centers, h)
    counts = np.bincount(idx, minlength=x.size)
    inside = np.all((pts >= -3 * h) & (pts < 3 * h), axis=0)
    assert np.array_equal(counts, inside.astype(np.int64))
    # members ascend within each box
    for c in range(len(centers)):
        assert np.all(np.diff(idx[off[c]:off[c + 1]]) > 0)
    # a point on a shared face belongs to the box above it (half-open boxes)
    k = int(np.nonzero(idx == 0)[0][0])
    c = int(np.searchsorted(off, k, side="right") - 1)
    assert np.all(centers[c] - h == -h)


def test_inject_energy_and_nearest_selection_with_ties():
    rng = np.random.default_rng(2)
    n = 500
    x, y, z = rng.uniform(-10, 10, (3, n))
    m = rng.uniform(0.5, 2.0, n)
    # plant exact distance ties around the centre: six points at distance 1
    for j, (a, b, c) in enumerate([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1),
                                   (0, 0, -1)]):
        x[100 + j], y[100 + j], z[100 + j] = a, b, c
    x[:5], y[:5], z[:5] = 0.1, 0.1, 0.1            # five coincident points nearest
    off, idx = osn.extract(x, y, z, np.zeros((1, 3)), 10.0)
    u0 = rng.uniform(1, 2, n)
    E = 5.0e7
    k_inj = 8                                        # 5 nearest + 3 of the 6 tied points
    u1 = osn.inject(x, y, z, m, off, idx, np.zeros((1, 3)), k_inj, E, u0)
    du = u1 - u0
    sel = np.nonzero(du)[0]
    assert sel.size == k_inj
    assert np.sum(m * du) == pytest.approx(E, rel=1e-13)
    assert np.allclose(du[sel], du[sel[0]], rtol=1e-15)        # one specific energy
    d2 = x * x + y * y + z * z
    rest = np.setdiff1d(idx, sel)
    assert d2[sel].max() <= d2[rest].min()
    # ties broken by index: the three lowest-index points of the tied six
    assert set(sel.tolist()) == {0, 1, 2, 3, 4, 100, 101, 102}


def test_ambient_by_hand():
    m = np.array([1.0, 3.0, 5.0])
    u = np.array([2.0, 4.0, 7.0])
    v = np.array([[1.0, -1.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 9.0]])
    off = np.array([0, 2, 2])
    idx = np.array([0, 1])
    a = osn.ambient(m, u, v[0], v[1], v[2], off, idx, 2.0, 10.0)
    # box 0: mass 4 in volume 8; T = (2 + 12) / 4 * 10 = 35; v = (1 - 3, 0 + 6) / 4
    assert a[0, 0] == pytest.approx(math.log10(0.5), abs=1e-15)
    assert a[0, 1] == pytest.approx(math.log10(35.0), abs=1e-15)
    assert a[0, 2] == pytest.approx(-0.5) and a[0, 3] == pytest.approx(1.5) and a[0, 4] == 0.0
    # empty box
    assert a[1].tolist() == [-30.0, 1.0, 0.0, 0.0, 0.0]
    # temperature floor
    b = osn.ambient(m, u * 1e-3, v[0], v[1], v[2], off, idx, 2.0, 10.0)
    assert b[0, 1] == 1.0


def _pred(rng, K, grid):
    p = np.zeros((K, grid ** 3, 5))
    p[..., 0] = rng.normal(size=(K, grid ** 3)) * 0.8 - 1.0
    p[..., 1] = rng.uniform(2.0, 6.0, (K, grid ** 3))
    p[..., 2:] = rng.normal(size=(K, grid ** 3, 3))
    return p


def test_resample_count_mass_and_stratified_inverse_cdf():
    # stratified uniforms u0 = (j + 1/2) / N hit voxel v exactly
    # floor(N C_v / C) - floor(N C_{v-1} / C) times, i.e. N p_v within one.
    rng = np.random.default_rng(5)
    grid, K = 6, 2
    pred = _pred(rng, K, grid)
    counts = np.array([3000, 1])
    uni = rng.uniform(0, 1, (int(counts.sum()), 4))
    uni[:3000, 0] = (np.arange(3000) + 0.5) / 3000
    centers = np.array([[0.0, 0.0, 0.0], [100.0, 50.0, 0.0]])
    out = osn.resample(pred, centers, grid, 60.0, counts, uni, 0.5)
    assert out["x"].size == counts.sum()                      # N_out = N_in
    w = 10.0 ** pred[0, :, 0]
    p = w / w.sum()
    got = np.bincount(out["voxel"][:3000], minlength=grid ** 3)
    assert np.all(np.abs(got - 3000 * p) <= 1.0 + 1e-9)
    # positions inside their voxel; T and v of that voxel
    dv = 60.0 / grid
    v = out["voxel"]
    X, Y, Z = v % grid, (v // grid) % grid, v // (grid * grid)
    cc = np.repeat(centers, counts, axis=0)
    for a, I in ((0, X), (1, Y), (2, Z)):
        pos = out["xyz"[a]] - (cc[:, a] - 30.0)
        assert np.all(pos >= I * dv - 1e-12) and np.all(pos < (I + 1) * dv + 1e-12)
    cube = np.repeat(np.arange(K), counts)
    assert np.allclose(out["u"], 10.0 ** pred[cube, v, 1] * 0.5, rtol=1e-14)
    assert np.array_equal(out["vz"], pred[cube, v, 4])
    # masses: the replaced particles keep theirs, so the region's mass is exact
    ids = np.arange(10, 3011)
    m = rng.uniform(0.5, 1.5, ids.size)
    fields = {"m": m, "x": np.zeros(ids.size)}
    new, missing = osn.replace(ids, fields, ids[:3000][::-1], {"x": out["x"][:3000]})
    assert missing == 0 and np.sum(new["m"]) == np.sum(m)


def test_resample_positions_chi_square_against_rho():
    rng = np.random.default_rng(6)
    grid = 8
    pred = _pred(rng, 1, grid)
    n = 200_000
    uni = rng.uniform(0, 1, (n, 4))
    out = osn.resample(pred, np.zeros((1, 3)), grid, 60.0, np.array([n]), uni, 1.0)
    dv = 60.0 / grid
    X = np.floor((out["x"] + 30.0) / dv).astype(int)
    Y = np.floor((out["y"] + 30.0) / dv).astype(int)
    Z = np.floor((out["z"] + 30.0) / dv).astype(int)
    hist = np.bincount((Z * grid + Y) * grid + X, minlength=grid ** 3)
    w = 10.0 ** pred[0, :, 0]
    expect = n * w / w.sum()
    keep = expect >= 5       # chi-square validity; the rest pooled
    obs = np.append(hist[keep], hist[~keep].sum())
    exp = np.append(expect[keep], expect[~keep].sum())
    chi2, pval = stats.chisquare(obs, exp)
    assert pval > 0.01
    # a uniform (density-blind) draw fails the same test
    U = rng.integers(0, grid ** 3, n)
    hu = np.bincount(U, minlength=grid ** 3)
    assert stats.chisquare(np.append(hu[keep], hu[~keep].sum()), exp)[1] < 1e-6


def test_check_and_replace_definitions():
    grid, K = 3, 4
    lo = np.array([-1.0, 0.0, -2.0, -3.0, 1.0])
    hi = np.array([1.0, 5.0, 2.0, 3.0, 2.0])
    rng = np.random.default_rng(7)
    v = rng.uniform(lo, hi, size=(K, grid ** 3, 5)).astype(np.float32)
    v[1, 3, 1] = 5.0 * 1.001
    v[2, 0, 0] = np.nan
    v[3, 5, 4] = np.float32(2.0)     # on the bound
    assert osn.check(v, lo, hi).tolist() == [True, False, False, True]
    ids = np.array([7, 3, 9, 1])
    f = {"x": np.array([0.0, 1.0, 2.0, 3.0])}
    new, missing = osn.replace(ids, f, np.array([9, 5, 9, 7]), {"x": np.array([10.0, 11.0, 12.0, 13.0])})
    # id 9 twice: the later entry wins; id 5 is missing
    assert new["x"].tolist() == [13.0, 1.0, 12.0, 3.0] and missing == 1
