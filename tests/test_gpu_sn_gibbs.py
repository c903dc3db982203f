"""GPU parity (through the C ABI) of the eight-cube encoding and the Gibbs
resampler against the oracle: element-wise on small cubes (ragged and empty
cubes, starts outside the box, zero sweeps) and on sampled particles of a
production-size call (64 cubes of 64^3 voxels)."""
import numpy as np
import pytest

from oracle import sn as osn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng(gx):
    e = gx.Engine(0)
    yield e
    e.close()


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _f32_ulps(got, ref):
    """Distance in FP32 units of the reference's magnitude."""
    r32 = np.abs(ref).astype(np.float32)
    return np.abs(got.astype(np.float64) - ref) / np.spacing(np.maximum(r32, np.float32(1e-30)))


@pytest.mark.parametrize("stride", [5, 7])
def test_encode8_decode8_match_oracle(gx, eng, stride):
    import torch
    rng = np.random.default_rng(41)
    V = 100_003
    phys = np.zeros((V, stride), np.float32)
    phys[:, 0] = rng.normal(size=V) - 1.0
    phys[:, 1] = rng.uniform(1.0, 7.0, V)
    mag = 10.0 ** rng.uniform(-3, 3.5, (V, 3))
    sign = rng.choice([-1.0, 0.0, 1.0], size=(V, 3), p=[0.45, 0.1, 0.45])
    phys[:, 2:5] = (mag * sign).astype(np.float32)
    v0 = 1.0
    out8 = torch.zeros(V * 8, dtype=torch.float32, device="cuda")
    eng.sn_encode8(_t(phys), V, v0, out8, in_stride=stride)
    got = out8.cpu().numpy().reshape(V, 8)
    ref = osn.encode8(phys[:, :5].astype(np.float64), v0)
    assert np.array_equal(got[:, :2], phys[:, :2])
    assert np.max(_f32_ulps(got[:, 2:], ref[:, 2:])) <= 1.0
    # decode of the FP32 encoding against the oracle's decode of the same values
    out5 = torch.zeros(V * 5, dtype=torch.float32, device="cuda")
    eng.sn_decode8(out8, V, out5)
    dec = out5.cpu().numpy().reshape(V, 5)
    rd = osn.decode8(got.astype(np.float64))
    assert np.array_equal(dec[:, :2], phys[:, :2])
    big = 10.0 ** got[:, 2::2].astype(np.float64) + 10.0 ** got[:, 3::2].astype(np.float64)
    err = np.abs(dec[:, 2:].astype(np.float64) - rd[:, 2:])
    assert np.all(err <= np.spacing(np.abs(rd[:, 2:]).astype(np.float32)) + 1e-14 * big)
    # and back to the physical velocities within the FP32 rounding of the logarithms
    assert np.allclose(dec[:, 2:], phys[:, 2:5], rtol=2e-6, atol=2e-6 * v0)


def _pred(rng, K, grid):
    p = np.zeros((K, grid ** 3, 5), np.float32)
    i = (np.arange(grid) + 0.5) / grid - 0.5
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z).reshape(-1)
    for c in range(K):
        # a shell at a random radius over a noisy background, as a blast leaves
        r0 = rng.uniform(0.15, 0.4)
        p[c, :, 0] = (-1.5 + 2.0 * np.exp(-((r - r0) / 0.04) ** 2)
                      + 0.3 * rng.normal(size=grid ** 3))
        p[c, :, 1] = rng.uniform(2, 7, grid ** 3)
        p[c, :, 2:] = rng.normal(size=(grid ** 3, 3)) * 50
    return p


def _run(eng, pred, centers, grid, counts, start, sweeps, uni, T_to_u):
    import torch
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    tot = int(off[-1])
    outs = [torch.zeros(max(tot, 1), dtype=torch.float64, device="cuda") for _ in range(7)]
    eng.sn_resample_gibbs(_t(pred), _t(centers), grid, 60.0, _t(off), int(max(counts.max(), 0)),
                          _t(start[:, 0]), _t(start[:, 1]), _t(start[:, 2]), sweeps,
                          _t(uni.reshape(-1)), T_to_u, *outs)
    return dict(zip(("x", "y", "z", "vx", "vy", "vz", "u"), (o.cpu().numpy()[:tot] for o in outs)))


def _voxel(got, centers, counts, grid):
    dv = 60.0 / grid
    cc = np.repeat(centers, counts, axis=0)
    v = [np.floor((got[a] - (cc[:, k] - 30.0)) / dv).astype(int) for k, a in enumerate("xyz")]
    return (v[2] * grid + v[1]) * grid + v[0]


def _compare(got, ref, sel, centers, counts, grid):
    vg = _voxel(got, centers, counts, grid)[sel]
    ok = vg == ref["voxel"]
    # a decision can differ only where a uniform lands on a line sum that the
    # two sides' 10^x round apart (last bit of FP64): essentially never
    assert ok.mean() >= 0.999, ok.mean()
    for a in ("x", "y", "z"):
        assert np.allclose(got[a][sel][ok], ref[a][ok], rtol=0, atol=1e-12)
    for a in ("vx", "vy", "vz"):
        assert np.array_equal(got[a][sel][ok], ref[a][ok])
    assert np.allclose(got["u"][sel][ok], ref["u"][ok], rtol=1e-12)
    return ok.mean()


@pytest.mark.parametrize("sweeps", [0, 1, 3])
def test_gibbs_matches_oracle(gx, eng, sweeps):
    rng = np.random.default_rng(42 + sweeps)
    grid, K = 16, 3
    pred = _pred(rng, K, grid)
    counts = np.array([4000, 0, 7001])
    centers = np.array([[0.0, 0, 0], [100.0, 0, 0], [0, 100.0, -50.0]])
    cc = np.repeat(centers, counts, axis=0)
    start = cc + rng.uniform(-33, 33, (counts.sum(), 3))      # some outside: clamped
    uni = rng.uniform(0, 1, (counts.sum(), 3 * sweeps + 3)).astype(np.float32)
    got = _run(eng, pred, centers, grid, counts, start, sweeps, uni, 1 / 48.46)
    ref = osn.resample_gibbs(pred.astype(np.float64), centers, grid, 60.0, counts, start, sweeps,
                             uni.astype(np.float64), 1 / 48.46)
    sel = np.arange(counts.sum())
    frac = _compare(got, ref, sel, centers, counts, grid)
    if sweeps == 0:
        assert frac == 1.0


def test_gibbs_production_size_sampled(gx, eng):
    # 64 cubes of 64^3 voxels, ~5,000 particles each, 4 sweeps; the oracle
    # follows 3,000 sampled chains one by one
    rng = np.random.default_rng(43)
    grid, K, sweeps = 64, 64, 4
    pred = _pred(rng, K, grid)
    counts = rng.integers(2000, 8000, K)
    centers = np.stack([np.arange(K) * 1000.0, np.zeros(K), np.zeros(K)], 1)
    cc = np.repeat(centers, counts, axis=0)
    start = cc + rng.uniform(-30, 30, (counts.sum(), 3))
    uni = rng.uniform(0, 1, (counts.sum(), 3 * sweeps + 3)).astype(np.float32)
    got = _run(eng, pred, centers, grid, counts, start, sweeps, uni, 1.0)
    sel = np.sort(rng.choice(counts.sum(), 3000, replace=False))
    ref = osn.resample_gibbs(pred.astype(np.float64), centers, grid, 60.0, counts, start, sweeps,
                             uni.astype(np.float64), 1.0, sel=sel)
    _compare(got, ref, sel, centers, counts, grid)


def test_surrogate_eight_cube_inputs_and_outputs(gx, eng):
    # inputs: the voxelized physical channels, encoded and standardized, in
    # BF16; outputs: the head's eight channels mapped back by the target
    # statistics and decoded to the physical ones
    import torch
    import ics
    from paper_2510_23330_amd.sn import SNBatch, Surrogate, SIDE, U_PER_K, V0_KMS
    grid, K = 16, 2
    sb = SNBatch(eng, ics.sn_batch([1000, 1001]))
    sb.inject()
    phys = sb.voxelize(grid=grid)                       # [K * V * 5] physical
    sur = Surrogate(eng, batch=2, base=16, levels=2, grid=grid, seed=3, encoding="8cube")
    V = grid ** 3
    si = torch.zeros(16, dtype=torch.float64, device="cuda")
    sur.channel_sums(phys.view(K, V * 5), si)
    sp = torch.zeros(10, dtype=torch.float64, device="cuda")
    eng.chan_stats(phys, 5, 5, sp)
    sur.set_stats(si, si, K * V, sums_phys=sp)
    P = phys.cpu().numpy().reshape(K * V, 5).astype(np.float64)
    enc = osn.encode8(P, V0_KMS)
    mean = enc.mean(axis=0)
    std = enc.std(axis=0)
    assert np.allclose(sur.mean_in.cpu().numpy(), mean, rtol=1e-5, atol=1e-6)
    assert np.allclose(sur.std_in.cpu().numpy(), np.maximum(std, 1e-3), rtol=1e-4)
    assert np.allclose(sur.mean_phys.cpu().numpy(), P.mean(axis=0), rtol=1e-5, atol=1e-5)
    amb = sb.ambient()
    xin = sur.inputs(sb.p, sb.g, sb.centers, SIDE, amb, K)
    got = xin.float().cpu().numpy().reshape(K * V, 8)
    ref = (enc - sur.mean_in.cpu().numpy()) / sur.std_in.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5)
    out = torch.empty(K * V * 5, dtype=torch.float32, device="cuda")
    sur.infer(xin, K, out)
    raw = sur.net.forward(xin).cpu().numpy().reshape(K * V, 16)[:, :8].astype(np.float64)
    c = raw * sur.std_out.cpu().numpy() + sur.mean_out.cpu().numpy()
    ref5 = osn.decode8(c)
    g5 = out.cpu().numpy().reshape(K * V, 5).astype(np.float64)
    assert np.allclose(g5[:, :2], ref5[:, :2], rtol=1e-6, atol=1e-6)
    mag = 10.0 ** c[:, 2::2] + 10.0 ** c[:, 3::2]
    assert np.all(np.abs(g5[:, 2:] - ref5[:, 2:]) <= 1e-5 * mag + 1e-6)
