"""GPU parity of the BF16-MFMA convolution blocks, the U-Net composition and
Adam against the FP64 oracle (through the C ABI).

Tolerances: both sides see the same BF16-rounded operands.  The GPU sums
products in FP32 (relative error ~ sqrt(K) 6e-8 for K = 27 Cin terms, < 1e-5)
and rounds BF16 outputs (2^-9 relative); so conv outputs agree to
2^-8 |y| + 1e-4 rms(y).  Through the whole network the BF16 storage of every
activation and gradient is mirrored by the oracle (``rb``); remaining
differences are rounding-boundary flips, bounded in norm by 2e-2.
"""
import numpy as np
import pytest

import oracle
from oracle import unet as ounet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng(gx):
    e = gx.Engine(0)
    yield e
    e.close()


def _bf(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float32).ravel(), device="cuda").to(torch.bfloat16)


def _np(t):
    import torch
    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else t.cpu().numpy().astype(np.float64)


def _close(got, ref, rel=2 ** -8, rms_frac=1e-4):
    rms = np.sqrt(np.mean(ref ** 2)) + 1e-30
    return np.all(np.abs(got - ref) <= rel * np.abs(ref) + rms_frac * rms)


# 3^3 shapes cover grids smaller than one output slab (S = 2, 4, 6), several
# slabs per axis (S = 20) and one- to eight-chunk reductions.
@pytest.mark.parametrize("B,S,Cin,Cout,k", [(2, 8, 8, 16, 3), (1, 8, 32, 32, 3), (2, 6, 32, 64, 3),
                                             (1, 8, 64, 128, 3), (2, 8, 32, 16, 1), (1, 5, 16, 48, 3),
                                             (2, 4, 16, 32, 3), (2, 2, 32, 64, 3), (1, 20, 8, 32, 3),
                                             (1, 10, 16, 64, 3)])
def test_conv_fwd(gx, eng, B, S, Cin, Cout, k):
    import torch
    rng = np.random.default_rng(B * 100 + S + Cin + Cout + k)
    kv = 27 if k == 3 else 1
    x = oracle.bf16_round(rng.normal(size=(B, S, S, S, Cin)))
    w = oracle.bf16_round(rng.normal(scale=0.2, size=(Cout, kv, Cin)))
    b = rng.normal(size=Cout).astype(np.float32).astype(np.float64)
    out = torch.zeros(B * S ** 3 * Cout, dtype=torch.float32, device="cuda")
    outb = torch.zeros(B * S ** 3 * Cout, dtype=torch.bfloat16, device="cuda")
    eng.conv3d_fwd(_bf(x), B, S, Cin, _bf(w), torch.as_tensor(b, dtype=torch.float32, device="cuda"),
                   k, Cout, 0, out_bf16=outb, out_f32=out)
    ref = oracle.conv3d(x, w, b, k).ravel()
    assert _close(_np(out), ref, rel=1e-5)
    assert _close(_np(outb), ref)
    # LeakyReLU epilogue
    eng.conv3d_fwd(_bf(x), B, S, Cin, _bf(w), torch.as_tensor(b, dtype=torch.float32, device="cuda"),
                   k, Cout, 1, out_f32=out)
    assert _close(_np(out), oracle.lrelu(ref), rel=1e-5)
    # a bf16-only output (staged through LDS and stored in 16-byte pieces by
    # the slab kernel) equals the bf16 rounding of the same values, bit for bit
    bias_t = torch.as_tensor(b, dtype=torch.float32, device="cuda")
    only = torch.full_like(outb, float("nan"))
    eng.conv3d_fwd(_bf(x), B, S, Cin, _bf(w), bias_t, k, Cout, 0, out_bf16=only)
    assert torch.equal(only.view(torch.int16), outb.view(torch.int16))
    only_act = torch.full_like(outb, float("nan"))
    eng.conv3d_fwd(_bf(x), B, S, Cin, _bf(w), bias_t, k, Cout, 1, out_bf16=only_act)
    assert torch.equal(only_act.view(torch.int16), out.to(torch.bfloat16).view(torch.int16))


@pytest.mark.parametrize("B,S,Cin,Cout,k", [(2, 8, 16, 32, 3), (1, 8, 64, 32, 3), (2, 6, 32, 16, 1),
                                             (2, 4, 32, 32, 3), (2, 2, 64, 32, 3)])
def test_conv_bwd_data(gx, eng, B, S, Cin, Cout, k):
    import torch
    rng = np.random.default_rng(7 + Cin)
    kv = 27 if k == 3 else 1
    dy = oracle.bf16_round(rng.normal(size=(B, S, S, S, Cout)))
    w = oracle.bf16_round(rng.normal(scale=0.2, size=(Cout, kv, Cin)))
    yin = oracle.bf16_round(rng.normal(size=(B, S, S, S, Cin)))
    din = torch.zeros(B * S ** 3 * Cin, dtype=torch.bfloat16, device="cuda")
    eng.conv3d_bwd_data(_bf(dy), B, S, Cin, _bf(w), k, Cout, None, din)
    ref = oracle.conv3d_bwd_data(dy, w, Cin, k).ravel()
    assert _close(_np(din), ref)
    eng.conv3d_bwd_data(_bf(dy), B, S, Cin, _bf(w), k, Cout, _bf(yin), din)
    ref2 = ref * np.where(yin.ravel() > 0, 1.0, 0.1)
    assert _close(_np(din), ref2)


# power-of-two grids of at least 8 take the channel-major kernel (including
# half-filled 16-channel input blocks and 32-channel output blocks); other
# grids the LDS-transposing one
@pytest.mark.parametrize("B,S,Cin,Cout,k", [(2, 8, 8, 16, 3), (1, 8, 32, 64, 3), (2, 6, 32, 16, 1),
                                             (1, 16, 16, 32, 3), (1, 32, 64, 32, 3),
                                             (1, 8, 256, 16, 1), (2, 12, 16, 48, 3),
                                             (1, 16, 128, 256, 3)])
def test_conv_bwd_weight(gx, eng, B, S, Cin, Cout, k):
    import torch
    rng = np.random.default_rng(11 + Cout)
    kv = 27 if k == 3 else 1
    x = oracle.bf16_round(rng.normal(size=(B, S, S, S, Cin)))
    dy = oracle.bf16_round(rng.normal(size=(B, S, S, S, Cout)))
    dw = torch.zeros(Cout * kv * Cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    eng.conv3d_bwd_weight(_bf(x), _bf(dy), B, S, Cin, k, Cout, dw, db)
    rw, rb = oracle.conv3d_bwd_weight(x, dy, k)
    assert _close(_np(dw), rw.ravel(), rel=1e-5, rms_frac=1e-5)
    assert _close(_np(db), rb, rel=1e-5, rms_frac=1e-5)


def test_pool_upsample_concat_exact(gx, eng):
    import torch
    rng = np.random.default_rng(3)
    B, S, C = 2, 8, 16
    x = oracle.bf16_round(rng.normal(size=(B, S, S, S, C)))
    out = torch.zeros(B * (S // 2) ** 3 * C, dtype=torch.bfloat16, device="cuda")
    eng.avgpool2(_bf(x), B, S, C, out)
    assert np.array_equal(_np(out), oracle.bf16_round(oracle.avgpool2(x)).ravel())
    up = torch.zeros(B * (2 * S) ** 3 * C, dtype=torch.bfloat16, device="cuda")
    eng.upsample2(_bf(x), B, S, C, up)
    assert np.array_equal(_np(up), oracle.upsample2(x).ravel())
    b = oracle.bf16_round(rng.normal(size=(B, S, S, S, 8)))
    cat = torch.zeros(B * S ** 3 * (C + 8), dtype=torch.bfloat16, device="cuda")
    xa, xb = _bf(x), _bf(b)
    eng.concat(xa, C, xb, 8, B * S ** 3, cat)
    assert np.array_equal(_np(cat), np.concatenate([x, b], axis=-1).ravel())
    ya = torch.zeros_like(xa)
    yb = torch.zeros_like(xb)
    eng.concat(ya, C, yb, 8, B * S ** 3, cat, split=True)
    assert torch.equal(ya, xa) and torch.equal(yb, xb)


def test_unet_forward_backward_matches_oracle(gx, eng):
    import torch
    from paper_2510_23330_amd.unet import UNet
    base, levels, S, B = 16, 3, 8, 2
    net = UNet(eng, S=S, batch=B, base=base, levels=levels, seed=3)
    theta = net.w32.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    x = np.zeros((B, S, S, S, 8))
    x[..., :5] = rng.normal(size=(B, S, S, S, 5))
    x = oracle.bf16_round(x)
    target = rng.normal(size=(B, S, S, S, 5)).astype(np.float32).astype(np.float64)
    xt = _bf(x)
    pred = net.forward(xt)
    th_bf = oracle.bf16_round(theta)
    tab, n, _ = ounet.layer_table(base, levels)
    # weights as the GPU sees them: bf16 weights, fp32 biases
    th_gpu = th_bf.copy()
    for name, d in tab.items():
        th_gpu[d["b"][0]:d["b"][1]] = theta[d["b"][0]:d["b"][1]]
    rb = oracle.bf16_round
    pr, A = ounet.forward(th_gpu, x, base, levels, rb=rb)
    got = _np(pred).reshape(pr.shape)
    err = np.linalg.norm(got - pr) / np.linalg.norm(pr)
    assert err < 2e-2
    V = B * S ** 3
    tt = torch.as_tensor(target.astype(np.float32).ravel(), device="cuda")
    loss = eng.mse(net.pred, 16, tt, 5, V, net.dpred)
    assert loss == pytest.approx(ounet.mse(got, target), rel=1e-6)
    net.zero_grad()
    net.backward(xt, net.dpred)
    dpred = np.zeros_like(pr)
    dpred[..., :5] = 2 * (got[..., :5] - target) / target.size
    dp_gpu = _np(net.dpred).reshape(pr.shape)
    assert np.allclose(dp_gpu, rb(dpred), rtol=2 ** -7, atol=1e-12)
    # The backward pass is checked on the network's own BF16 activations and
    # output gradient: an activation whose FP32 sum lands next to a BF16
    # rounding boundary can round the other way than the FP64 oracle's, and
    # the randomly initialised layers amplify such a flip downstream (to a
    # few 1e-3 of an activation), which would otherwise dominate the
    # comparison.  What remains are the backward kernels' own FP32 sums and
    # BF16 gradient roundings.
    Ag = {k: _np(v).reshape(A[k].shape) for k, v in net.acts.items()}
    g = ounet.backward(th_gpu, x, Ag, dp_gpu, base, levels, rb=rb)
    gg = net.grad.cpu().numpy().astype(np.float64)
    for name, d in tab.items():
        sl = slice(*d["w"])
        e = np.linalg.norm(gg[sl] - g[sl]) / (np.linalg.norm(g[sl]) + 1e-30)
        assert e < 1e-2, (name, e)


def test_adam_matches_oracle(gx, eng):
    import torch
    rng = np.random.default_rng(5)
    n = 1000
    w = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    m = rng.normal(size=n).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=n)).astype(np.float32) * 0.1
    W, G, M, Vv = (torch.as_tensor(a, device="cuda") for a in (w, g, m, v))
    wb = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
    eng.adam_step(W, G, M, Vv, 1e-3, 0.9, 0.999, 1e-8, 7, wb)
    th, mo, vo = ounet.adam(w.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                            v.astype(np.float64), 7, lr=1e-3)
    # FP32 update of FP32 inputs: each moment is a two-term sum, so its error is
    # a few units of 2^-24 of the terms' magnitudes (cancellation can leave a
    # small result with that absolute error).
    ulp = 2.0 ** -24
    em = 4 * ulp * (0.9 * np.abs(m) + 0.1 * np.abs(g))
    ev = 4 * ulp * (0.999 * v + 0.001 * g * g)
    assert np.all(np.abs(M.cpu().numpy() - mo) <= em)
    assert np.all(np.abs(Vv.cpu().numpy() - vo) <= ev)
    assert np.allclose(W.cpu().numpy(), th, rtol=1e-5, atol=1e-7)
    assert np.array_equal(_np(wb), oracle.bf16_round(W.cpu().numpy()))


def test_training_trajectory_matches_oracle(gx, eng):
    # Sixty Adam steps through the project's kernels against the FP64 oracle
    # network (BF16 storage mirrored, FP64 master weights and moments): the
    # loss curves agree step by step.
    import torch
    from paper_2510_23330_amd.unet import UNet
    base, levels, S, B = 16, 2, 8, 1
    net = UNet(eng, S=S, batch=B, base=base, levels=levels, seed=4)
    theta = net.w32.cpu().numpy().astype(np.float64)
    tab, n, _ = ounet.layer_table(base, levels)
    rng = np.random.default_rng(10)
    x = np.zeros((B, S, S, S, 8))
    x[..., :5] = rng.normal(size=(B, S, S, S, 5))
    x = oracle.bf16_round(x)
    target = np.tanh(x[..., :5] * 0.8).astype(np.float32).astype(np.float64)
    xt = _bf(x)
    tt = torch.as_tensor(target.astype(np.float32).ravel(), device="cuda")
    rb = oracle.bf16_round
    is_w = np.zeros(n, bool)
    for d in tab.values():
        is_w[d["w"][0]:d["w"][1]] = True
    m = np.zeros(n)
    v = np.zeros(n)
    lr = 2e-3
    lg, lr_ = [], []
    for step in range(1, 61):
        lg.append(net.train_step(xt, tt, lr=lr))
        th_gpu = np.where(is_w, rb(theta), theta.astype(np.float32))
        pr, A = ounet.forward(th_gpu, x, base, levels, rb=rb)
        lr_.append(ounet.mse(pr, target))
        dpred = np.zeros_like(pr)
        dpred[..., :5] = 2 * (pr[..., :5] - target) / target.size
        g = ounet.backward(th_gpu, x, A, rb(dpred), base, levels, rb=rb)
        theta, m, v = ounet.adam(theta, g, m, v, step, lr=lr)
    lg, lr_ = np.array(lg), np.array(lr_)
    print("trajectory gpu", np.round(lg[::5], 4), "oracle", np.round(lr_[::5], 4))
    # Adam moves every parameter by about lr whatever its gradient's size, so
    # BF16 rounding flips in tiny gradients separate the two runs slowly; the
    # first steps agree closely, the rest stays within a widening band.
    rel = np.abs(lg - lr_) / lr_
    assert np.all(rel[:5] < 1e-2), rel[:5]
    assert np.all(rel < 0.25), rel
    assert lg[-1] < 0.5 * lg[0] and lr_[-1] < 0.5 * lr_[0]


def test_unet_loss_decreases(gx, eng):
    # Training by the project's own kernels on a fixed pair of samples.  An
    # independent FP32 PyTorch CPU run of the same network, initialisation,
    # data and optimiser (Adam, lr 1e-3) reaches 0.20x the initial loss after
    # 150 steps; the BF16 path must reach 0.3x.  (At lr 3e-3 the BF16 run
    # leaves the stable regime.)
    import torch
    from paper_2510_23330_amd.unet import UNet
    S, B = 16, 2
    net = UNet(eng, S=S, batch=B, base=16, levels=3, seed=1)
    rng = np.random.default_rng(2)
    x = np.zeros((B, S, S, S, 8), np.float32)
    x[..., :5] = rng.normal(size=(B, S, S, S, 5))
    tgt = np.tanh(x[..., :5] * 0.7 + 0.3 * np.roll(x[..., :5], 1, axis=1)).astype(np.float32)
    xt = _bf(x)
    tt = torch.as_tensor(tgt.ravel(), device="cuda")
    losses = [net.train_step(xt, tt, lr=1e-3) for _ in range(150)]
    print("loss", np.round(losses[::10], 4))
    assert losses[-1] < 0.3 * losses[0]
    assert losses[-1] < min(losses[:100])


def test_cube_symmetries(gx, eng):
    # The 48 symmetries of the cube used to augment training pairs: a scalar
    # field that depends only on the distance to the centre and the radial
    # velocity field (an explosion) are invariant under every one; a field
    # equal to the input x coordinate and a uniform x velocity land on the
    # axis that the permutation sends x to, reversed by its flip; two equal
    # flips cancel.
    import torch
    S, C = 6, 5
    c = (S - 1) / 2.0
    z, y, x = np.meshgrid(*(np.arange(S, dtype=np.float64),) * 3, indexing="ij")
    rad = np.zeros((S, S, S, C), np.float32)
    rad[..., 0] = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    rad[..., 1] = 1.0
    rad[..., 2], rad[..., 3], rad[..., 4] = x - c, y - c, z - c
    lin = np.zeros((S, S, S, C), np.float32)
    lin[..., 0] = x
    lin[..., 2] = 1.0
    syms = np.arange(48, dtype=np.int32)
    B = syms.size
    for field, invariant in ((rad, True), (lin, False)):
        inp = torch.as_tensor(np.broadcast_to(field, (B,) + field.shape).copy().ravel(), device="cuda")
        out = torch.empty_like(inp)
        eng.cube_sym(inp, B, S, C, 2, torch.as_tensor(syms, device="cuda"), out)
        o = out.cpu().numpy().reshape(B, S, S, S, C)
        perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
        for sidx in range(B):
            if invariant:
                assert np.array_equal(o[sidx], field), sidx
                continue
            P, fl = perms[sidx >> 3], sidx & 7
            a = P.index(0)                       # output axis that carries input x
            coord = (x, y, z)[a]
            exp = (S - 1 - coord) if (fl >> a) & 1 else coord
            assert np.array_equal(o[sidx][..., 0], exp.astype(np.float32)), sidx
            v = np.zeros(3)
            v[a] = -1.0 if (fl >> a) & 1 else 1.0
            for k in range(3):
                assert np.all(o[sidx][..., 2 + k] == v[k]), (sidx, k)
    # flips only: applying the same element twice is the identity
    rng = np.random.default_rng(0)
    f = rng.normal(size=(8, S, S, S, C)).astype(np.float32)
    t = torch.as_tensor(f.ravel(), device="cuda")
    sym = torch.arange(8, dtype=torch.int32, device="cuda")
    once, twice = torch.empty_like(t), torch.empty_like(t)
    eng.cube_sym(t, 8, S, C, 2, sym, once)
    eng.cube_sym(once, 8, S, C, 2, sym, twice)
    assert torch.equal(twice, t)


@pytest.mark.parametrize("case,S,Ca,Cb,Cout", [("upsample", 16, 64, 0, 32), ("concat", 16, 32, 32, 32),
                                               ("upsample", 64, 64, 0, 32), ("concat", 64, 32, 32, 32),
                                               ("both", 8, 16, 16, 48)])
def test_wgrad_fused_inputs_equal_materialized(gx, eng, case, S, Ca, Cb, Cout):
    # The weight gradient of a layer whose input is assembled on the fly
    # (nearest x2 upsampling and/or a channel concatenation), as the U-Net's
    # up path trains without materialising those inputs, equals the weight
    # gradient on the materialised input bit for bit (the same channel-major
    # copy, gathered from the sources).
    import torch
    rng = np.random.default_rng(23)
    B = 2
    up = case in ("upsample", "both")
    Sin = S // 2 if up else S
    a = _bf(oracle.bf16_round(rng.normal(size=(B, Sin, Sin, Sin, Ca))))
    b = _bf(oracle.bf16_round(rng.normal(size=(B, Sin, Sin, Sin, Cb)))) if case != "upsample" else None
    Cin = Ca + (Cb if b is not None else 0)
    V = B * S ** 3
    dy = _bf(oracle.bf16_round(rng.normal(size=(B, S, S, S, Cout))))
    if b is not None:
        cat = torch.zeros(B * Sin ** 3 * Cin, dtype=torch.bfloat16, device="cuda")
        eng.concat(a, Ca, b, Cb, B * Sin ** 3, cat)
    else:
        cat = a
    if up:
        full = torch.zeros(V * Cin, dtype=torch.bfloat16, device="cuda")
        eng.upsample2(cat, B, Sin, Cin, full)
    else:
        full = cat
    dw_ref = torch.zeros(Cout * 27 * Cin, dtype=torch.float32, device="cuda")
    db_ref = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    eng.conv3d_bwd_weight(full, dy, B, S, Cin, 3, Cout, dw_ref, db_ref)
    dw, db = torch.zeros_like(dw_ref), torch.zeros_like(db_ref)
    eng.conv3d_bwd_weight_fused(a, Ca if b is not None else Cin, b, int(up), dy, B, S, Cin, 3, Cout,
                                dw, db)
    assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)
    assert float(dw_ref.abs().max()) > 0


@pytest.mark.parametrize("case,Ca,Cb", [("upsample", 32, 0), ("concat", 32, 32), ("concat", 16, 16),
                                        ("both", 32, 32)])
def test_conv_fused_inputs_equal_materialized(gx, eng, case, Ca, Cb):
    # Convolving an input assembled on the fly (nearest x2 upsampling and/or a
    # channel concatenation) gives what upsample2 / concat followed by the
    # plain convolution gives: bit for bit when both reduce the channels in
    # the same chunks.
    import torch
    rng = np.random.default_rng(21)
    B, S, Cout = 2, 10, 32
    up = case in ("upsample", "both")
    Sin = S // 2 if up else S
    a = _bf(oracle.bf16_round(rng.normal(size=(B, Sin, Sin, Sin, Ca))))
    b = _bf(oracle.bf16_round(rng.normal(size=(B, Sin, Sin, Sin, Cb)))) if case != "upsample" else None
    Cin = Ca + (Cb if b is not None else 0)
    w = _bf(oracle.bf16_round(rng.normal(scale=0.1, size=(Cout, 27, Cin))))
    bias = torch.as_tensor(rng.normal(size=Cout).astype(np.float32), device="cuda")
    # materialized reference
    V = B * S ** 3
    if b is not None:
        cat = torch.zeros(B * Sin ** 3 * Cin, dtype=torch.bfloat16, device="cuda")
        eng.concat(a, Ca, b, Cb, B * Sin ** 3, cat)
    else:
        cat = a
    if up:
        full = torch.zeros(V * Cin, dtype=torch.bfloat16, device="cuda")
        eng.upsample2(cat, B, Sin, Cin, full)
    else:
        full = cat
    ref = torch.zeros(V * Cout, dtype=torch.float32, device="cuda")
    eng.conv3d_fwd(full, B, S, Cin, w, bias, 3, Cout, 1, out_f32=ref)
    got = torch.zeros_like(ref)
    eng.conv3d_fwd_fused(a, Ca if b is not None else Cin, b, int(up), B, S, Cin, w, bias, Cout, 1,
                         out_f32=got)
    if Ca % 32 == 0 and Cb % 32 == 0:
        assert torch.equal(got, ref)
    else:
        # 16-channel sources are reduced in 16-channel chunks (another FP32
        # summation order than the 32-channel chunks of the plain call)
        r = ref.cpu().numpy()
        assert np.max(np.abs(got.cpu().numpy() - r)) <= 1e-5 * np.sqrt(np.mean(r ** 2))


def test_unet_inference_equals_training_forward(gx, eng):
    # The inference-mode network (fused up-path inputs, no saved tensors) and
    # the training-mode network compute the same prediction bit for bit
    # (channel counts multiples of 32: the same reduction chunks).
    import torch
    from paper_2510_23330_amd.unet import UNet
    S, B = 16, 2
    tr = UNet(eng, S=S, batch=B, base=32, levels=3, seed=5)
    inf = UNet(eng, S=S, batch=B, base=32, levels=3, seed=5, train=False)
    rng = np.random.default_rng(6)
    x = np.zeros((B, S, S, S, 8), np.float32)
    x[..., :5] = rng.normal(size=(B, S, S, S, 5))
    xt = _bf(x)
    assert torch.equal(tr.forward(xt).clone(), inf.forward(xt))


@pytest.mark.parametrize("B,S,Cin,Cout", [(2, 16, 8, 32), (1, 12, 32, 64), (2, 10, 16, 128),
                                          (1, 8, 16, 16)])
def test_conv_pool_equals_conv_then_pool(gx, eng, B, S, Cin, Cout):
    # The pooled copy written by the convolution (in the slab kernel's
    # epilogue for outputs a multiple of 32; by a second launch otherwise)
    # equals gx_avgpool2 of the convolution's output, bit for bit; S = 10 and
    # 12 leave partial slabs, Cout = 128 takes two column blocks.
    import torch
    rng = np.random.default_rng(5)
    x = _bf(oracle.bf16_round(rng.normal(size=(B, S, S, S, Cin))))
    w = _bf(oracle.bf16_round(rng.normal(scale=0.1, size=(Cout, 27, Cin))))
    bias = torch.as_tensor(rng.normal(size=Cout).astype(np.float32), device="cuda")
    V = B * S ** 3
    ref = torch.zeros(V * Cout, dtype=torch.bfloat16, device="cuda")
    eng.conv3d_fwd(x, B, S, Cin, w, bias, 3, Cout, 1, out_bf16=ref)
    refp = torch.zeros(V * Cout // 8, dtype=torch.bfloat16, device="cuda")
    eng.avgpool2(ref, B, S, Cout, refp)
    out = torch.zeros_like(ref)
    pool = torch.full_like(refp, float("nan"))
    eng.conv3d_fwd_pool(x, B, S, Cin, w, bias, Cout, 1, out, pool)
    assert torch.equal(out, ref)
    assert torch.equal(pool.view(torch.int16), refp.view(torch.int16))


@pytest.mark.parametrize("B,S,Cin,Cout,nc", [(2, 9, 32, 16, 5), (1, 16, 32, 32, 7)])
def test_conv_head_equals_conv_then_affine(gx, eng, B, S, Cin, Cout, nc):
    # The head convolution writing scale * y + shift for its first nc outputs
    # equals the 1^3 convolution followed by gx_chan_affine, bit for bit
    # (S = 9 leaves a partial 256-voxel block).
    import torch
    rng = np.random.default_rng(8)
    x = _bf(oracle.bf16_round(rng.normal(size=(B, S, S, S, Cin))))
    w = _bf(oracle.bf16_round(rng.normal(scale=0.2, size=(Cout, 1, Cin))))
    bias = torch.as_tensor(rng.normal(size=Cout).astype(np.float32), device="cuda")
    scale = torch.as_tensor(rng.uniform(0.5, 2.0, nc).astype(np.float32), device="cuda")
    shift = torch.as_tensor(rng.normal(size=nc).astype(np.float32), device="cuda")
    V = B * S ** 3
    full = torch.zeros(V * Cout, dtype=torch.float32, device="cuda")
    eng.conv3d_fwd(x, B, S, Cin, w, bias, 1, Cout, 0, out_f32=full)
    ref = torch.zeros(V * nc, dtype=torch.float32, device="cuda")
    eng.chan_affine(full, Cout, nc, scale, shift, out=ref, out_stride=nc)
    got = torch.full_like(ref, float("nan"))
    eng.conv_head(x, B, S, Cin, w, bias, Cout, nc, scale, shift, got, nc)
    assert torch.equal(got, ref)
