"""The surrogate network at its production shape -- 64^3 voxels, 4 levels of
32, 64, 128, 256 channels, one sample -- against the FP64 oracle, element by
element, through the whole-network calls gx_unet_forward / gx_unet_backward.

Layer by layer: every convolution of the inference pass (including the
pooling fused into the encoder convolutions, the up-path convolutions that
read upsampled and concatenated inputs on the fly, and the head's output
scaling) and of the training pass (forward, data gradient, weight gradient)
is recomputed by the oracle's naive FP64 loops from the network's own BF16
input to that layer, so each comparison isolates one kernel launch at a
production shape (S = 64 with 8 -> 32, 32 -> 32 and 64 -> 32 channels down
to S = 8 with 256 channels).

Bounds, from the arithmetic:
* BF16 outputs: the FP32 sum of K = 27 Cin <= 6,912 products of BF16
  operands is within ~1e-5 relative of the FP64 sum; both are rounded to
  BF16 (8 significant bits), and where the two sums straddle a rounding
  boundary the results differ by one unit in the last place, up to 2^-7 of
  the value: |got - ref| <= 2^-7 |ref| + 1e-4 rms(ref).
* FP32 outputs: the head (|d| <= 1e-5 |ref| + 1e-6 rms) and the weight
  gradients, FP32 sums over 2.6e5 voxels in a fixed chunked order
  (|d| <= 1e-3 rms(ref) + 1e-4 |ref|).
* End to end against the oracle network with BF16 storage mirrored: each of
  the 20 BF16 roundings on the longest path (e0a ... e3b, then u2c ... d0b,
  the head) can land one unit apart from the oracle's, and the differences
  add like a random walk, sqrt(20) units ~ 2^-4.8 of a value; allowed per
  element 2^-4 (|ref| + rms), at the 99th percentile 2^-6 rms, and 5e-3 in
  relative norm (one such case measured 2.5e-2, 8.5e-3 and 2.5e-3).
"""
import numpy as np
import pytest

import oracle
from oracle import unet as ounet

pytestmark = pytest.mark.gpu

S, BASE, LEVELS = 64, 32, 4
rb = oracle.bf16_round


@pytest.fixture(scope="module")
def eng(gx):
    e = gx.Engine(0)
    yield e
    e.close()


def _bf(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float32).ravel(),
                           device="cuda").to(torch.bfloat16)


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _check_bf16(name, got, ref):
    rms = np.sqrt(np.mean(ref ** 2)) + 1e-30
    bad = np.abs(got - ref) > 2 ** -7 * np.abs(ref) + 1e-4 * rms
    assert not bad.any(), (name, int(bad.sum()), float(np.max(np.abs(got - ref)) / rms))


def _check_f32(name, got, ref, rel, rms_frac):
    rms = np.sqrt(np.mean(ref ** 2)) + 1e-30
    bad = np.abs(got - ref) > rel * np.abs(ref) + rms_frac * rms
    assert not bad.any(), (name, int(bad.sum()), float(np.max(np.abs(got - ref)) / rms))


def _lrelu(z):
    return np.where(z > 0, z, 0.1 * z)


def _dact(g, y):
    return g * np.where(y > 0, 1.0, 0.1)


def _shape(s, c):
    return (1, s, s, s, c)


def _setup(gx, eng, train, seed):
    from paper_2510_23330_amd.unet import UNet
    net = UNet(eng, S=S, batch=1, base=BASE, levels=LEVELS, seed=seed, train=train)
    rng = np.random.default_rng(seed + 100)
    x = np.zeros(_shape(S, 8))
    x[..., :5] = rng.normal(size=_shape(S, 5))
    x = rb(x)
    theta = net.w32.cpu().numpy().astype(np.float64)
    tab, n, ch = ounet.layer_table(BASE, LEVELS)
    assert n == net.n_params
    for ly in net.L:   # the library's layer table is the oracle's
        assert (tab[ly.name]["w"][0], tab[ly.name]["b"][0]) == (ly.w_off, ly.b_off)
    W, Bias = {}, {}
    for name, d in tab.items():
        W[name] = rb(theta[d["w"][0]:d["w"][1]]).reshape(d["cout"], d["kv"], d["cin"])
        Bias[name] = theta[d["b"][0]:d["b"][1]].astype(np.float32).astype(np.float64)
    return net, x, theta, tab, ch, W, Bias


def _forward_checks(net, x, tab, ch, W, Bias, materialized):
    """Each forward convolution (and pooling) from the GPU's own inputs."""
    top = LEVELS - 1
    A = {}
    names = []
    for l in range(LEVELS):
        names += [f"e{l}a", f"e{l}b"] + ([f"p{l}", f"u{l}c", f"d{l}a", f"d{l}b"] if l < top else [])
        if materialized and l < top:
            names += [f"up{l}", f"c{l}"]
    for nm in names:
        l = int(nm[-1]) if nm[0] in "pc" or nm.startswith("up") else int(nm[1])
        s = S >> l
        c = ch[l] * (2 if nm[0] == "c" else 1)
        if nm.startswith("up"):
            s, c = S >> l, ch[l + 1]
        if nm[0] == "p":
            s = (S >> l) // 2
        A[nm] = _np(net.eng.unet_saved(nm)).reshape(_shape(s, c))

    def conv(name, h):
        return rb(_lrelu(oracle.conv3d(h, W[name], Bias[name], 3)))

    for l in range(LEVELS):
        src = x if l == 0 else A[f"p{l - 1}"]
        _check_bf16(f"e{l}a", A[f"e{l}a"], conv(f"e{l}a", src))
        _check_bf16(f"e{l}b", A[f"e{l}b"], conv(f"e{l}b", A[f"e{l}a"]))
        if l < top:
            _check_bf16(f"p{l}", A[f"p{l}"], rb(oracle.avgpool2(A[f"e{l}b"])))
    for l in range(top - 1, -1, -1):
        below = A[f"d{l + 1}b"] if l + 1 < top else A[f"e{top}b"]
        up = oracle.upsample2(below)
        if materialized:
            assert np.array_equal(A[f"up{l}"], up)
        _check_bf16(f"u{l}c", A[f"u{l}c"], conv(f"u{l}c", up))
        cat = np.concatenate([A[f"u{l}c"], A[f"e{l}b"]], axis=-1)
        if materialized:
            assert np.array_equal(A[f"c{l}"], cat)
        _check_bf16(f"d{l}a", A[f"d{l}a"], conv(f"d{l}a", cat))
        _check_bf16(f"d{l}b", A[f"d{l}b"], conv(f"d{l}b", A[f"d{l}a"]))
    return A


def test_production_unet_inference_layer_by_layer(gx, eng):
    import torch
    net, x, theta, tab, ch, W, Bias = _setup(gx, eng, False, 11)
    rng = np.random.default_rng(12)
    scale = rng.uniform(0.5, 2.0, 5).astype(np.float32)
    shift = rng.normal(size=5).astype(np.float32)
    out = torch.zeros(S ** 3 * 5, dtype=torch.float32, device="cuda")
    net.forward(_bf(x), out_phys=out, scale=torch.as_tensor(scale, device="cuda"),
                shift=torch.as_tensor(shift, device="cuda"))
    A = _forward_checks(net, x, tab, ch, W, Bias, materialized=False)
    y = oracle.conv3d(A["d0b"], W["head"], Bias["head"], 1)[..., :5]
    ref = y * scale.astype(np.float64) + shift.astype(np.float64)
    _check_f32("head", out.cpu().numpy().astype(np.float64).reshape(ref.shape), ref, 1e-5, 1e-6)
    # end to end against the oracle network (BF16 storage mirrored)
    th_gpu = theta.copy()
    for name, d in tab.items():
        th_gpu[d["w"][0]:d["w"][1]] = rb(theta[d["w"][0]:d["w"][1]])
        th_gpu[d["b"][0]:d["b"][1]] = Bias[name]
    pr, _ = ounet.forward(th_gpu, x, BASE, LEVELS, rb=rb)
    ref = pr[..., :5] * scale.astype(np.float64) + shift.astype(np.float64)
    got = out.cpu().numpy().astype(np.float64).reshape(ref.shape)
    rms = np.sqrt(np.mean(ref ** 2))
    d = np.abs(got - ref)
    print(f"production U-Net end to end: rel norm {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}, "
          f"max |d|/rms {d.max() / rms:.2e}, p99 {np.percentile(d, 99) / rms:.2e}")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 5e-3
    assert np.percentile(d, 99) <= 2 ** -6 * rms
    assert np.all(d <= 2 ** -4 * (np.abs(ref) + rms))


def test_production_unet_training_layer_by_layer(gx, eng):
    import torch
    net, x, theta, tab, ch, W, Bias = _setup(gx, eng, True, 21)
    xt = _bf(x)
    pred = net.forward(xt)
    A = _forward_checks(net, x, tab, ch, W, Bias, materialized=True)
    _check_f32("head", _np(pred).reshape(_shape(S, 16)),
               oracle.conv3d(A["d0b"], W["head"], Bias["head"], 1), 1e-5, 1e-6)
    rng = np.random.default_rng(22)
    target = rng.normal(size=_shape(S, 5)).astype(np.float32)
    V = S ** 3
    eng.mse(pred, 16, torch.as_tensor(target.ravel(), device="cuda"), 5, V, net.dpred)
    net.zero_grad()
    net.backward(xt, net.dpred)
    dpred = _np(net.dpred).reshape(_shape(S, 16))
    top = LEVELS - 1
    G = {}
    for l in range(LEVELS):
        s = S >> l
        G[f"e{l}a"] = _np(eng.unet_saved(f"e{l}a", True)).reshape(_shape(s, ch[l]))
        G[f"e{l}b"] = _np(eng.unet_saved(f"e{l}b", True)).reshape(_shape(s, ch[l]))
        if l < top:
            G[f"p{l}"] = _np(eng.unet_saved(f"p{l}", True)).reshape(_shape(s // 2, ch[l]))
            G[f"skip{l}"] = _np(eng.unet_saved(f"skip{l}", True)).reshape(_shape(s, ch[l]))
            G[f"up{l}"] = _np(eng.unet_saved(f"up{l}", True)).reshape(_shape(s, ch[l + 1]))
            G[f"c{l}"] = _np(eng.unet_saved(f"c{l}", True)).reshape(_shape(s, 2 * ch[l]))
            for k in (f"u{l}c", f"d{l}a", f"d{l}b"):
                G[k] = _np(eng.unet_saved(k, True)).reshape(_shape(s, ch[l]))
    grad = net.grad.cpu().numpy().astype(np.float64)

    def wcheck(name, X, dY):
        d = tab[name]
        dw, db = oracle.conv3d_bwd_weight(X, dY, d["k"])
        _check_f32(name + ".dw", grad[d["w"][0]:d["w"][1]], dw.ravel(), 1e-4, 1e-3)
        _check_f32(name + ".db", grad[d["b"][0]:d["b"][1]], db, 1e-4, 1e-3)

    def dcheck(name, dY, got, y_in):
        d = tab[name]
        g = oracle.conv3d_bwd_data(dY, W[name], d["cin"], d["k"])
        ref = rb(_dact(g, y_in)) if y_in is not None else rb(g)
        _check_bf16(name + ".dx", got, ref)

    wcheck("head", A["d0b"], dpred)
    dcheck("head", dpred, G["d0b"], A["d0b"])
    for l in range(top):
        wcheck(f"d{l}b", A[f"d{l}a"], G[f"d{l}b"])
        dcheck(f"d{l}b", G[f"d{l}b"], G[f"d{l}a"], A[f"d{l}a"])
        wcheck(f"d{l}a", A[f"c{l}"], G[f"d{l}a"])
        dcheck(f"d{l}a", G[f"d{l}a"], G[f"c{l}"], None)
        # the concatenation's gradient splits; the up-path part takes its
        # activation derivative
        assert np.array_equal(G[f"skip{l}"], G[f"c{l}"][..., ch[l]:])
        _check_bf16(f"u{l}c.g", G[f"u{l}c"], rb(_dact(G[f"c{l}"][..., :ch[l]], A[f"u{l}c"])))
        wcheck(f"u{l}c", A[f"up{l}"], G[f"u{l}c"])
        dcheck(f"u{l}c", G[f"u{l}c"], G[f"up{l}"], None)
        # through the upsampling (sum of the 8 fine cells) into the coarser
        # level's output, times its activation derivative
        below = f"d{l + 1}b" if l + 1 < top else f"e{top}b"
        gup = G[f"up{l}"]
        h = gup.shape[1] // 2
        gco = gup.reshape(1, h, 2, h, 2, h, 2, -1).sum(axis=(2, 4, 6))
        _check_bf16(below + ".g", G[below], rb(_dact(rb(gco), A[below])))
    for l in range(top, -1, -1):
        wcheck(f"e{l}b", A[f"e{l}a"], G[f"e{l}b"])
        dcheck(f"e{l}b", G[f"e{l}b"], G[f"e{l}a"], A[f"e{l}a"])
        if l == 0:
            wcheck("e0a", x, G["e0a"])
        else:
            wcheck(f"e{l}a", A[f"p{l - 1}"], G[f"e{l}a"])
            dcheck(f"e{l}a", G[f"e{l}a"], G[f"p{l - 1}"], None)
            # through the pooling, plus the skip's share, into level l-1's output
            fine = rb(oracle.upsample2(G[f"p{l - 1}"]) / 8.0)
            _check_bf16(f"e{l - 1}b.g", G[f"e{l - 1}b"],
                        rb(_dact(fine + G[f"skip{l - 1}"], A[f"e{l - 1}b"])))
