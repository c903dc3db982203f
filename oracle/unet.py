"""FP64 oracle of the 3-D U-Net surrogate -- TEST INFRASTRUCTURE ONLY.

Plain composition of the oracle's naive convolution loops (gx_oracle.c) with
NumPy pooling, upsampling, concatenation and LeakyReLU, following the network
of Sec. 3.3 as built here: per level two 3^3 convolutions (bias, LeakyReLU
0.1), 2^3 average pooling down, nearest x2 upsampling + 3^3 convolution up,
skips by channel concatenation, a linear 1^3 head, mean-squared-error loss.

``rb`` (a rounding function, identity by default) is applied wherever the GPU
stores a tensor in BF16 -- activations, pre-activation gradients, loss
gradient -- so that parity tests compare like with like; with the identity
the functions are the exact FP64 network used by the finite-difference pins.
Parameters use the same flat layout as the HIP implementation: every layer's
weights [Cout][kvol][Cin] in layer order, then every layer's bias.
"""
from __future__ import annotations

import numpy as np

from . import avgpool2, conv3d, conv3d_bwd_data, conv3d_bwd_weight, upsample2

SLOPE = 0.1


def layer_table(base=32, levels=4, cin=8, cout=16):
    ch = [base * 2 ** l for l in range(levels)]
    L = []
    c = cin
    for l in range(levels):
        L.append((f"e{l}a", c, ch[l], 3, True))
        L.append((f"e{l}b", ch[l], ch[l], 3, True))
        c = ch[l]
    for l in range(levels - 2, -1, -1):
        L.append((f"u{l}c", ch[l + 1], ch[l], 3, True))
        L.append((f"d{l}a", 2 * ch[l], ch[l], 3, True))
        L.append((f"d{l}b", ch[l], ch[l], 3, True))
    L.append(("head", ch[0], cout, 1, False))
    off = 0
    tab = {}
    for name, ci, co, k, act in L:
        kv = 27 if k == 3 else 1
        tab[name] = dict(cin=ci, cout=co, k=k, act=act, w=(off, off + co * kv * ci), kv=kv)
        off += co * kv * ci
    for name, ci, co, k, act in L:
        tab[name]["b"] = (off, off + co)
        off += co
    return tab, off, ch


def _params(theta, t, name):
    d = t[name]
    w = theta[d["w"][0]:d["w"][1]].reshape(d["cout"], d["kv"], d["cin"])
    b = theta[d["b"][0]:d["b"][1]]
    return w, b


def forward(theta, x, base=32, levels=4, rb=lambda a: a):
    """x [B,S,S,S,8] -> (pred [B,S,S,S,16], saved tensors)."""
    t, _, ch = layer_table(base, levels)
    A = {}

    def conv(name, h):
        w, b = _params(theta, t, name)
        z = conv3d(h, w, b, t[name]["k"])
        return rb(np.where(z > 0, z, SLOPE * z)) if t[name]["act"] else z

    h = x
    for l in range(levels):
        A[f"e{l}a"] = conv(f"e{l}a", h)
        A[f"e{l}b"] = conv(f"e{l}b", A[f"e{l}a"])
        if l < levels - 1:
            A[f"p{l}"] = rb(avgpool2(A[f"e{l}b"]))
            h = A[f"p{l}"]
    h = A[f"e{levels - 1}b"]
    for l in range(levels - 2, -1, -1):
        A[f"up{l}"] = upsample2(h)
        A[f"u{l}c"] = conv(f"u{l}c", A[f"up{l}"])
        A[f"c{l}"] = np.concatenate([A[f"u{l}c"], A[f"e{l}b"]], axis=-1)
        A[f"d{l}a"] = conv(f"d{l}a", A[f"c{l}"])
        A[f"d{l}b"] = conv(f"d{l}b", A[f"d{l}a"])
        h = A[f"d{l}b"]
    pred = conv("head", h)
    return pred, A


def mse(pred, target, nc=5):
    d = pred[..., :nc] - target
    return float(np.mean(d * d))


def backward(theta, x, A, dpred, base=32, levels=4, rb=lambda a: a):
    """Gradient of the loss w.r.t. the flat parameters, given dL/dpred."""
    t, n, ch = layer_table(base, levels)
    g = np.zeros(n)

    def dact(gpost, y):
        return gpost * np.where(y > 0, 1.0, SLOPE)

    def wgrad(name, h, dy):
        dw, db = conv3d_bwd_weight(h, dy, t[name]["k"])
        g[t[name]["w"][0]:t[name]["w"][1]] += dw.ravel()
        g[t[name]["b"][0]:t[name]["b"][1]] += db

    def dgrad(name, dy):
        w, _ = _params(theta, t, name)
        return conv3d_bwd_data(dy, w, t[name]["cin"], t[name]["k"])

    top = levels - 1
    G = {}
    wgrad("head", A["d0b"], dpred)
    G["d0b"] = rb(dact(dgrad("head", dpred), A["d0b"]))
    skip = {}
    for l in range(0, top):
        wgrad(f"d{l}b", A[f"d{l}a"], G[f"d{l}b"])
        G[f"d{l}a"] = rb(dact(dgrad(f"d{l}b", G[f"d{l}b"]), A[f"d{l}a"]))
        wgrad(f"d{l}a", A[f"c{l}"], G[f"d{l}a"])
        gc = rb(dgrad(f"d{l}a", G[f"d{l}a"]))
        gu, skip[l] = gc[..., :ch[l]], gc[..., ch[l]:]
        G[f"u{l}c"] = rb(dact(gu, A[f"u{l}c"]))
        wgrad(f"u{l}c", A[f"up{l}"], G[f"u{l}c"])
        gup = rb(dgrad(f"u{l}c", G[f"u{l}c"]))
        B, S2, _, _, C = gup.shape
        gcoarse = gup.reshape(B, S2 // 2, 2, S2 // 2, 2, S2 // 2, 2, C).sum(axis=(2, 4, 6))
        below = f"d{l + 1}b" if l + 1 < top else f"e{top}b"
        G[below] = rb(dact(rb(gcoarse), A[below]))
    for l in range(top, -1, -1):
        wgrad(f"e{l}b", A[f"e{l}a"], G[f"e{l}b"])
        G[f"e{l}a"] = rb(dact(dgrad(f"e{l}b", G[f"e{l}b"]), A[f"e{l}a"]))
        if l == 0:
            wgrad("e0a", x, G["e0a"])
            break
        wgrad(f"e{l}a", A[f"p{l - 1}"], G[f"e{l}a"])
        gp = rb(dgrad(f"e{l}a", G[f"e{l}a"]))
        gfine = rb(upsample2(gp) / 8.0)
        G[f"e{l - 1}b"] = rb(dact(gfine + skip[l - 1], A[f"e{l - 1}b"]))
    return g


def adam(theta, g, m, v, t, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in FP64; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
