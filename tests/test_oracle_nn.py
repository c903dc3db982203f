"""Pins of the surrogate oracle: convolution closed forms and adjointness,
finite-difference gradients of the whole U-Net, Adam's first step, BF16
rounding, and the voxelizer's Shepard partition of unity and mass."""
import math

import numpy as np
import pytest

import ics
import oracle
from oracle import unet as ounet


def test_bf16_round_known_values():
    v = np.array([1.0, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5, 3.140625, 1e-40])
    r = oracle.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even
    assert r[2] == 1.0 + 2 ** -7          # tie -> even (up)
    assert r[3] == -2.5
    assert r[4] == 3.140625
    assert abs(r[5]) < 1e-39


def test_conv_delta_response():
    # A unit impulse at voxel p, channel ci returns w[co][tap][ci] at p - d(tap).
    rng = np.random.default_rng(1)
    S, Cin, Cout = 5, 3, 4
    w = rng.normal(size=(Cout, 27, Cin))
    x = np.zeros((1, S, S, S, Cin))
    x[0, 2, 2, 2, 1] = 1.0
    y = oracle.conv3d(x, w, None, 3)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                assert np.allclose(y[0, 2 - dz, 2 - dy, 2 - dx], w[:, tap, 1], rtol=0, atol=1e-15)
    mask = np.ones((S, S, S), bool)
    mask[1:4, 1:4, 1:4] = False
    assert np.all(y[0][mask] == 0)


def test_conv_identity_kernel_and_bias():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 4, 4, 6))
    w = np.zeros((6, 27, 6))
    w[:, 13, :] = np.eye(6)
    b = np.arange(6.0)
    assert np.allclose(oracle.conv3d(x, w, b, 3), x + b, atol=1e-14)
    w1 = np.eye(6).reshape(6, 1, 6)
    assert np.allclose(oracle.conv3d(x, w1, None, 1), x, atol=1e-14)


@pytest.mark.parametrize("ksize", [3, 1])
def test_conv_adjoint(ksize):
    # <conv(x), y> = <x, conv_bwd_data(y)> and = <w, conv_bwd_weight(x, y)>.
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 5, 5, 5, 4))
    kv = 27 if ksize == 3 else 1
    w = rng.normal(size=(3, kv, 4))
    y = rng.normal(size=(2, 5, 5, 5, 3))
    lhs = np.sum(oracle.conv3d(x, w, None, ksize) * y)
    assert np.sum(x * oracle.conv3d_bwd_data(y, w, 4, ksize)) == pytest.approx(lhs, rel=1e-12)
    dw, db = oracle.conv3d_bwd_weight(x, y, ksize)
    assert np.sum(w * dw) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, y.sum(axis=(0, 1, 2, 3)), rtol=1e-12)


def test_unet_gradient_finite_difference():
    # Exact FP64 network: backward matches central differences of the MSE loss.
    base, levels, S = 16, 2, 4
    tab, n, _ = ounet.layer_table(base, levels)
    rng = np.random.default_rng(4)
    theta = rng.normal(scale=0.15, size=n)
    x = rng.normal(size=(1, S, S, S, 8))
    target = rng.normal(size=(1, S, S, S, 5))

    def loss(th):
        p, _ = ounet.forward(th, x, base, levels)
        return ounet.mse(p, target)

    pred, A = ounet.forward(theta, x, base, levels)
    d = np.zeros_like(pred)
    d[..., :5] = 2 * (pred[..., :5] - target) / target.size
    g = ounet.backward(theta, x, A, d, base, levels)
    picks = rng.choice(n, 40, replace=False)
    for i in picks:
        h = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-4, abs=1e-9)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = ounet.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    # t = 1: mhat = g, vhat = g^2 -> step = -lr g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def _sn_like(n=3000, seed=5):
    rng = np.random.default_rng(seed)
    p = {k: rng.uniform(-30, 30, n) for k in ("x", "y", "z")}
    p["m"] = np.ones(n)
    p["H"] = rng.uniform(4.0, 8.0, n)
    p["u"] = np.full(n, 2.5)
    p["vx"], p["vy"], p["vz"] = np.full(n, 1.5), np.full(n, -3.0), np.zeros(n)
    return p


def test_voxelize_shepard_partition_of_unity():
    # Constant temperature and velocity fields are returned exactly wherever a
    # kernel reaches (Shepard normalisation).
    p = _sn_like()
    out = oracle.voxelize(p, 48.46, np.zeros(3), 60.0, 16, np.array([-3.0, 2.0, 0, 0, 0]))
    assert np.allclose(out[..., 1], math.log10(2.5 * 48.46), atol=1e-12)
    assert np.allclose(out[..., 2], 1.5, atol=1e-12)
    assert np.allclose(out[..., 3], -3.0, atol=1e-12)


def test_voxelize_mass_of_interior():
    # Sum of rho dV over a cube that contains every kernel equals the total mass
    # (kernel normalisation), up to the grid's quadrature error.
    rng = np.random.default_rng(6)
    n = 400
    p = {k: rng.uniform(-10, 10, n) for k in ("x", "y", "z")}
    p["m"] = np.full(n, 2.0)
    p["H"] = np.full(n, 6.0)
    p["u"] = np.ones(n)
    p["vx"] = p["vy"] = p["vz"] = np.zeros(n)
    out = oracle.voxelize(p, 1.0, np.zeros(3), 60.0, 48, np.array([-12.0, 1, 0, 0, 0]))
    dv = (60.0 / 48) ** 3
    assert np.sum(10 ** out[..., 0]) * dv == pytest.approx(800.0, rel=2e-3)
