"""Pins of the FP64 SPH and leapfrog oracle: kernel normalisation and
derivative, lattice density, symmetry and conservation identities, a linear
pressure gradient, and exactness of the kick-drift-kick update."""
import math

import numpy as np
import pytest
from scipy import integrate

import ics
import oracle

GAMMA = 5.0 / 3.0


def test_kernel_normalisation():
    for H in (0.3, 1.0, 2.7):
        val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.wendland_c4(r, H), 0, H,
                                epsabs=1e-14, epsrel=1e-13)
        assert val == pytest.approx(1.0, abs=1e-12)


def test_kernel_derivative_matches_finite_difference():
    H = 0.8
    for r in np.linspace(0.01, 0.79, 23):
        h = 1e-6
        fd = (oracle.wendland_c4(r + h, H) - oracle.wendland_c4(r - h, H)) / (2 * h)
        assert oracle.wendland_c4_dr(r, H) == pytest.approx(fd, rel=1e-7, abs=1e-9)
    assert oracle.wendland_c4(0.8, 0.8) == 0.0 and oracle.wendland_c4_dr(0.8, 0.8) == 0.0


def test_kernel_compact_support_smooth():
    # W and dW/dr vanish continuously at q = 1 (Wendland C4 is C^4 there).
    H = 1.0
    assert oracle.wendland_c4(1 - 1e-4, H) < 1e-20
    assert abs(oracle.wendland_c4_dr(1 - 1e-4, H)) < 1e-16


def _interior(p, nside, margin):
    lo, hi = margin, (nside - 1) - margin
    return np.where((p["x"] >= lo) & (p["x"] <= hi) & (p["y"] >= lo) & (p["y"] <= hi)
                    & (p["z"] >= lo) & (p["z"] <= hi))[0]


@pytest.mark.parametrize("n_ngb,bias", [(64.0, 0.015), (128.0, 0.003), (256.0, 5e-4)])
def test_lattice_density_is_uniform_density(n_ngb, bias):
    # A cubic lattice of spacing 1 and unit masses has rho0 = 1; the SPH estimate
    # returns it up to the kernel's lattice bias, which vanishes as the
    # neighbour number grows (1.1 % at 64, 0.19 % at 128, 0.035 % at 256).
    nside = 24
    p = ics.lattice(nside)
    H, rho, it, nfail = oracle.sph_density(p, n_ngb, 1e-10, 200)
    assert nfail == 0
    inner = _interior(p, nside, 7)
    assert np.max(np.abs(rho[inner] - 1.0)) < bias
    # every interior particle sees the same neighbourhood: identical H
    assert np.ptp(H[inner]) < 1e-9 * np.mean(H[inner])
    # the solution satisfies its defining relation (4 pi / 3) H^3 rho / m = N_ngb
    neff = 4 * math.pi / 3 * H ** 3 * rho / p["m"]
    assert np.max(np.abs(neff - n_ngb)) < 1e-9


def test_density_neighbour_set_complete():
    # Every particle within H contributes: compare with an all-pairs sum at the
    # oracle's own H on a small random set.
    g = ics.gas_sphere(600, 31)
    H, rho, it, nfail = oracle.sph_density(g, 64.0, 1e-12, 200)
    x = np.stack([g["x"], g["y"], g["z"]], 1)
    r = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    W = np.vectorize(oracle.wendland_c4)(r, H[:, None])
    assert np.allclose(W @ g["m"], rho, rtol=1e-12, atol=0)


def test_density_newton_iterations_warm_start():
    # With a good initial kernel size the iteration converges in about two steps
    # (Sec. 5.2.5); from a perturbed previous solution we allow a mean <= 3.
    g = ics.gas_sphere(4096, 2)
    H, rho, it, nfail = oracle.sph_density(g, 64.0, 1e-3, 64)
    H2, rho2, it2, nf2 = oracle.sph_density(g, 64.0, 1e-3, 64, H_guess=H * 1.02)
    assert nfail == 0 and nf2 == 0
    assert np.mean(it2) <= 3.0


def test_uniform_lattice_force_vanishes():
    nside = 16
    p = ics.lattice(nside, u=2.0)
    H, rho, _, _ = oracle.sph_density(p, 64.0, 1e-12, 200)
    ax, ay, az, dudt, vsig = oracle.sph_force(p, H, rho, GAMMA, 1.0)
    inner = _interior(p, nside, 5)
    P = (GAMMA - 1) * rho * 2.0
    scale = np.mean(P / rho) / np.mean(H)
    for a in (ax, ay, az):
        assert np.max(np.abs(a[inner])) < 1e-12 * scale
    assert np.max(np.abs(dudt[inner])) < 1e-12 * scale
    c = math.sqrt(GAMMA * (GAMMA - 1) * 2.0)
    assert np.allclose(vsig[inner], 2 * c, rtol=1e-12)


def test_linear_pressure_gradient():
    # u = u0 (1 + g x) on a uniform lattice: -grad P / rho = -(gamma - 1) u0 g.
    nside = 20
    p = ics.lattice(nside)
    u0, gr = 1.0, 0.01
    p["u"] = u0 * (1 + gr * p["x"])
    H, rho, _, _ = oracle.sph_density(p, 64.0, 1e-12, 200)
    ax, ay, az, dudt, vsig = oracle.sph_force(p, H, rho, GAMMA, 1.0)
    inner = _interior(p, nside, 5)
    expect = -(GAMMA - 1) * u0 * gr
    assert np.mean(ax[inner]) == pytest.approx(expect, rel=0.03)
    assert np.max(np.abs(ay[inner])) < 1e-3 * abs(expect)


def test_force_conserves_momentum_and_energy():
    g = ics.gas_sphere(4096, 2)
    H, rho, _, _ = oracle.sph_density(g, 64.0, 1e-10, 200)
    ax, ay, az, dudt, vsig = oracle.sph_force(g, H, rho, GAMMA, 1.0)
    m = g["m"]
    scale = np.sum(m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2))
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) <= 1e-13 * scale
    dE = np.sum(m * (g["vx"] * ax + g["vy"] * ay + g["vz"] * az + dudt))
    assert abs(dE) <= 1e-13 * np.sum(m * np.abs(dudt))
    # viscosity only heats: with alpha > 0 and no pressure work from a static
    # lattice the heating is non-negative; here check the signal speed bound
    c = np.sqrt(GAMMA * (GAMMA - 1) * g["u"])
    assert np.all(vsig >= c - 1e-15)


def test_viscosity_heats_converging_flow():
    # A uniformly converging lattice (v = -k r) has only compressive pairs:
    # every interior particle is heated, and more with larger alpha.
    nside = 14
    p = ics.lattice(nside)
    c0 = (nside - 1) / 2
    k = 0.3
    p["vx"], p["vy"], p["vz"] = -k * (p["x"] - c0), -k * (p["y"] - c0), -k * (p["z"] - c0)
    H, rho, _, _ = oracle.sph_density(p, 64.0, 1e-12, 200)
    inner = _interior(p, nside, 4)
    du0 = oracle.sph_force(p, H, rho, GAMMA, 0.0)[3]
    du1 = oracle.sph_force(p, H, rho, GAMMA, 1.0)[3]
    # compression work alone: du/dt = (P / rho) div(-v) > 0
    assert np.all(du0[inner] > 0)
    assert np.all(du1[inner] > du0[inner])


def test_kdk_constant_acceleration_exact():
    rng = np.random.default_rng(4)
    x0 = rng.normal(size=(3, 50))
    v0 = rng.normal(size=(3, 50))
    a = rng.normal(size=(3, 50))
    dt = 0.125
    x, v, _, _, _ = oracle.kick_drift(x0, v0, a, dt / 2, dt)
    _, v, _, _, _ = oracle.kick_drift(x, v, a, dt / 2, 0.0)
    assert np.allclose(x, x0 + v0 * dt + 0.5 * a * dt * dt, rtol=0, atol=1e-15)
    assert np.allclose(v, v0 + a * dt, rtol=0, atol=1e-15)


def test_kdk_second_order_energy_error():
    # One-dimensional harmonic oscillator a = -x: the largest energy error over a fixed time
    # scales as dt^2 for the second-order leapfrog.
    def run(dt, T=10.0):
        x = np.array([[1.0], [0.0], [0.0]])
        v = np.array([[0.0], [0.0], [0.0]])
        a = -x
        worst = 0.0
        for _ in range(int(round(T / dt))):
            x, v, _, _, _ = oracle.kick_drift(x, v, a, dt / 2, dt)
            a = -x
            _, v, _, _, _ = oracle.kick_drift(x, v, a, dt / 2, 0.0)
            worst = max(worst, abs(np.sum(v * v) + np.sum(x * x) - 1.0) / 2)
        return worst
    e1, e2 = run(0.1), run(0.05)
    assert 3.5 < e1 / e2 < 4.5
