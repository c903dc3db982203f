"""Pins of the oracle parts that the closed forms and brute-force checks of the
other CPU tests leave open: the opening criterion (strict inequality,
geometric cell side, box-to-box distance), the mass-weighted mean softening
of a cell, the magnitude of the signal-velocity viscosity, and the energy
audit and equation of state.  Each test is built so that a plausible slip in
the oracle (a <= for the <, a centre distance, an unweighted mean, a dropped
receiver softening, another viscosity factor, a missing 1/2) fails it."""
import math

import numpy as np
import pytest

import oracle

GAMMA = 5.0 / 3.0


def _pset(pts, m=None, eps2=None):
    pts = np.asarray(pts, np.float64)
    n = len(pts)
    return {"x": pts[:, 0].copy(), "y": pts[:, 1].copy(), "z": pts[:, 2].copy(),
            "m": np.ones(n) if m is None else np.asarray(m, np.float64),
            "eps2": np.zeros(n, np.float32) if eps2 is None else np.asarray(eps2, np.float32)}


# --------------------------------------------------------------------------
# Opening criterion: accept cell c for group G when l_c < theta * d, with
# l_c = L / 2^level the geometric side and d the minimum distance between the
# tight boxes of G and c.
# --------------------------------------------------------------------------
def _mac_setup():
    # anchor at the origin and a far corner at (1, 1, 1): root corner 0, root
    # side L = 1 * (1 + 2^-40).  The receiver P0 and the pair c1, c2 have
    # dyadic coordinates; c1, c2 share the level-1, -2 and -3 cells with x in
    # [5L/8, 6L/8) and split at level 4, so three nested nodes hold exactly
    # {c1, c2} (same tight box).  The box distance from P0 is along x only:
    # d = 41/64 - 25/64 = 1/4 exactly (P0's y, z lie inside the pair's range).
    pts = [(0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
           (25 / 64, 1 / 16, 1 / 16),       # P0, the receiving group
           (41 / 64, 1 / 32, 1 / 32),       # c1
           (47 / 64, 3 / 32, 3 / 32)]       # c2
    p = _pset(pts)
    T = oracle.Tree(p, 1, 1)
    nd = T.nodes()
    key, perm = T.sorted()
    slot = {int(perm[s]): s for s in range(len(perm))}
    g_of = {}
    for g, node in enumerate(T.groups()):
        for s in range(nd["begin"][node], nd["end"][node]):
            g_of[int(perm[s])] = g

    def node_of(members, level):
        ss = sorted(slot[i] for i in members)
        hit = [k for k in range(T.n_nodes) if nd["level"][k] == level and nd["begin"][k] == ss[0]
               and nd["end"][k] == ss[-1] + 1]
        assert len(hit) == 1
        return hit[0]

    L = 1.0 * (1.0 + 2.0 ** -40)
    return T, g_of[2], {lev: node_of([3, 4], lev) for lev in (1, 2, 3)}, \
        (node_of([3], 4), node_of([4], 4)), L


def _pc_of(T, g, theta):
    pp_off, pp, pc_off, pc, _ = T.lists(theta)
    return set(pc[pc_off[g]:pc_off[g + 1]].tolist()), set(pp[pp_off[g]:pp_off[g + 1]].tolist())


def test_mac_accepts_strictly_below_theta_d():
    T, g, pair, leaves, L = _mac_setup()
    assert T.box()[3] == L
    # theta = L / 2 makes l_3^2 == theta^2 d^2 exactly in FP64 (d^2 = 1/16,
    # theta^2 = fl(L^2) / 4, l_3^2 = fl(L^2) / 64): equality does not accept,
    # so the level-3 node is opened and its two leaves (level 4, side L/16)
    # are accepted instead.
    th = L / 2
    assert (L / 8) ** 2 == (th * th) * (1 / 16)
    pc, pp = _pc_of(T, g, th)
    assert pair[3] not in pc and pair[2] not in pc and pair[1] not in pc
    assert set(leaves) <= pc
    # one ulp above: the level-3 node is accepted (its parents are not)
    pc, pp = _pc_of(T, g, np.nextafter(th, 1.0))
    assert pair[3] in pc and pair[2] not in pc and pair[1] not in pc
    assert not (set(leaves) & pc)


def test_mac_uses_box_distance_and_geometric_side():
    T, g, pair, leaves, L = _mac_setup()
    lc3, d = L / 8, 0.25
    # just below l_3 / d: the level-3 node is opened.  A centre-to-centre
    # distance (0.296875 here) or the pair's tight side (6/64 < l_3) in place
    # of l_3 would accept it.
    pc, _ = _pc_of(T, g, lc3 / d * (1 - 1e-9))
    assert pair[3] not in pc
    # just above l_2 / d the level-2 node (side L/4) is accepted, and only it
    pc, _ = _pc_of(T, g, (L / 4) / d * (1 + 1e-9))
    assert pair[2] in pc and pair[3] not in pc and pair[1] not in pc
    # between l_3 / d and l_2 / d: level 3 accepted, level 2 not
    pc, _ = _pc_of(T, g, 0.75 * L)
    assert pair[3] in pc and pair[2] not in pc


def test_mac_cell_holding_the_group_never_accepted():
    # every node that contains a member of the group has d = 0 and is opened,
    # whatever theta
    T, g, pair, leaves, L = _mac_setup()
    nd = T.nodes()
    gnode = T.groups()[g]
    anc = [k for k in range(T.n_nodes)
           if nd["begin"][k] <= nd["begin"][gnode] and nd["end"][gnode] <= nd["end"][k]]
    for th in (0.5, 2.0, 1e6):
        pc, _ = _pc_of(T, g, th)
        assert not (set(anc) & pc)


# --------------------------------------------------------------------------
# Cell softening: the mass-weighted mean of the members' eps^2.  For a cell of
# coincident particles (no quadrupole) the expansion
#   sum_j m_j (r^2 + e_i + e_j)^-1/2 = M (r^2 + e_i + ebar)^-1/2 + O(e^2 / r^5)
# holds to first order in e only with ebar = sum m_j e_j / M, and the
# second-order remainder is (3/8) M Var_m(e) / r^5 (Var_m the mass-weighted
# variance of the e_j).  An unweighted mean, a maximum, or a dropped receiver
# softening e_i leaves a first-order error, which is ~400 times larger here.
# --------------------------------------------------------------------------
def test_cell_softening_is_mass_weighted_mean():
    m1, m2 = 1.0, 3.0
    e1, e2, ei = 0.04, 0.0004, 0.01
    r = 3.0
    p = _pset([(0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (r, 0.0, 0.0)], m=[m1, m2, 1e-30],
              eps2=[e1, e2, ei])
    e1, e2, ei = (float(np.float32(v)) for v in (e1, e2, ei))
    T = oracle.Tree(p, 1, 1)
    nd = T.nodes()
    pair = [k for k in range(T.n_nodes) if nd["end"][k] - nd["begin"][k] == 2]
    assert nd["eps2bar"][pair[0]] == pytest.approx((m1 * e1 + m2 * e2) / (m1 + m2), rel=1e-15)
    ax, ay, az, pot, npp, npc = T.gravity(1.0, 0.5, True)
    k = 2
    assert npc >= 1
    # the receiver's field from the pair: tree (one accepted cell) vs direct
    d = oracle.direct_gravity(p, 1.0, idx=np.array([k]))
    M = m1 + m2
    ebar = (m1 * e1 + m2 * e2) / M
    var = (m1 * (e1 - ebar) ** 2 + m2 * (e2 - ebar) ** 2) / M
    second = 3.0 / 8.0 * M * var / r ** 5
    diff = pot[k] - d[3][0]
    assert abs(diff) == pytest.approx(second, rel=0.02)
    # the unweighted mean would be off by M (e_mean - ebar) / (2 r^3) at first order
    first = M * abs(0.5 * (e1 + e2) - ebar) / (2 * r ** 3)
    assert first > 100 * second
    # acceleration: the same expansion differentiated, (15/8) M Var / r^6
    assert abs(ax[k] - d[0][0]) == pytest.approx(15.0 / 8.0 * M * var / r ** 6, rel=0.03)


# --------------------------------------------------------------------------
# Signal-velocity viscosity (Monaghan 1997), alpha = 1: a head-on pair with
# given densities, internal energies and kernel sizes, computed by hand.
# --------------------------------------------------------------------------
def test_head_on_pair_viscosity_by_hand():
    # particle 0 at x = 0 moving +1, particle 1 at x = 0.5 moving -1; masses
    # 1 and 2; rho 1 and 2; u 0.9 and 3.6 (gamma 5/3: c = 1 and 2); H = 1 for
    # both (q = 0.5 on both kernels).
    g = {"x": np.array([0.0, 0.5]), "y": np.zeros(2), "z": np.zeros(2),
         "vx": np.array([1.0, -1.0]), "vy": np.zeros(2), "vz": np.zeros(2),
         "m": np.array([1.0, 2.0]), "u": np.array([0.9, 3.6])}
    H = np.array([1.0, 1.0])
    rho = np.array([1.0, 2.0])
    ax, ay, az, dudt, vsig = oracle.sph_force(g, H, rho, GAMMA, 1.0)
    # c_0 = sqrt(10/9 * 0.9) = 1, c_1 = sqrt(10/9 * 3.6) = 2
    # w = v_01 . r_01 / r = (2)(-0.5) / 0.5 = -2 (approaching)
    # v_sig = 1 + 2 - 3 (-2) = 9;  Pi = -1 * 9 * (-2) / (1 + 2) = 6
    # A_0 = P_0 / rho_0^2 = (2/3)(1)(0.9) / 1 = 0.6;  A_1 = (2/3)(2)(3.6) / 4 = 1.2
    # gW at q = 1/2, H = 1: -1155 / (4 pi) * (1 + 5/2) * (1/2)^5 = -1155 * 3.5 / (128 pi)
    gw = -1155.0 * 3.5 / (128.0 * math.pi)
    # a_0 = -m_1 [A_0 gW + A_1 gW + Pi gW] r_01 = -2 (0.6 + 1.2 + 6) gW (-0.5) = 7.8 gW
    assert ax[0] == pytest.approx(7.8 * gw, rel=1e-13)
    # a_1 = -m_0 [A_1 + A_0 + Pi] gW r_10 = -1 (7.8) gW (+0.5) = -3.9 gW
    assert ax[1] == pytest.approx(-3.9 * gw, rel=1e-13)
    # du_0/dt = m_1 [A_0 gW + Pi gW / 2] (v_01 . r_01) = 2 (0.6 + 3) gW (-1) = -7.2 gW
    assert dudt[0] == pytest.approx(-7.2 * gw, rel=1e-13)
    # du_1/dt = m_0 [A_1 + Pi / 2] gW (v_10 . r_10) = 1 (1.2 + 3) gW (-1) = -4.2 gW
    assert dudt[1] == pytest.approx(-4.2 * gw, rel=1e-13)
    assert vsig[0] == pytest.approx(9.0, rel=1e-15) and vsig[1] == pytest.approx(9.0, rel=1e-15)
    assert ay[0] == 0.0 and az[1] == 0.0
    # receding pair: no viscosity, v_sig = c_0 + c_1
    g2 = dict(g, vx=np.array([-1.0, 1.0]))
    ax2, _, _, dudt2, vsig2 = oracle.sph_force(g2, H, rho, GAMMA, 1.0)
    assert ax2[0] == pytest.approx(-2.0 * 1.8 * gw * -0.5, rel=1e-13)
    assert vsig2[0] == pytest.approx(3.0, rel=1e-15)
    # pair beyond both kernels (r >= max H): no interaction, v_sig = own c
    g3 = dict(g, x=np.array([0.0, 1.0]))
    ax3, _, _, du3, vs3 = oracle.sph_force(g3, H, rho, GAMMA, 1.0)
    assert ax3[0] == 0.0 and du3[0] == 0.0 and vs3[0] == pytest.approx(1.0) and vs3[1] == pytest.approx(2.0)


def test_unequal_kernels_use_each_side():
    # H_0 = 1, H_1 = 0.4 at r = 0.5: particle 1's kernel does not reach 0, so
    # only the A_0 gW(H_0) term and half the viscosity gradient remain; the
    # pair still interacts (r < max(H_0, H_1)).
    g = {"x": np.array([0.0, 0.5]), "y": np.zeros(2), "z": np.zeros(2),
         "vx": np.zeros(2), "vy": np.zeros(2), "vz": np.zeros(2),
         "m": np.array([1.0, 2.0]), "u": np.array([0.9, 3.6])}
    H = np.array([1.0, 0.4])
    rho = np.array([1.0, 2.0])
    ax, _, _, _, _ = oracle.sph_force(g, H, rho, GAMMA, 1.0)
    gw = -1155.0 * 3.5 / (128.0 * math.pi)
    assert ax[0] == pytest.approx(-2.0 * 0.6 * gw * -0.5, rel=1e-13)
    assert ax[1] == pytest.approx(-1.0 * 0.6 * gw * 0.5, rel=1e-13)


# --------------------------------------------------------------------------
# Energy audit and equation of state.
# --------------------------------------------------------------------------
def test_energy_by_hand():
    m = np.array([2.0, 3.0])
    v = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 1.0]])
    # two bodies 5 apart, pair softening 0.5^2 + 0.5^2: W counts the pair once
    p = _pset([(0.0, 0.0, 0.0), (3.0, 4.0, 0.0)], m=m, eps2=[0.25, 0.25])
    _, _, _, pot = oracle.direct_gravity(p, 2.0)
    K, W, U = oracle.energy(m, v, pot, u_gas=np.array([0.5, 0.25]), m_gas=m)
    assert K == 0.5 * (2.0 * 25.0 + 3.0 * 1.0)
    assert W == pytest.approx(-2.0 * 2.0 * 3.0 / math.sqrt(25.5), rel=1e-15)
    assert U == 2.0 * 0.5 + 3.0 * 0.25


def test_eos_by_hand_and_sound_speed_identity():
    P, c = oracle.eos(np.array([2.0]), np.array([0.9]), GAMMA)
    assert P[0] == pytest.approx(1.2, rel=1e-15) and c[0] == pytest.approx(1.0, rel=1e-15)
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.1, 10.0, 100)
    u = rng.uniform(0.01, 100.0, 100)
    for gam in (5.0 / 3.0, 1.4):
        P, c = oracle.eos(rho, u, gam)
        assert np.allclose(c * c, gam * P / rho, rtol=1e-14)      # adiabatic sound speed
        assert np.allclose(P / (rho * u), gam - 1.0, rtol=1e-14)  # ideal gas
