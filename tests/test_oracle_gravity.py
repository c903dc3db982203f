"""Pins of the FP64 gravity oracle (direct sum and tree) against closed forms,
invariants and limits the paper's Eq. 1 and the Barnes-Hut method fix."""
import math

import numpy as np
import pytest

import ics
import oracle


def _two(x2, m2=0.7, e1=0.01, e2=0.02):
    return {"x": np.array([0.0, x2[0]]), "y": np.array([0.0, x2[1]]),
            "z": np.array([0.0, x2[2]]), "m": np.array([1.3, m2]),
            "eps2": np.array([e1, e2], np.float32)}


def test_two_body_closed_form():
    # Eq. 1 for one pair: |a_1| = G m_2 r / (r^2 + eps_1^2 + eps_2^2)^{3/2}, towards body 2.
    p = _two((3.0, 4.0, 0.0))
    G = 2.5
    ax, ay, az, pot = oracle.direct_gravity(p, G)
    e = float(np.float32(0.01)) + float(np.float32(0.02))
    s = (25.0 + e) ** 1.5
    assert ax[0] == pytest.approx(G * 0.7 * 3.0 / s, rel=1e-14)
    assert ay[0] == pytest.approx(G * 0.7 * 4.0 / s, rel=1e-14)
    assert az[0] == 0.0
    assert ax[1] == pytest.approx(-G * 1.3 * 3.0 / s, rel=1e-14)
    assert pot[0] == pytest.approx(-G * 0.7 / math.sqrt(25.0 + e), rel=1e-14)
    assert pot[1] == pytest.approx(-G * 1.3 / math.sqrt(25.0 + e), rel=1e-14)


def test_momentum_conservation_direct():
    p = ics.plummer(2048, 11)
    ax, ay, az, _ = oracle.direct_gravity(p)
    m = p["m"]
    scale = np.sum(m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2))
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) <= 1e-14 * scale


def test_plummer_binding_energy_closed_form():
    # W = 1/2 sum m phi -> -3 pi G M^2 / (32 a) for a Plummer sphere.
    p = ics.plummer(8192, 1)
    _, _, _, pot = oracle.direct_gravity(p)
    W = 0.5 * np.sum(p["m"] * pot)
    assert W == pytest.approx(-3.0 * math.pi / 32.0, rel=0.02)


def test_plummer_potential_profile():
    # phi(r) = -G M / sqrt(r^2 + a^2) on average over the sample.
    p = ics.plummer(8192, 1)
    _, _, _, pot = oracle.direct_gravity(p)
    r = np.sqrt(p["x"] ** 2 + p["y"] ** 2 + p["z"] ** 2)
    ratio = pot / (-1.0 / np.sqrt(r * r + 1.0))
    assert abs(np.mean(ratio) - 1.0) < 0.01


def test_plummer_virial():
    p = ics.plummer(8192, 1)
    _, _, _, pot = oracle.direct_gravity(p)
    K = 0.5 * np.sum(p["m"] * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2))
    W = 0.5 * np.sum(p["m"] * pot)
    assert 2 * K / abs(W) == pytest.approx(1.0, abs=0.06)


def _shell(n=6000, R=1.0):
    k = np.arange(n) + 0.5
    cz = 1 - 2 * k / n
    ph = math.pi * (1 + 5 ** 0.5) * k
    s = np.sqrt(1 - cz * cz)
    return R * s * np.cos(ph), R * s * np.sin(ph), R * cz


def test_shell_theorem():
    # Outside a uniform shell the field is G M / r^2; inside it vanishes.
    sx, sy, sz = _shell()
    for r0, expect in ((3.0, -1.0 / 9.0), (0.3, 0.0)):
        p = {"x": np.append(sx, r0), "y": np.append(sy, 0.0), "z": np.append(sz, 0.0),
             "m": np.append(np.full(sx.size, 1.0 / sx.size), 0.0),
             "eps2": np.zeros(sx.size + 1, np.float32)}
        ax, ay, az, pot = oracle.direct_gravity(p, idx=np.array([sx.size]))
        assert ax[0] == pytest.approx(expect, abs=2e-4)
        assert abs(ay[0]) < 2e-4 and abs(az[0]) < 2e-4


def test_tree_theta_zero_is_direct():
    p = ics.plummer(2048, 5)
    d = oracle.direct_gravity(p)
    T = oracle.Tree(p, 16, 256)
    t = T.gravity(1.0, 1e-12, True)
    for k in range(4):
        assert np.max(np.abs(t[k] - d[k])) <= 1e-13 * np.max(np.abs(d[k]))
    assert t[5] == 0 and t[4] == 2048 * 2048


def test_tree_lists_cover_every_particle_once():
    # Every group's list (pp leaves + accepted cells) partitions the particle set.
    p = ics.disk_galaxy(20000, 9)
    T = oracle.Tree(p, 16, 256)
    nd = T.nodes()
    pp_off, pp, pc_off, pc, npp = T.lists(0.5)
    for g in range(T.n_groups):
        cover = np.zeros(T.n, np.int32)
        for leaf in pp[pp_off[g]:pp_off[g + 1]]:
            cover[nd["begin"][leaf]:nd["end"][leaf]] += 1
        for c in pc[pc_off[g]:pc_off[g + 1]]:
            cover[nd["begin"][c]:nd["end"][c]] += 1
        assert np.all(cover == 1)
        mass = (np.sum(nd["mass"][pc[pc_off[g]:pc_off[g + 1]]])
                + np.sum(nd["mass"][pp[pp_off[g]:pp_off[g + 1]]]))
        assert mass == pytest.approx(np.sum(p["m"]), rel=1e-12)


def test_tree_structure_invariants():
    p = ics.plummer(8192, 1)
    T = oracle.Tree(p, 16, 256)
    nd = T.nodes()
    cnt = nd["end"] - nd["begin"]
    # leaves hold at most n_leaf particles unless at the finest level; groups partition.
    assert np.all((cnt[nd["leaf"] == 1] <= 16) | (nd["level"][nd["leaf"] == 1] == 21))
    assert np.all(cnt[nd["leaf"] == 0] > 16)
    g = T.groups()
    ge = np.sort(nd["begin"][g])
    assert ge[0] == 0 and np.all(np.diff(np.concatenate([nd["begin"][g], [T.n]])) > 0)
    assert np.all(cnt[g] <= 256)
    # the parent of every group holds more than n_g particles (maximality)
    for gi in g[:50]:
        if gi == 0:
            continue
        par = [k for k in range(gi) if nd["begin"][k] <= nd["begin"][gi] and nd["next"][k] > gi]
        assert cnt[max(par)] > 256


def test_morton_octant_order():
    # The 8 octant corners of a cube sort as octant index 4 bx + 2 by + bz.
    pts = np.array([(bx, by, bz) for bx in (0.1, 0.9) for by in (0.1, 0.9) for bz in (0.1, 0.9)])
    rng = np.random.default_rng(0)
    perm = rng.permutation(8)
    p = {"x": pts[perm, 0], "y": pts[perm, 1], "z": pts[perm, 2]}
    keys = oracle.morton_keys(p)
    order = perm[np.argsort(keys)]
    assert list(order) == list(range(8))


def test_morton_key_bits():
    # Key bits interleave the 21-bit cell coordinates with x most significant.
    p = ics.plummer(1000, 3)
    box = oracle.root_box(p)
    keys = oracle.morton_keys(p, box)
    scale = 2097152.0 / box[3]
    for i in range(0, 1000, 97):
        cells = [min(2097151, int(math.floor((p[a][i] - box[k]) * scale)))
                 for k, a in enumerate("xyz")]
        dec = [0, 0, 0]
        for b in range(21):
            for k in range(3):
                dec[k] |= int((int(keys[i]) >> (3 * b + 2 - k)) & 1) << b
        assert dec == cells


def _far_field(T, node, d, quad):
    nd = T.nodes()
    com = nd["com"][node]
    r = com + np.array([d, 0.31 * d, -0.17 * d])
    return r, T.node_field(node, r, quad)


def test_quadrupole_convergence_order():
    # Relative error of a cell's expansion falls ~8x per distance doubling with the
    # quadrupole (third order) and ~4x with the monopole alone (second order).
    p = ics.plummer(4096, 21)
    p["eps2"] = np.zeros(4096, np.float32)
    T = oracle.Tree(p, 16, 256)
    nd = T.nodes()
    node = int(np.argmax(np.where(nd["level"] == 3, nd["end"] - nd["begin"], 0)))
    mem = slice(nd["begin"][node], nd["end"][node])
    key, perm = T.sorted()
    ids = perm[mem]
    size = np.max(nd["hi"][node] - nd["lo"][node])
    ratios = {}
    for quad in (False, True):
        errs = []
        for d in (4 * size, 8 * size, 16 * size):
            r, f = _far_field(T, node, d, quad)
            q = {"x": np.append(p["x"][ids], r[0]), "y": np.append(p["y"][ids], r[1]),
                 "z": np.append(p["z"][ids], r[2]), "m": np.append(p["m"][ids], 0.0),
                 "eps2": np.zeros(ids.size + 1, np.float32)}
            ax, ay, az, pot = oracle.direct_gravity(q, idx=np.array([ids.size]))
            a = np.array([ax[0], ay[0], az[0]])
            errs.append(np.linalg.norm(f[:3] - a) / np.linalg.norm(a))
        ratios[quad] = (errs[0] / errs[1], errs[1] / errs[2])
    assert all(2.8 < x < 5.5 for x in ratios[False])
    assert all(5.5 < x < 11.0 for x in ratios[True])


def test_quadrupole_two_point_masses():
    # Two masses m at +-b on the x axis: Q_xx = 4 m b^2, Q_yy = Q_zz = -2 m b^2.
    b, m = 0.3, 2.0
    p = {"x": np.array([-b, b]), "y": np.zeros(2), "z": np.zeros(2), "m": np.array([m, m]),
         "eps2": np.zeros(2, np.float32)}
    T = oracle.Tree(p, 1, 256)
    nd = T.nodes()
    q = nd["quad"][0]
    assert q[0] == pytest.approx(4 * m * b * b, rel=1e-14)
    assert q[1] == pytest.approx(-2 * m * b * b, rel=1e-14)
    assert q[2] == pytest.approx(-2 * m * b * b, rel=1e-14)
    assert np.all(np.abs(q[3:]) < 1e-15)
    assert nd["mass"][0] == 2 * m and np.allclose(nd["com"][0], 0.0)


@pytest.mark.parametrize("quad,bound", [(True, 1e-3), (False, 3e-3)])
def test_tree_error_vs_direct_plummer(quad, bound):
    p = ics.plummer(8192, 1)
    d = oracle.direct_gravity(p)
    t = oracle.Tree(p, 16, 256).gravity(1.0, 0.5, quad)
    a = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    err = np.sqrt((t[0] - d[0]) ** 2 + (t[1] - d[1]) ** 2 + (t[2] - d[2]) ** 2) / a
    assert np.percentile(err, 99) <= bound


def test_tree_error_vs_direct_disk_1m():
    # The 1M-particle disk galaxy at theta = 0.5 with quadrupoles, n_g = 256:
    # relative force error vs the FP64 direct sum, p99 <= 1e-3 (sampled receivers).
    p = ics.disk_galaxy(1_000_000, 3)
    G = ics.G_KPC
    idx = ics.sample_indices(p["x"].size, 1000, 17)
    d = oracle.direct_gravity(p, G, idx)
    t = oracle.Tree(p, 16, 256).gravity(G, 0.5, True)
    a = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    err = np.sqrt((t[0][idx] - d[0]) ** 2 + (t[1][idx] - d[1]) ** 2 + (t[2][idx] - d[2]) ** 2) / a
    assert np.percentile(err, 99) <= 1e-3
    assert np.median(err) <= 3e-4
