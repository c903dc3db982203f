"""GPU parity of the tree build, interaction lists and gravity kernels against
the FP64 oracle (through the C ABI).

Tolerances
----------
* keys, permutation, nodes, groups, lists: bit-exact (integer work).
* node moments: mass/centre of mass FP64 (1e-12 relative, summation order);
  quadrupoles are stored in FP32 (2^-24 relative to the largest component).
* forces: the kernel rounds group-relative coordinates and pair terms to FP32
  and sums each tile (<= 256 terms) in FP32, tiles in FP64.  With unit
  roundoff u = 6e-8, a tile sum of n terms carries a relative error of order
  sqrt(n) u ~ 1e-6 of the summed magnitude, so the per-particle relative error
  against the FP64 result is of order 1e-6 and is bounded by 1e-5 at p99 (the
  direct-sum target).  The FP64 build of the same kernel must agree to 1e-12.
"""
import numpy as np
import pytest

import ics
import oracle

pytestmark = pytest.mark.gpu


def _dev(gx, d):
    return gx.ParticleSet.from_numpy(d)


def _zeros(n, k=4):
    import torch
    return [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(k)]


def _relerr(a, b):
    an = np.sqrt(b[0] ** 2 + b[1] ** 2 + b[2] ** 2)
    return np.sqrt((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2 + (a[2] - b[2]) ** 2) / an


def _np(ts):
    return [t.cpu().numpy() for t in ts]


@pytest.fixture(scope="module")
def eng(gx):
    e = gx.Engine(0)
    yield e
    e.close()


def _check_tree(gx, eng, d, n_leaf, n_group):
    p = _dev(gx, d)
    st = eng.tree_build(p, gx.GX_TREE_ALL, n_leaf, n_group)
    T = oracle.Tree(d, n_leaf, n_group)
    key, perm = T.sorted()
    g = eng.tree_export(gx.GX_TREE_ALL, p.n)
    assert np.array_equal(g["box"], T.box())
    assert np.array_equal(g["keys"], key)
    assert np.array_equal(g["perm"].astype(np.int64), perm)
    nd = T.nodes()
    assert st["n_nodes"] == T.n_nodes and st["n_groups"] == T.n_groups
    for k in ("begin", "end", "next", "level", "leaf"):
        assert np.array_equal(g[k].astype(np.int64), nd[k].astype(np.int64)), k
    assert np.array_equal(g["lo"], nd["lo"]) and np.array_equal(g["hi"], nd["hi"])
    assert np.allclose(g["mass"], nd["mass"], rtol=1e-12, atol=0)
    scale = np.abs(nd["com"]).max()
    assert np.max(np.abs(g["com"] - nd["com"])) <= 1e-12 * scale
    # quadrupoles are stored in FP32; their natural scale is M * side^2
    side = g["box"][3] * np.ldexp(1.0, -nd["level"].astype(np.int64))
    qs = (nd["mass"] * side * side)[:, None]
    assert np.max(np.abs(g["quad"] - nd["quad"]) / qs) < 1e-6
    assert np.allclose(g["eps2bar"], nd["eps2bar"], rtol=1e-6)
    assert np.array_equal(g["groups"].astype(np.int64), T.groups())
    return p, T


@pytest.mark.parametrize("case", ["plummer", "disk", "tiny", "ragged"])
def test_tree_matches_oracle(gx, eng, case):
    if case == "plummer":
        d, nl, ngr = ics.plummer(8192, 1), 16, 256
    elif case == "disk":
        d, nl, ngr = ics.disk_galaxy(60000, 3), 16, 256
    elif case == "tiny":
        d, nl, ngr = ics.plummer(10, 4), 16, 256
    else:
        d, nl, ngr = ics.plummer(5001, 8), 7, 100
    _check_tree(gx, eng, d, nl, ngr)


def test_tree_duplicate_positions(gx, eng):
    # coincident particles: equal keys, stable order, level-21 leaves
    d = ics.plummer(3000, 12)
    for k in ("x", "y", "z"):
        d[k][1000:1100] = d[k][5]
    _check_tree(gx, eng, d, 16, 64)


def _list_sets(T, nd, lists_o, g_lists):
    pp_off, pp, pc_off, pc, npp = lists_o
    for gi in range(T.n_groups):
        oc = np.sort(pc[pc_off[gi]:pc_off[gi + 1]])
        gc = np.sort(g_lists["pc"][g_lists["pc_off"][gi]:g_lists["pc_off"][gi + 1]].astype(np.int64))
        assert np.array_equal(oc, gc), f"pc list of group {gi}"
        leaves = pp[pp_off[gi]:pp_off[gi + 1]]
        o_slots = np.concatenate([np.arange(nd["begin"][l], nd["end"][l]) for l in leaves])
        r = slice(g_lists["pp_off"][gi], g_lists["pp_off"][gi + 1])
        g_slots = np.concatenate([np.arange(b, e) for b, e in
                                  zip(g_lists["pp_begin"][r], g_lists["pp_end"][r])])
        assert np.array_equal(np.sort(o_slots), np.sort(g_slots)), f"pp list of group {gi}"


@pytest.mark.parametrize("n,theta", [(8192, 0.5), (40000, 0.5), (20000, 0.3), (20000, 0.9)])
def test_lists_match_oracle(gx, eng, n, theta):
    d = ics.disk_galaxy(n, 5) if n != 8192 else ics.plummer(n, 1)
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(p.n)
    eng.gravity_forces(p, 1.0, theta, gx.GX_QUAD, *out)
    T = oracle.Tree(d, 16, 256)
    _list_sets(T, T.nodes(), T.lists(theta), eng.gravity_lists())


def test_direct_fp32_vs_fp64_oracle(gx, eng):
    # FP32 relative-coordinate direct sum vs FP64 direct sum: p99 <= 1e-5.
    d = ics.plummer(8192, 1)
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(p.n)
    st = eng.gravity_forces(p, 1.0, 0.5, gx.GX_DIRECT, *out)
    assert st["n_pp"] == 8192 * 8192 and st["n_pc"] == 0
    ax, ay, az, pot = _np(out)
    o = oracle.direct_gravity(d)
    err = _relerr((ax, ay, az), o[:3])
    assert np.percentile(err, 99) <= 1e-5
    assert np.median(err) <= 2e-6
    assert np.max(np.abs(pot - o[3]) / np.abs(o[3])) <= 1e-5
    m = d["m"]
    scale = np.sum(m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2))
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) <= 1e-6 * scale


@pytest.mark.parametrize("mode", ["tree_quad", "tree_mono", "direct", "tree_fp64"])
def test_one_and_two_particle_systems(gx, eng, mode):
    # Degenerate systems with closed forms (Eq. 1): a lone particle feels no
    # force and no potential (its own pair is excluded), and two particles
    # attract along their separation with the softened law, softening
    # eps_i^2 + eps_j^2 (values exact in the FP32 storage of eps^2).
    flags = {"tree_quad": gx.GX_QUAD, "tree_mono": 0, "direct": gx.GX_DIRECT,
             "tree_fp64": gx.GX_QUAD | gx.GX_PREC_FP64}[mode]
    tol = 1e-12 if mode == "tree_fp64" else 1e-5
    G = 1.0
    zero = lambda n: np.zeros(n)
    d1 = dict(x=np.array([0.25]), y=np.array([-0.5]), z=np.array([0.125]), vx=zero(1),
              vy=zero(1), vz=zero(1), m=np.array([2.0]), eps2=np.array([1 / 64], np.float32))
    p = _dev(gx, d1)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(1)
    eng.gravity_forces(p, G, 0.5, flags, *out)
    assert all(float(v[0]) == 0.0 for v in _np(out))
    x, y, z = np.array([0.25, 0.55]), np.array([-0.5, -0.7]), np.array([0.125, 0.225])
    m, e2 = np.array([2.0, 0.5]), np.array([1 / 64, 1 / 256], np.float32)
    d2 = dict(x=x, y=y, z=z, vx=zero(2), vy=zero(2), vz=zero(2), m=m, eps2=e2)
    p = _dev(gx, d2)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(2)
    eng.gravity_forces(p, G, 0.5, flags, *out)
    ax, ay, az, pot = _np(out)
    o = oracle.direct_gravity(d2, G)
    for i, j in ((0, 1), (1, 0)):
        r = np.array([x[j] - x[i], y[j] - y[i], z[j] - z[i]])
        s2 = r @ r + float(e2[i]) + float(e2[j])
        a = G * m[j] / s2 ** 1.5 * r
        phi = -G * m[j] / np.sqrt(s2)
        assert np.max(np.abs(np.array([ax[i], ay[i], az[i]]) - a)) <= tol * np.linalg.norm(a)
        assert abs(pot[i] - phi) <= tol * abs(phi)
        assert np.max(np.abs(np.array([o[0][i], o[1][i], o[2][i]]) - a)) <= 1e-14 * np.linalg.norm(a)
        assert abs(o[3][i] - phi) <= 1e-14 * abs(phi)


def test_direct_fp64_mode_matches_oracle(gx, eng):
    d = ics.plummer(4096, 2)
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(p.n)
    eng.gravity_forces(p, 1.0, 0.5, gx.GX_DIRECT | gx.GX_PREC_FP64, *out)
    ax, ay, az, pot = _np(out)
    o = oracle.direct_gravity(d)
    assert np.max(_relerr((ax, ay, az), o[:3])) <= 1e-12
    assert np.max(np.abs(pot - o[3]) / np.abs(o[3])) <= 1e-12


# n_group 600: groups above one 256-lane block (several receiver passes);
# n_group 16: many receiver slices per block.
@pytest.mark.parametrize("quad,ngr", [(True, 256), (False, 256), (True, 600), (True, 16)])
def test_tree_fp32_vs_oracle_tree(gx, eng, quad, ngr):
    # Same lists on both sides: only FP32 rounding separates them.
    d = ics.disk_galaxy(60000, 6)
    G = ics.G_KPC
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, ngr)
    out = _zeros(p.n)
    flags = gx.GX_QUAD if quad else 0
    st = eng.gravity_forces(p, G, 0.5, flags, *out)
    ax, ay, az, pot = _np(out)
    t = oracle.Tree(d, 16, ngr).gravity(G, 0.5, quad)
    err = _relerr((ax, ay, az), t[:3])
    assert np.percentile(err, 99) <= 1e-5
    assert np.max(np.abs(pot - t[3]) / np.abs(t[3])) <= 1e-5
    assert st["n_pp"] == t[4] and st["n_pc"] == t[5]
    # FP64 pair arithmetic: what remains is the FP32 storage of cell quadrupoles
    # and mean softening (2^-24 relative on terms well below the total): 1e-7.
    out64 = _zeros(p.n)
    eng.gravity_forces(p, G, 0.5, flags | gx.GX_PREC_FP64, *out64)
    a64 = _np(out64)
    assert np.max(_relerr(a64[:3], t[:3])) <= 1e-7
    assert np.max(np.abs(a64[3] - t[3]) / np.abs(t[3])) <= 1e-8


def test_tree_1m_disk_error_vs_direct(gx, eng):
    # The 1M-particle disk: GPU FP32 tree (theta 0.5, quadrupoles, n_g 256) against
    # the FP64 direct sum on a seeded sample of receivers: p99 <= 1e-3.
    d = ics.disk_galaxy(1_000_000, 3)
    G = ics.G_KPC
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(p.n)
    eng.gravity_forces(p, G, 0.5, gx.GX_QUAD, *out)
    ax, ay, az, pot = _np(out)
    idx = ics.sample_indices(p.n, 2000, 17)
    o = oracle.direct_gravity(d, G, idx)
    err = _relerr((ax[idx], ay[idx], az[idx]), o[:3])
    assert np.percentile(err, 99) <= 1e-3
    assert np.median(err) <= 3e-4


def test_stale_and_unbuilt_errors(gx):
    import torch
    e = gx.Engine(0)
    d = ics.plummer(1000, 3)
    p = _dev(gx, d)
    out = _zeros(p.n)
    with pytest.raises(gx.GxError) as ei:
        e.gravity_forces(p, 1.0, 0.5, gx.GX_QUAD, *out)
    assert ei.value.code == -4
    e.tree_build(p)
    q = _dev(gx, d)
    with pytest.raises(gx.GxError) as ei:
        e.gravity_forces(q, 1.0, 0.5, gx.GX_QUAD, *out)
    assert ei.value.code == -5
    with pytest.raises(gx.GxError):
        e.tree_build(p, gx.GX_TREE_ALL, 0, 256)
    e.close()


def test_kick_drift_matches_oracle(gx, eng):
    import torch
    rng = np.random.default_rng(3)
    n, ng = 5000, 1200
    d = {k: rng.normal(size=n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    d["m"] = np.full(n, 1.0 / n)
    a = rng.normal(size=(3, n))
    u = rng.uniform(1, 2, ng)
    du = rng.normal(size=ng)
    p = _dev(gx, d)
    A = [torch.as_tensor(a[k], device="cuda") for k in range(3)]
    U = torch.as_tensor(u, device="cuda")
    DU = torch.as_tensor(du, device="cuda")
    vp = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    up = torch.zeros(ng, dtype=torch.float64, device="cuda")
    dt = 0.01
    eng.kick_drift(p, dt / 2, dt, *A, u=U, dudt=DU, vpred=vp, upred=up)
    x0 = np.stack([d["x"], d["y"], d["z"]])
    v0 = np.stack([d["vx"], d["vy"], d["vz"]])
    x, v, un, vpred, upred = oracle.kick_drift(x0, v0, a, dt / 2, dt, u, du)
    got_x = np.stack(_np([p.x, p.y, p.z]))
    got_v = np.stack(_np([p.vx, p.vy, p.vz]))
    assert np.allclose(got_x, x, rtol=1e-14, atol=1e-15)
    assert np.allclose(got_v, v, rtol=1e-14, atol=1e-15)
    assert np.allclose(vp.cpu().numpy().reshape(3, n), vpred, rtol=1e-14, atol=1e-15)
    assert np.allclose(U.cpu().numpy(), un, rtol=1e-14)
    assert np.allclose(up.cpu().numpy(), upred, rtol=1e-14)


def test_energy_matches_oracle(gx, eng):
    import torch
    d = ics.plummer(8192, 1)
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    out = _zeros(p.n)
    eng.gravity_forces(p, 1.0, 0.5, gx.GX_DIRECT | gx.GX_PREC_FP64, *out)
    ug = np.linspace(1, 2, 100)
    mg = np.full(100, 0.01)
    K, W, U = eng.energy(p, out[3], torch.as_tensor(mg, device="cuda"),
                         torch.as_tensor(ug, device="cuda"))
    o = oracle.direct_gravity(d)
    Ko, Wo, Uo = oracle.energy(d["m"], np.stack([d["vx"], d["vy"], d["vz"]]), o[3], ug, mg)
    assert K == pytest.approx(Ko, rel=1e-13)
    assert W == pytest.approx(Wo, rel=1e-11)
    assert U == pytest.approx(Uo, rel=1e-13)
    # deterministic reduction: identical on repeat
    assert eng.energy(p, out[3], torch.as_tensor(mg, device="cuda"),
                      torch.as_tensor(ug, device="cuda")) == (K, W, U)


def test_one_leapfrog_step_plummer(gx, eng):
    # One KDK step of the 8,192-body Plummer sphere (direct sum, dt = 1e-3) on the
    # GPU against the same step by the oracle: positions/velocities to 1e-9.
    import torch
    d = ics.plummer(8192, 1)
    dt = 1e-3
    p = _dev(gx, d)
    acc = _zeros(p.n)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    eng.gravity_forces(p, 1.0, 0.5, gx.GX_DIRECT, *acc)
    eng.kick_drift(p, dt / 2, dt, *acc[:3])
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    eng.gravity_forces(p, 1.0, 0.5, gx.GX_DIRECT, *acc)
    eng.kick_drift(p, dt / 2, 0.0, *acc[:3])
    o = oracle.direct_gravity(d)
    x, v, _, _, _ = oracle.kick_drift(np.stack([d["x"], d["y"], d["z"]]),
                                      np.stack([d["vx"], d["vy"], d["vz"]]), np.stack(o[:3]),
                                      dt / 2, dt)
    d2 = dict(d, x=x[0], y=x[1], z=x[2])
    o2 = oracle.direct_gravity(d2)
    _, v, _, _, _ = oracle.kick_drift(x, v, np.stack(o2[:3]), dt / 2, 0.0)
    gx_x = np.stack(_np([p.x, p.y, p.z]))
    gx_v = np.stack(_np([p.vx, p.vy, p.vz]))
    assert np.max(np.abs(gx_x - x)) <= 1e-9
    amax = np.max(np.abs(np.stack(o[:3])))
    assert np.max(np.abs(gx_v - v)) <= 1e-5 * dt * amax


def test_list_slots_equal_two_pass_and_fall_back(gx, eng):
    # The first call builds the lists in two passes (count, scan, fill) with
    # the stackless walk; the next call on the same tree builds them in one
    # wave-cooperative pass into per-group slots sized from the first: the
    # same lists as sets (in another order), so the same forces up to FP32
    # summation order.  A call whose lists outgrow the slots (smaller theta)
    # takes the two-pass path again; every call matches the oracle's lists.
    d = ics.disk_galaxy(30000, 6)
    p = _dev(gx, d)
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    runs = []
    for theta in (0.5, 0.5, 0.3, 0.3):
        out = _zeros(p.n)
        eng.gravity_forces(p, 1.0, theta, gx.GX_QUAD, *out)
        runs.append((_np(out), eng.gravity_lists()))
    T = oracle.Tree(d, 16, 256)
    for k, theta in enumerate((0.5, 0.5, 0.3, 0.3)):
        _list_sets(T, T.nodes(), T.lists(theta), runs[k][1])
    for i, j in ((0, 1), (2, 3)):
        a, b = runs[i][0], runs[j][0]
        err = _relerr(b[:3], a[:3])
        assert np.percentile(err, 99) <= 1e-6 and err.max() <= 1e-5
        assert np.max(np.abs(b[3] - a[3]) / np.abs(a[3])) <= 1e-6


@pytest.mark.parametrize("limit", ["tiny", "half"])
def test_walk_small_stack_overflow_retries_with_large_stack(gx, limit):
    # The first calls on a tree learn the list slot sizes (two-pass, then the
    # one-pass walk).  With the walk's small stack limited
    # (gx_set_walk_stack_limit) to 24 entries (every group overflows it) or to
    # half the deepest stack of the previous call (only the deeper groups do),
    # the next call tries that small stack first: the walk stops pushing in
    # those groups and flags them while the lists still fit their slots, so
    # the call walks once more with the large stack and stays on the one-pass
    # path, with the same lists in the same order as the call before it: the
    # same forces bit for bit, and the oracle's lists as sets.
    d = ics.disk_galaxy(30000, 6)
    e = gx.Engine(0)
    p = _dev(gx, d)
    e.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    res = []
    for k in range(5):
        if k == 4:
            cap = 24 if limit == "tiny" else res[3][1]["n_iter_max"] // 2
            e.set_walk_stack_limit(cap)
        out = _zeros(p.n)
        st = e.gravity_forces(p, 1.0, 0.5, gx.GX_QUAD, *out)
        res.append((_np(out), st, e.gravity_lists()))
    e.set_walk_stack_limit(0)
    e.close()
    (a, sa, _), (b, sb, lb) = res[3], res[4]
    assert sa["n_rewalk"] == 0 and sb["n_rewalk"] == 0
    assert sb["n_iter_max"] == sa["n_iter_max"] > cap
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    T = oracle.Tree(d, 16, 256)
    _list_sets(T, T.nodes(), T.lists(0.5), lb)
