#!/usr/bin/env python
"""Benchmark: one shared-timestep step of the N-body/SPH hot path on the
16M-particle synthetic disk galaxy (8e6 stars, 6.4e6 halo, 1.6e6 gas;
theta = 0.5 with quadrupoles, groups of <= 256, SPH with 64 neighbours,
dt = 2,000 yr), on one MI355X.

A step is the whole hot path: half kick + drift (FP64), gravity tree build,
interaction lists and pairwise gravity (FP32 group-relative), gas tree build,
kernel size + density, hydro force, second half kick, FP64 energy audit.

Each step also hands 64 supernova regions (60 pc boxes around seeded disk
stars) to the surrogate -- extract, voxelize, U-Net inference, resample --
and replaces returned regions by particle ID 50 steps later (with the trained
weights when their file exists, else a random initialisation whose
predictions all fail the trust check and fall back).

Prints ONE JSON line.  ``value`` = gravity interactions (particle-particle +
particle-cell) per second of whole-step wall time.  ``roofline`` reports the
dominant kernel (pairwise gravity) against the FP32 vector peak, timed live
with HIP events on the library's stream.  ``sn_region`` compares, for 64 SN
cubes of 1 Msun particles, the plain small-timestep SPH to 0.1 Myr with the
surrogate path on the same cubes, and the network's inference throughput at
batch 256.  ``galaxy_0p1Myr`` compares 0.1 Myr of the disk with the
surrogate (50 global steps) against a shared step held to the SN regions'
Courant step.  The CPU-baseline leg (skipped by --no-cpu) is the only part
that runs the FP64 oracle: ``cpu_baseline`` times its tree gravity on a
seeded sample of the same workload's groups, and ``force_error`` gives the
relative force error of the GPU against its direct sum (16M, 1M, Plummer).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interactions/s & s/step at 16M particles; SN region: surrogate vs plain SPH"
YEAR_IN_KPC_TIME = 1.0 / 0.97779e9  # time unit kpc/(km/s) = 0.97779 Gyr
PEAK_FP32 = 157.3e12                 # MI355X FP32 vector, FLOP/s
HBM_PEAK = 8.0e12                    # B/s
TREE_BYTES_PER_PARTICLE = 330        # algorithmic bytes of one tree build per particle
FLOP_PP = 27                         # per particle-particle interaction (Table 4 convention)
FLOP_PC = 63                         # per particle-cell interaction, monopole + quadrupole
FLOP_DENS = 73                       # per SPH density candidate pair evaluation (Table 4)
FLOP_FORCE = 101                     # per SPH force candidate pair (Table 4)

# HBM traffic of one k_grav_force<float,true> launch on this workload, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, WRITE_SIZE in KiB per
# dispatch) scaled by what the same counters read for a reference copy of
# known size (hbm_calib.py beside this script: FETCH_SIZE reads half the bytes copied, WRITE_SIZE
# all of them).  Valid only for the kernel source with this SHA-256 (of
# gx_gravity.hip followed by gx_internal.hpp) and the particle order named
# (the outputs are scattered to the caller's order); any change to either
# file, or the other order, makes the bench report null.
GRAV_TRAFFIC = {"source_sha256": "d5f58f57fffbbe3981b12cdf92d962fd7112c216f3bfad1aefda51e5565594fd",
                "particle_order": "morton",
                "fetch_kib": 6767743.375, "write_kib": 1407528.0625,
                "fetch_scale": 2.0, "write_scale": 1.0}


def grav_source_sha256():
    """SHA-256 over the gravity kernel's source followed by the shared header
    (record layouts, block-to-group mapping): the counters hold for exactly
    this pair."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gx_gravity.hip", "gx_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2510_23330_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def grav_traffic_bytes(order):
    if order != GRAV_TRAFFIC["particle_order"]:
        return None
    if GRAV_TRAFFIC["source_sha256"] is None:
        return None
    if grav_source_sha256() != GRAV_TRAFFIC["source_sha256"]:
        return None
    return 1024.0 * (GRAV_TRAFFIC["fetch_kib"] * GRAV_TRAFFIC["fetch_scale"] +
                     GRAV_TRAFFIC["write_kib"] * GRAV_TRAFFIC["write_scale"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16_000_000)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--cpu-groups", type=int, default=1024,
                    help="groups in the oracle's timed sample (0 skips the CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU-baseline leg (oracle timing and force errors)")
    ap.add_argument("--sn-sites", type=int, default=64,
                    help="SN regions handed to the surrogate per step (0: plain step only)")
    ap.add_argument("--sn-cubes", type=int, default=64,
                    help="SN cubes of the plain-SPH vs surrogate region comparison (0 skips)")
    ap.add_argument("--sn-infer-batch", type=int, default=256)
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2510_23330_amd", "weights",
                                                      "sn_unet_5ch.npz"),
                    help="trained surrogate weights (random initialisation when absent)")
    ap.add_argument("--no-force-error", action="store_true",
                    help="skip the force errors against the oracle's direct sum")
    ap.add_argument("--sph-stream", choices=("own", "shared"), default="own",
                    help="gas tree, density and hydro force on a second context and stream "
                         "beside the gravity kernel (default), or in series after it")
    ap.add_argument("--sn-mode", choices=("async", "sync"), default="async",
                    help="surrogate hand-over on its own stream in a worker thread (default), "
                         "or in series on the galaxy's stream")
    ap.add_argument("--sn-start", choices=("after_gravity", "now"), default="after_gravity",
                    help="asynchronous hand-over: start after the next gravity kernel (default) "
                         "or as soon as the snapshot is taken")
    ap.add_argument("--resampler", choices=("cdf", "gibbs"), default="cdf",
                    help="grid-to-particle mapping of the surrogate: inverse CDF or Gibbs chains")
    ap.add_argument("--sweeps", type=int, default=4, help="Gibbs sweeps per particle")
    ap.add_argument("--n-group", type=int, default=256, help="gravity group size n_g")
    ap.add_argument("--n-leaf", type=int, default=16, help="gravity tree leaf size")
    ap.add_argument("--sph-group", type=int, default=64, help="SPH group size")
    ap.add_argument("--sph-leaf", type=int, default=8, help="gas tree leaf size")
    ap.add_argument("--plain-steps", type=int, default=5,
                    help="steps without the surrogate after the timed ones (step cost without it)")
    ap.add_argument("--ic-order", choices=("morton", "generated"), default="morton",
                    help="particle array order: Morton order of a 1024^3 grid per block "
                         "(default) or the generator's order")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _err_stats(a, ref):
    """Relative force error |a - ref| / |ref| per receiver: n, median, p99, max,
    and the fraction of force nulls (|ref| below 1e-3 of the median |ref|)."""
    an = np.sqrt(ref[0] ** 2 + ref[1] ** 2 + ref[2] ** 2)
    e = np.sqrt((a[0] - ref[0]) ** 2 + (a[1] - ref[1]) ** 2 + (a[2] - ref[2]) ** 2) / an
    return {"n": int(e.size), "median": float(np.median(e)), "p99": float(np.percentile(e, 99)),
            "max": float(e.max()), "null_frac": float(np.mean(an < 1e-3 * np.median(an)))}


def force_errors(eng, sim, n_recv=256, seed=31):
    """Relative force error against the FP64 oracle's direct sum (Eq. 1 over
    every source): the benchmark's 16M particles in their state after the
    timed steps (tree gravity, the timed configuration), the 1M disk (tree),
    and the 8,192-particle Plummer sphere (direct sum in FP32)."""
    import torch
    import ics
    import oracle
    import paper_2510_23330_amd as gx
    G = ics.G_KPC
    out = {}
    p = sim.p
    n = p.n
    acc = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    eng.tree_build(p, gx.GX_TREE_ALL, 16, 256)
    eng.gravity_forces(p, G, 0.5, gx.GX_QUAD, *acc)
    host = {k: getattr(p, k).cpu().numpy() for k in ("x", "y", "z", "m")}
    host["eps2"] = p.eps2.cpu().numpy()
    idx = ics.sample_indices(n, n_recv, seed)
    ref = oracle.direct_gravity(host, G, idx)
    out["disk16M_tree_vs_fp64_direct"] = dict(
        _err_stats([a.cpu().numpy()[idx] for a in acc[:3]], ref[:3]),
        receivers=f"{len(idx)} seeded of {n}")
    del acc, host
    d1 = ics.disk_galaxy(1_000_000, 3)
    p1 = gx.ParticleSet.from_numpy(d1)
    acc = [torch.zeros(p1.n, dtype=torch.float64, device="cuda") for _ in range(4)]
    eng.tree_build(p1, gx.GX_TREE_ALL, 16, 256)
    eng.gravity_forces(p1, G, 0.5, gx.GX_QUAD, *acc)
    idx = ics.sample_indices(p1.n, 16384, 17)
    ref = oracle.direct_gravity(d1, G, idx)
    out["disk1M_tree_vs_fp64_direct"] = dict(
        _err_stats([a.cpu().numpy()[idx] for a in acc[:3]], ref[:3]),
        receivers=f"{len(idx)} seeded of {p1.n}")
    d0 = ics.plummer(8192, 1)
    p0 = gx.ParticleSet.from_numpy(d0)
    acc = [torch.zeros(p0.n, dtype=torch.float64, device="cuda") for _ in range(4)]
    eng.tree_build(p0, gx.GX_TREE_ALL, 16, 256)
    eng.gravity_forces(p0, 1.0, 0.5, gx.GX_DIRECT, *acc)
    ref = oracle.direct_gravity(d0, 1.0)
    out["plummer8k_direct_fp32_vs_fp64"] = dict(
        _err_stats([a.cpu().numpy() for a in acc[:3]], ref[:3]), receivers="all 8192")
    out["targets_p99"] = {"tree": 1e-3, "direct": 1e-5}
    return out


def hbm_phases(n_part, n_gas, tree_ms, kd_ms):
    """The HBM-bound phases against 8 TB/s with their algorithmic bytes: both
    tree builds at ~330 B per particle (keys, 8 sort passes, permute, cells,
    moments), and the four kick/drift calls of a step (stars 192 B, gas 272 B
    per particle: positions, velocities, accelerations, u, du/dt, the
    predictions)."""
    n_star = n_part - n_gas
    tree_b = TREE_BYTES_PER_PARTICLE * (n_part + n_gas)
    kd_b = 192 * n_star + 272 * n_gas
    return {
        "tree_builds": {"bytes": tree_b, "ms": tree_ms, "GB_s": tree_b / tree_ms / 1e6,
                        "frac": tree_b / (tree_ms / 1e3) / HBM_PEAK,
                        "note": "a chain of small dependent kernels (sort passes, cells, one "
                                "moment launch per level): launch- and latency-bound"},
        "kick_drift": {"bytes": kd_b, "ms": kd_ms, "GB_s": kd_b / kd_ms / 1e6,
                       "frac": kd_b / (kd_ms / 1e3) / HBM_PEAK},
        "peak_GB_s": HBM_PEAK / 1e9}


def cpu_baseline_leg(args, eng, sim, d):
    """The benchmark's CPU-baseline leg, the only part of it that runs the
    FP64 oracle: the oracle's tree gravity timed on the host cores
    (``cpu_baseline``) and, unless --no-force-error, the oracle's FP64 direct
    sum as the reference of the GPU forces (``force_error``).  --no-cpu skips
    the leg."""
    res = {"cpu_baseline": None}
    if args.no_cpu:
        return res
    if not args.no_force_error:
        t0 = time.perf_counter()
        res["force_error"] = force_errors(eng, sim)
        log(f"[bench] force errors {time.perf_counter() - t0:.1f} s")
    if args.cpu_groups > 0:
        t0 = time.perf_counter()
        res["cpu_baseline"] = cpu_baseline(d, args.cpu_groups, 99)
        res["cpu_baseline"]["one_thread_disk1M"] = oracle_one_thread_disk1M()
        log(f"[bench] cpu baseline {time.perf_counter() - t0:.1f} s")
    return res


def oracle_one_thread_disk1M(n_groups=256, seed=98):
    """The oracle's tree gravity on one host thread for a seeded sample of
    the 1M disk's groups, in a child process started with OMP_NUM_THREADS=1
    (it touches no GPU)."""
    import subprocess
    code = ("import time, ics, oracle\n"
            "d = ics.disk_galaxy(1_000_000, 3)\n"
            "T = oracle.Tree(d, 16, 256)\n"
            f"g = ics.sample_indices(T.n_groups, {n_groups}, {seed})\n"
            "t0 = time.perf_counter()\n"
            "r = T.gravity_groups(g, ics.G_KPC, 0.5, True)\n"
            "dt = time.perf_counter() - t0\n"
            "print(r[4] + r[5], dt, T.n_groups)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                             text=True, timeout=600, check=True).stdout.split()
    except (subprocess.SubprocessError, OSError) as e:
        return {"error": str(e)[:200]}
    inter, dt, ng = float(out[-3]), float(out[-2]), int(out[-1])
    return {"value": inter / dt, "unit": "interactions/s", "cores": 1,
            "sample": f"FP64 oracle tree gravity for {n_groups} of {ng} groups of the 1M disk "
                      f"({inter:.3e} interactions in {dt:.2f} s)"}


def cpu_baseline(d, n_groups_sample, seed):
    import oracle
    import ics
    t0 = time.perf_counter()
    T = oracle.Tree(d, 16, 256)
    build_s = time.perf_counter() - t0
    gsel = ics.sample_indices(T.n_groups, n_groups_sample, seed)
    t0 = time.perf_counter()
    r = T.gravity_groups(gsel, ics.G_KPC, 0.5, True)
    dt = time.perf_counter() - t0
    inter = r[4] + r[5]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": inter / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"FP64 oracle tree gravity (theta 0.5, quadrupole) for {len(gsel)} of "
                       f"{T.n_groups} groups of the 16M disk ({inter:.3e} interactions in "
                       f"{dt:.2f} s; oracle tree build {build_s:.1f} s not included)")}


def load_surrogate(eng, batch, weights, resampler="cdf", sweeps=4):
    """The network for inference: the trained weights when the file exists,
    else a random initialisation (then only its cost is meaningful)."""
    from paper_2510_23330_amd.sn import Surrogate
    have = bool(weights) and os.path.exists(weights)
    enc = Surrogate.file_encoding(weights) if have else "5ch"
    sur = Surrogate(eng, batch=batch, seed=0, train=False, encoding=enc,
                    resampler=resampler, sweeps=sweeps)
    if have:
        sur.load(weights)
        return sur, os.path.relpath(weights, ROOT)
    return sur, None


def _abs_err_stats(pred, ref):
    d = np.abs(pred - ref)
    return {"median": float(np.median(d)), "p90": float(np.percentile(d, 90))}


def sn_region_leg(eng, n_cubes, infer_batch, weights, resampler="cdf", sweeps=4, seed0=5000):
    """Per SN region: plain small-dt SPH to 0.1 Myr against the surrogate path
    (extract, ambient, gas tree, voxelize, infer, resample) on the same cubes.
    Plain SPH runs twice: with one shared Courant step for all cubes (what a
    galaxy with a shared global step must take) and with each cube on its own
    Courant step (the fair cost per region).  With trained weights the
    surrogate's per-voxel error against the per-cube plain SPH is reported,
    beside persistence (no change).  Plus inference throughput at the stated
    batch."""
    import torch
    import ics
    from paper_2510_23330_amd.sn import GRID, SNBatch, generate
    from paper_2510_23330_amd.unet import flops_forward
    seeds = list(range(seed0, seed0 + n_cubes))
    _, _, info_sh = generate(eng, seeds)
    x0, y, info = generate(eng, seeds, per_cube=True)
    cube_steps = np.asarray(info["cube_steps"])
    sur, wfile = load_surrogate(eng, 64, weights, resampler, sweeps)
    sb = SNBatch(eng, ics.sn_batch(seeds))
    sb.voxelize()
    sur.regions(sb.p, sb.g, sb.centers, cap=sb.n)         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, idx, new, pred = sur.regions(sb.p, sb.g, sb.centers, cap=sb.n)
    torch.cuda.synchronize()
    sur_s = time.perf_counter() - t0
    res = {"regions": n_cubes, "particles": info["n_particles"],
           "plain_sph_shared_step": {"steps": info_sh["steps"], "s": info_sh["seconds"],
                                     "ms_per_region": info_sh["seconds"] / n_cubes * 1e3},
           "plain_sph_per_cube_step": {"steps_min": int(cube_steps.min()),
                                       "steps_median": float(np.median(cube_steps)),
                                       "steps_max": int(cube_steps.max()),
                                       "s": info["seconds"],
                                       "ms_per_region": info["seconds"] / n_cubes * 1e3},
           "surrogate_s": sur_s, "surrogate_ms_per_region": sur_s / n_cubes * 1e3,
           "speedup_vs_per_cube": info["seconds"] / sur_s,
           "speedup_vs_shared_step": info_sh["seconds"] / sur_s,
           "weights": wfile or "random init (timing only)",
           "encoding": sur.encoding,
           "resampler": sur.resampler + (f" ({sur.sweeps} sweeps)" if sur.resampler == "gibbs" else "")}
    if wfile:
        V = GRID ** 3
        P = pred.view(n_cubes, V, 5).cpu().numpy().astype(np.float64)
        Y = y.view(n_cubes, V, 5).cpu().numpy().astype(np.float64)
        X = x0.view(n_cubes, V, 5).cpu().numpy().astype(np.float64)
        res["error_vs_plain_sph"] = {
            "surrogate": {"dlog_rho": _abs_err_stats(P[..., 0], Y[..., 0]),
                          "dlog_T": _abs_err_stats(P[..., 1], Y[..., 1])},
            "persistence": {"dlog_rho": _abs_err_stats(X[..., 0], Y[..., 0]),
                            "dlog_T": _abs_err_stats(X[..., 1], Y[..., 1])},
            "unit": "dex per voxel (64^3 voxels x regions)"}
    # inference throughput at infer_batch regions (chunks of the network's batch)
    V = GRID ** 3
    xin = torch.zeros(infer_batch * V * 8, dtype=torch.bfloat16, device="cuda")
    pr = torch.empty(infer_batch * V * 5, dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sur.infer(xin[:32 * V * 8], 32, pr)
    ev0.record()
    sur.infer(xin, infer_batch, pr)
    ev1.record()
    torch.cuda.synchronize()
    inf_s = ev0.elapsed_time(ev1) / 1e3
    fl = flops_forward(GRID) * infer_batch
    res.update({"infer_batch": infer_batch, "infer_s": inf_s, "infer_tflops": fl / inf_s / 1e12,
                "infer_frac_bf16_peak": fl / inf_s / 2.5e15})
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1 "
                          "(sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    import ics
    import paper_2510_23330_amd as gx
    from paper_2510_23330_amd.sim import GalaxyStep, StepConfig

    t0 = time.perf_counter()
    d = ics.disk_galaxy(args.n, args.seed)
    if args.ic_order == "morton":
        ics.spatial_order(d)
    log(f"[bench] generated {args.n} particles ({args.ic_order} order) in "
        f"{time.perf_counter() - t0:.1f} s")
    eng = gx.Engine(0)
    p = gx.ParticleSet.from_numpy(d)
    u = torch.as_tensor(d["u_gas"], device="cuda")
    cfg = StepConfig(G=ics.G_KPC, dt=2000.0 * YEAR_IN_KPC_TIME, theta=0.5, quad=True,
                     n_leaf=args.n_leaf, n_group=args.n_group, sph_leaf=args.sph_leaf,
                     sph_group=args.sph_group, n_ngb=64.0, u_floor=10.0 * ics.U_PER_K)
    hydro = gx.Engine(0, stream=torch.cuda.Stream()) if args.sph_stream == "own" else None
    sim = GalaxyStep(eng, p, int(d["gas_offset"]), u, cfg, timing=True, hydro=hydro)
    coupling = None
    if args.sn_sites > 0:
        from paper_2510_23330_amd.coupling import SNCoupling
        asyn = args.sn_mode == "async"
        sur_eng = gx.Engine(0, stream=torch.cuda.Stream() if asyn else None)
        sur, wfile = load_surrogate(sur_eng, 64, args.weights, args.resampler, args.sweeps)
        coupling = SNCoupling(sim, sur, n_sites=args.sn_sites, delay=50, asynchronous=asyn,
                              start=args.sn_start)
    torch.cuda.synchronize()
    log("[bench] set-up done; initial forces (cold kernel sizes) ...")
    t0 = time.perf_counter()
    sim.initial_forces()
    torch.cuda.synchronize()
    log(f"[bench] initial forces (cold kernel sizes) {time.perf_counter() - t0:.2f} s")
    sn_ms = []

    def sn_phase(i):
        if coupling is None:
            return
        if coupling.asynchronous:  # hand-over only; the work overlaps the next steps
            coupling.apply_due(i)
            coupling.launch(i)
            return
        torch.cuda.synchronize()
        t = time.perf_counter()
        coupling.apply_due(i)
        coupling.launch(i)
        torch.cuda.synchronize()
        sn_ms.append((time.perf_counter() - t) * 1e3)

    for w in range(args.warmup):
        sim.step()
        sn_phase(w)
        sim.energy()
        log(f"[bench] warmup step {w} done")
    sn_ms.clear()
    if coupling is not None:
        coupling.drain()
        coupling.sur_ms.clear()
    torch.cuda.synchronize()

    per = []
    grav_ms, grav_kernel_ms, dens_ms, hydro_ms, tree_ms = [], [], [], [], []
    n_pp = n_pc = n_sph = 0
    dens_k_ms, hydro_k_ms, dens_it = [], [], []
    n_dens_eval = n_dens_ngb = n_force_list = n_force_ngb = 0
    energies = []
    walk_diag = []
    kd_ev, list_sizes = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st = sim.step()
        sn_phase(args.warmup + k)
        energies.append(sim.energy())
        per.append(time.perf_counter() - ts)
        grav_ms.append(st["gravity"]["ms"])
        grav_kernel_ms.append(st["gravity"]["ms_kernel"])
        dens_ms.append(st["density"]["ms"])
        hydro_ms.append(st["hydro"]["ms"])
        tree_ms.append(st["tree_all"]["ms"] + st["tree_gas"]["ms"])
        walk_diag.append((st["gravity"]["n_rewalk"], st["gravity"]["n_iter_max"]))
        kd_ev.append(st["kd_events"])
        list_sizes.append(eng.gravity_list_sizes())
        n_pp += st["gravity"]["n_pp"]
        n_pc += st["gravity"]["n_pc"]
        n_sph += st["density"]["n_sph_list"] + st["hydro"]["n_sph_list"]
        dens_k_ms.append(st["density"]["ms_kernel"])
        hydro_k_ms.append(st["hydro"]["ms_kernel"])
        dens_it.append(st["density"]["n_iter_max"])
        n_dens_eval += st["density"]["n_sph_list"]
        n_dens_ngb += st["density"]["n_sph_ngb"]
        n_force_list += st["hydro"]["n_sph_list"]
        n_force_ngb += st["hydro"]["n_sph_ngb"]
        log(f"[bench] step {k}: {per[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = elapsed / args.steps * 1e3
    kd_ms = float(np.mean([e[0].elapsed_time(e[1]) + e[2].elapsed_time(e[3]) for e in kd_ev]))
    alone_ms = None
    if hydro is not None:
        # two untimed steps with the SPH after the gravity kernel instead of
        # beside it (and no hand-over in flight): the pairwise kernel with the
        # GPU to itself
        if coupling is not None:
            coupling.drain()
        sim.concurrent = False
        al = {"gk": [], "tree": [], "dk": [], "hk": [], "kd": []}
        for _ in range(2):
            st = sim.step()
            al["gk"].append(st["gravity"]["ms_kernel"])
            al["tree"].append(st["tree_all"]["ms"] + st["tree_gas"]["ms"])
            al["dk"].append(st["density"]["ms_kernel"])
            al["hk"].append(st["hydro"]["ms_kernel"])
            al["kd"].append(st["kd_events"])
        torch.cuda.synchronize()
        al["kd"] = [e[0].elapsed_time(e[1]) + e[2].elapsed_time(e[3]) for e in al["kd"]]
        sim.concurrent = True
        al = {k: float(np.mean(v)) for k, v in al.items()}
        alone_ms = al["gk"]
    # kernel rates and HBM phases from the steps where each phase ran alone
    dens_k = al["dk"] if alone_ms is not None else float(np.mean(dens_k_ms))
    hydro_k = al["hk"] if alone_ms is not None else float(np.mean(hydro_k_ms))
    tree_alone = al["tree"] if alone_ms is not None else float(np.mean(tree_ms))
    kd_alone = al["kd"] if alone_ms is not None else kd_ms
    walk_ms = float(np.mean(grav_ms) - np.mean(grav_kernel_ms))
    sn_async = None
    applied_at_end = 0
    if coupling is not None:
        coupling.drain()
        sur_ms = list(coupling.sur_ms)
        # a run shorter than the 50-step delay has no result falling due while
        # timed: apply the queued ones now, untimed, so that replacement by ID
        # runs on what the network predicted for these regions
        applied_at_end = len(coupling.queue)
        coupling.apply_due(10 ** 9)
        if coupling.asynchronous and args.plain_steps > 0:
            # the same steps without the hand-over: what the surrogate adds
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                sim.step()
                sim.energy()
            torch.cuda.synchronize()
            ms_plain = (time.perf_counter() - t0) / args.plain_steps * 1e3
            # and the hand-over alone, in series (nothing else on the GPU)
            serial = []
            for k in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                coupling.launch(10 ** 6 + k)
                coupling.drain()
                torch.cuda.synchronize()
                serial.append((time.perf_counter() - t0) * 1e3)
            added = ms_step - ms_plain
            sn_async = {"handover_serial_ms": float(np.median(serial)),
                        "step_ms_without_surrogate": ms_plain,
                        "step_ms_added": added,
                        "hidden_fraction": 1.0 - added / float(np.median(serial)),
                        "surrogate_stream_ms_per_handover": float(np.mean(sur_ms)),
                        "note": "surrogate on its own stream and host thread, started after the "
                                "next gravity kernel; hidden fraction = 1 - (step with - step "
                                "without) / the hand-over's cost in series"}
            sn_ms[:] = []
        coupling.close()
    inter_step = (n_pp + n_pc) / args.steps
    value = inter_step / (ms_step / 1e3)
    kernel_s = float(np.mean(grav_kernel_ms)) / 1e3
    flops = (FLOP_PP * n_pp + FLOP_PC * n_pc) / args.steps
    achieved = flops / kernel_s
    E0 = sum(energies[0])
    E1 = sum(energies[-1])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"disk galaxy {args.n / 1e6:g}M: 50 % disk stars, 40 % NFW halo, "
                               f"10 % gas disk; theta 0.5 + quadrupole, n_leaf {args.n_leaf}, "
                               f"groups <= {args.n_group}; SPH Wendland C4, 64 neighbours, gas "
                               f"leaves {args.sph_leaf}, groups <= {args.sph_group}; dt 2000 yr; "
                               f"{args.sn_sites} SN regions per step to the surrogate",
                   "n_particles": args.n, "seed": args.seed, "particle_order": args.ic_order,
                   "n_group": args.n_group, "n_leaf": args.n_leaf, "sph_group": args.sph_group,
                   "sph_leaf": args.sph_leaf, "sph_stream": args.sph_stream},
        "s_per_step": ms_step / 1e3,
        "grav_interactions_per_step": inter_step,
        "grav_pp_per_step": n_pp / args.steps,
        "grav_pc_per_step": n_pc / args.steps,
        "sph_pairs_per_step": n_sph / args.steps,
        "phase_ms": {"tree_builds": float(np.mean(tree_ms)), "gravity": float(np.mean(grav_ms)),
                     "gravity_kernel": float(np.mean(grav_kernel_ms)),
                     "sph_density": float(np.mean(dens_ms)), "sph_force": float(np.mean(hydro_ms)),
                     "kick_drift": kd_ms,
                     "sn_surrogate": float(np.mean(sn_ms)) if sn_ms else None},
        "ms_per_step_median": float(np.median(per)) * 1e3,
        "phase_ms_alone": None if alone_ms is None else {
            "tree_builds": al["tree"], "gravity_kernel": al["gk"], "sph_density_kernel": al["dk"],
            "sph_force_kernel": al["hk"], "kick_drift": al["kd"],
            "note": "two untimed steps with the SPH after the gravity kernel, no hand-over in "
                    "flight; in the timed steps the gas tree and SPH run beside the tree, walk "
                    "and gravity of all particles, so phase_ms overlap"},
        "sn_coupling": None if coupling is None else dict(
            coupling.stats, sites_per_step=args.sn_sites, delay_steps=50, mode=args.sn_mode, start=args.sn_start,
            handovers_applied_after_timing=applied_at_end,
            weights=wfile or "random init (timing only; every region falls back)",
            encoding=coupling.sur.encoding, resampler=coupling.sur.resampler),
        "sn_async": sn_async,
        "gravity_kernel_interactions_per_s": inter_step / kernel_s,
        "sph": {"density_pair_evals_per_step": n_dens_eval / args.steps,
                "density_ngb_evals_per_step": n_dens_ngb / args.steps,
                "density_kernel_ms": dens_k,
                "density_tflops_73": FLOP_DENS * n_dens_eval / args.steps / (dens_k / 1e3) / 1e12,
                "density_tflops_73_ngb": FLOP_DENS * n_dens_ngb / args.steps / (dens_k / 1e3)
                / 1e12,
                "density_max_iterations": int(max(dens_it)),
                "force_list_pairs_per_step": n_force_list / args.steps,
                "force_ngb_pairs_per_step": n_force_ngb / args.steps,
                "force_kernel_ms": hydro_k,
                "force_tflops_101": FLOP_FORCE * n_force_list / args.steps / (hydro_k / 1e3)
                / 1e12,
                "force_tflops_101_ngb": FLOP_FORCE * n_force_ngb / args.steps / (hydro_k / 1e3)
                / 1e12,
                "convention": "list: every candidate pair evaluated (Table 4 convention); ngb: "
                              "only pairs inside the kernel supports (density: summed over the "
                              "kernel-size passes); kernel times from steps with the SPH alone "
                              "on the GPU when it otherwise runs beside the gravity kernel"},
        "gravity_lists": {"two_pass_steps": int(sum(w[0] for w in walk_diag)),
                          "max_walk_stack": int(max(w[1] for w in walk_diag)),
                          "pc_entries_per_step": float(np.mean([l[1] for l in list_sizes])),
                          "pp_ranges_per_step": float(np.mean([l[2] for l in list_sizes])),
                          "walk_ms": walk_ms,
                          "list_entries_per_s": float(np.mean([l[1] + l[2] for l in list_sizes]))
                          / (walk_ms / 1e3),
                          "note": "walk_ms = gravity call minus its pairwise kernel (the list "
                                  "walk, the list totals and one host round trip); the walk is "
                                  "latency-bound"},
        "hbm_phases": hbm_phases(n_part=args.n, n_gas=sim.ng, tree_ms=tree_alone,
                                 kd_ms=kd_alone),
        "energy_drift_rel": abs(E1 - E0) / abs(E0),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": grav_traffic_bytes(args.ic_order),
                     "kernel": "k_grav_force<float,true>",
                     "flop_convention": f"{FLOP_PP}/pp + {FLOP_PC}/pc"},
    }
    if alone_ms is not None:
        # the timed launches share the GPU with the SPH kernels of the hydro
        # stream; the same FLOP over the kernel's time with the GPU to itself
        out["roofline"]["concurrent_with"] = "gas tree, density and hydro force on a second stream"
        out["roofline"]["alone"] = {"ms": alone_ms, "achieved": flops / (alone_ms / 1e3) / 1e12,
                                    "frac": flops / (alone_ms / 1e3) / PEAK_FP32,
                                    "steps": 2, "note": "untimed steps with the SPH after the "
                                    "gravity kernel"}
    if args.sn_cubes > 0:
        t0 = time.perf_counter()
        out["sn_region"] = sn_region_leg(eng, args.sn_cubes, args.sn_infer_batch, args.weights,
                                         args.resampler, args.sweeps)
        log(f"[bench] SN region leg {time.perf_counter() - t0:.1f} s")
        if sn_ms or sn_async:
            # 0.1 Myr of the disk with 64 SNe per step: 50 global steps of
            # 2,000 yr with the surrogate hand-over in each, against a shared
            # step that the SN regions hold to their Courant step (the shared-
            # step SPH of the 1 Msun cubes gives it) at the step cost without
            # the surrogate
            n_sh = out["sn_region"]["plain_sph_shared_step"]["steps"]
            plain_step_s = (sn_async["step_ms_without_surrogate"] if sn_async
                            else ms_step - float(np.mean(sn_ms))) / 1e3
            out["galaxy_0p1Myr"] = {
                "surrogate_s": 50 * ms_step / 1e3,
                "plain_shared_step_s": n_sh * plain_step_s,
                "speedup": n_sh * plain_step_s / (50 * ms_step / 1e3),
                "global_steps": {"surrogate": 50, "plain": n_sh},
                "dt_cfl_sn_yr": 0.1e6 / n_sh, "dt_global_yr": 2000.0}
    out.update(cpu_baseline_leg(args, eng, sim, d))
    sim.close()
    if hydro is not None:
        hydro.close()
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
