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
and replaces returned regions by particle ID 50 steps later (the network is
randomly initialised here: only its cost is measured).

Prints ONE JSON line.  ``value`` = gravity interactions (particle-particle +
particle-cell) per second of whole-step wall time.  ``roofline`` reports the
dominant kernel (pairwise gravity) against the FP32 vector peak, timed live
with HIP events on the library's stream.  ``sn_region`` compares, for 64 SN
cubes of 1 Msun particles, the plain small-timestep SPH to 0.1 Myr with the
surrogate path on the same cubes, and the network's inference throughput at
batch 256.  ``cpu_baseline`` times the FP64 oracle's tree gravity on a
seeded sample of the same workload's groups.
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
FLOP_PP = 27                         # per particle-particle interaction (Table 4 convention)
FLOP_PC = 63                         # per particle-cell interaction, monopole + quadrupole
FLOP_DENS = 73                       # per SPH density candidate pair evaluation (Table 4)
FLOP_FORCE = 101                     # per SPH force candidate pair (Table 4)

# HBM traffic of one k_grav_force<float,true> launch on this workload, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, WRITE_SIZE in KiB per
# dispatch) scaled by what the same counters read for a reference copy of
# known size (hbm_calib.py: FETCH_SIZE reads half the bytes copied, WRITE_SIZE
# all of them).  Valid only for the kernel source with this SHA-256 and the
# particle order named (the outputs are scattered to the caller's order); any
# change to gx_gravity.hip, or the other order, makes the bench report null.
GRAV_TRAFFIC = {"source_sha256": "a3d3eb3e96b0f3b25b0277057df50d3442b69ec67b795f182ff062edd99fd8f4",
                "particle_order": "morton",
                "fetch_kib": 3676699.3125, "write_kib": 2289833.4375,
                "fetch_scale": 2.0, "write_scale": 1.0}


def grav_traffic_bytes(order):
    import hashlib
    if order != GRAV_TRAFFIC["particle_order"]:
        return None
    src = os.path.join(ROOT, "paper_2510_23330_amd", "csrc", "gx_gravity.hip")
    if GRAV_TRAFFIC["source_sha256"] is None:
        return None
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != GRAV_TRAFFIC["source_sha256"]:
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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sn-sites", type=int, default=64,
                    help="SN regions handed to the surrogate per step (0: plain step only)")
    ap.add_argument("--sn-cubes", type=int, default=64,
                    help="SN cubes of the plain-SPH vs surrogate region comparison (0 skips)")
    ap.add_argument("--sn-infer-batch", type=int, default=256)
    ap.add_argument("--ic-order", choices=("morton", "generated"), default="morton",
                    help="particle array order: Morton order of a 1024^3 grid per block "
                         "(default) or the generator's order")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
            "sample": (f"FP64 oracle tree gravity (theta 0.5, quadrupole) for {len(gsel)} of "
                       f"{T.n_groups} groups of the 16M disk ({inter:.3e} interactions in "
                       f"{dt:.2f} s; oracle tree build {build_s:.1f} s not included)")}


def sn_region_leg(eng, n_cubes, infer_batch, seed0=5000):
    """Per SN region: plain small-dt SPH to 0.1 Myr vs the surrogate path
    (extract, ambient, gas tree, voxelize, infer, resample) on the same cubes,
    plus network inference throughput at the stated batch."""
    import torch
    import ics
    from paper_2510_23330_amd.sn import GRID, SNBatch, Surrogate, generate
    from paper_2510_23330_amd.unet import flops_forward
    seeds = list(range(seed0, seed0 + n_cubes))
    x, y, info = generate(eng, seeds)
    plain_s = info["seconds"]
    sur = Surrogate(eng, batch=64, seed=0, train=False)
    sb = SNBatch(eng, ics.sn_batch(seeds))
    sb.voxelize()
    sur.regions(sb.p, sb.g, sb.centers, cap=sb.n)         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.regions(sb.p, sb.g, sb.centers, cap=sb.n)
    torch.cuda.synchronize()
    sur_s = time.perf_counter() - t0
    # inference throughput at infer_batch regions (chunks of the network's batch)
    V = GRID ** 3
    xin = torch.zeros(infer_batch * V * 8, dtype=torch.bfloat16, device="cuda")
    pred = torch.empty(infer_batch * V * 5, dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sur.infer(xin[:32 * V * 8], 32, pred)
    ev0.record()
    sur.infer(xin, infer_batch, pred)
    ev1.record()
    torch.cuda.synchronize()
    inf_s = ev0.elapsed_time(ev1) / 1e3
    fl = flops_forward(GRID) * infer_batch
    return {"regions": n_cubes, "particles": info["n_particles"], "plain_sph_steps": info["steps"],
            "plain_sph_s": plain_s, "surrogate_s": sur_s, "speedup": plain_s / sur_s,
            "plain_sph_ms_per_region": plain_s / n_cubes * 1e3,
            "surrogate_ms_per_region": sur_s / n_cubes * 1e3,
            "infer_batch": infer_batch, "infer_s": inf_s,
            "infer_tflops": fl / inf_s / 1e12, "infer_frac_bf16_peak": fl / inf_s / 2.5e15,
            "weights": "random init (timing only; accuracy comes from the trained network)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(sharding across GPUs is not built)"}))
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
                     n_leaf=16, n_group=256, sph_leaf=8, sph_group=64, n_ngb=64.0,
                     u_floor=10.0 * ics.U_PER_K)
    sim = GalaxyStep(eng, p, int(d["gas_offset"]), u, cfg)
    coupling = None
    if args.sn_sites > 0:
        from paper_2510_23330_amd.coupling import SNCoupling
        from paper_2510_23330_amd.sn import Surrogate
        sur_eng = gx.Engine(0)
        coupling = SNCoupling(sim, Surrogate(sur_eng, batch=64, seed=0, train=False),
                              n_sites=args.sn_sites, delay=50)
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
    torch.cuda.synchronize()

    per = []
    grav_ms, grav_kernel_ms, dens_ms, hydro_ms, tree_ms = [], [], [], [], []
    n_pp = n_pc = n_sph = 0
    dens_k_ms, hydro_k_ms, dens_it = [], [], []
    n_dens_eval = n_force_list = n_force_ngb = 0
    energies = []
    walk_diag = []
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
        n_pp += st["gravity"]["n_pp"]
        n_pc += st["gravity"]["n_pc"]
        n_sph += st["density"]["n_sph_list"] + st["hydro"]["n_sph_list"]
        dens_k_ms.append(st["density"]["ms_kernel"])
        hydro_k_ms.append(st["hydro"]["ms_kernel"])
        dens_it.append(st["density"]["n_iter_max"])
        n_dens_eval += st["density"]["n_sph_list"]
        n_force_list += st["hydro"]["n_sph_list"]
        n_force_ngb += st["hydro"]["n_sph_ngb"]
        log(f"[bench] step {k}: {per[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = elapsed / args.steps * 1e3
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
        "config": {"workload": "disk galaxy 16M: 8e6 disk stars, 6.4e6 NFW halo, 1.6e6 gas disk; "
                               "theta 0.5 + quadrupole, n_leaf 16, groups <= 256; SPH Wendland C4, "
                               "64 neighbours, groups <= 64; dt 2000 yr; 64 SN regions per step "
                               "to the surrogate",
                   "n_particles": args.n, "seed": args.seed, "particle_order": args.ic_order},
        "s_per_step": ms_step / 1e3,
        "grav_interactions_per_step": inter_step,
        "grav_pp_per_step": n_pp / args.steps,
        "grav_pc_per_step": n_pc / args.steps,
        "sph_pairs_per_step": n_sph / args.steps,
        "phase_ms": {"tree_builds": float(np.mean(tree_ms)), "gravity": float(np.mean(grav_ms)),
                     "gravity_kernel": float(np.mean(grav_kernel_ms)),
                     "sph_density": float(np.mean(dens_ms)), "sph_force": float(np.mean(hydro_ms)),
                     "sn_surrogate": float(np.mean(sn_ms)) if sn_ms else None},
        "sn_coupling": None if coupling is None else dict(coupling.stats, sites_per_step=args.sn_sites,
                                                          delay_steps=50),
        "gravity_kernel_interactions_per_s": inter_step / kernel_s,
        "sph": {"density_pair_evals_per_step": n_dens_eval / args.steps,
                "density_kernel_ms": float(np.mean(dens_k_ms)),
                "density_tflops_73": FLOP_DENS * n_dens_eval / args.steps
                / (float(np.mean(dens_k_ms)) / 1e3) / 1e12,
                "density_max_iterations": int(max(dens_it)),
                "force_list_pairs_per_step": n_force_list / args.steps,
                "force_ngb_pairs_per_step": n_force_ngb / args.steps,
                "force_kernel_ms": float(np.mean(hydro_k_ms)),
                "force_tflops_101": FLOP_FORCE * n_force_list / args.steps
                / (float(np.mean(hydro_k_ms)) / 1e3) / 1e12},
        "gravity_lists": {"two_pass_steps": int(sum(w[0] for w in walk_diag)),
                          "max_walk_stack": int(max(w[1] for w in walk_diag))},
        "energy_drift_rel": abs(E1 - E0) / abs(E0),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": grav_traffic_bytes(args.ic_order),
                     "kernel": "k_grav_force<float,true>",
                     "flop_convention": f"{FLOP_PP}/pp + {FLOP_PC}/pc"},
    }
    if args.sn_cubes > 0:
        t0 = time.perf_counter()
        out["sn_region"] = sn_region_leg(eng, args.sn_cubes, args.sn_infer_batch)
        log(f"[bench] SN region leg {time.perf_counter() - t0:.1f} s")
    if not args.no_cpu and args.cpu_groups > 0:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(d, args.cpu_groups, 99)
        log(f"[bench] cpu baseline {time.perf_counter() - t0:.1f} s")
    else:
        out["cpu_baseline"] = None
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
