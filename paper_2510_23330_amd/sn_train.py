"""Supernova surrogate: data generation, training and held-out evaluation
(Sec. 3.3) on one GPU, every arithmetic step in libgx.

    python -m paper_2510_23330_amd.sn_train --n-train 256 --n-test 64 \
        --train-seconds 600 --out <dir>

1. Training pairs: K cubes per batch of plain small-timestep SPH (cube seeds
   sorted by particle count so one shared Courant step suits a batch), each
   voxelized to 64^3 x 5 channels before the explosion and 0.1 Myr after it.
2. Channel statistics of the training inputs and targets (standardisation)
   in the network's encoding (--encoding: the five physical channels, or the
   paper's eight cubes with the velocity components split by sign).
3. Adam on the MSE of the standardized target channels, shuffled mini-batches,
   until the epoch count or the time budget is reached.
4. Held-out cubes: the surrogate's prediction against plain SPH, against the
   pre-explosion state (persistence) and against plain SPH forced to the
   galaxy's 2,000 yr step; the resample -> density -> voxelize round trip of
   the replacement particles for each resampler (inverse CDF, Gibbs); wall
   time of plain SPH vs the surrogate path for the same regions.

Writes metrics.json, the weights (surrogate.npz) and a log to --out.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import GX_TREE_GAS, Engine, GasState, GxError, ParticleSet
from .sn import GRID, MYR, SIDE, U_PER_K, SNBatch, SPHConfig, Surrogate, generate

DT_GLOBAL_MYR = 2.0e-3


def _log_fn(path):
    f = open(path, "a") if path else None

    def log(msg):
        line = f"[{time.strftime('%H:%M:%S')}] {msg}"
        print(line, flush=True)
        if f:
            f.write(line + "\n")
            f.flush()
    return log


def batches_by_size(seeds, per_batch):
    import ics
    seeds = sorted(seeds, key=lambda s: (ics.sn_cube_n(s), s))
    return [seeds[i:i + per_batch] for i in range(0, len(seeds), per_batch)]


def generate_set(eng, seeds, per_batch, log, dt_fixed_myr=None, grid=GRID):
    """Plain-SPH pairs for `seeds`; returns (X, Y, order, infos) with X, Y
    device float [n, V * 5] in the order `order` (a permutation of seeds)."""
    import torch
    V5 = grid ** 3 * 5
    n = len(seeds)
    X = torch.empty((n, V5), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, V5), dtype=torch.float32, device="cuda")
    order, infos = [], []
    k = 0
    for bs in batches_by_size(seeds, per_batch):
        try:
            x, y, info = generate(eng, bs, dt_fixed_myr=dt_fixed_myr, log=log, grid=grid)
        except (FloatingPointError, GxError) as e:
            if dt_fixed_myr is None:
                raise
            log(f"fixed-step SPH of cubes {bs[0]}..: {e}")
            x = y = None
            info = {"steps": -1, "seconds": float("nan"), "n_particles": 0, "diverged": str(e)}
        if y is None:
            # a diverged run predicts nothing: count it as the pre-explosion state
            import ics
            sb = SNBatch(eng, ics.sn_batch(bs))
            x = sb.voxelize(grid=grid)
            y = torch.full_like(x, float("nan"))
            info["n_particles"] = sb.n
        X[k:k + len(bs)] = x.view(len(bs), V5)
        Y[k:k + len(bs)] = y.view(len(bs), V5)
        k += len(bs)
        order += bs
        infos.append({kk: v for kk, v in info.items() if kk != "batch"})
        log(f"generated {k}/{n} cubes: batch of {len(bs)} ({info['n_particles']} particles) "
            f"{info['steps']} steps in {info['seconds']:.1f} s")
    return X, Y, order, infos


def abs_log_err(pred, ref):
    """Per-voxel |d log10 rho|, |d log10 T| and |d v| (km/s) as numpy arrays."""
    import torch
    p = pred.view(-1, 5)
    r = ref.view(-1, 5)
    d = torch.nan_to_num((p - r).abs(), nan=1e3, posinf=1e3, neginf=1e3)
    dv = torch.sqrt((d[:, 2:] ** 2).sum(dim=1))
    return d[:, 0].cpu().numpy(), d[:, 1].cpu().numpy(), dv.cpu().numpy()


def summarize(pred, ref):
    out = {}
    for name, a in zip(("log_rho", "log_T", "v"), abs_log_err(pred, ref)):
        out[name] = {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
                     "mean": float(np.mean(a))}
    return out


def train(sur: Surrogate, Xp, Yp, Xt, Yt, epochs, seconds, lr, log, seed=0, augment=True):
    """Xp, Yp: physical training pairs, device float [n, V*5]; Xt, Yt: the
    held-out pairs standardized (bf16 [m, V*8], f32 [m, V*nc]).  The cube
    symmetries act on the physical channels, before the encoding.  Each
    mini-batch is drawn at random, mapped by a random symmetry of the cube
    (augment) and standardized on the device.  The weights with the lowest
    held-out MSE seen at an epoch end are kept."""
    import torch
    eng, net = sur.eng, sur.net
    B = net.B
    n = Xp.shape[0]
    V, S = sur.V, sur.grid
    rng = np.random.default_rng(seed)
    f32 = dict(dtype=torch.float32, device="cuda")
    xg = torch.empty(B * V * 5, **f32)
    yg = torch.empty(B * V * 5, **f32)
    xa = torch.empty(B * V * 5, **f32)
    ya = torch.empty(B * V * 5, **f32)
    xb = torch.empty(B * V * 8, dtype=torch.bfloat16, device="cuda")
    yb = torch.empty(B * V * sur.nc, **f32)
    best = (float("inf"), None, -1)
    t0 = time.perf_counter()
    hist = []
    step = 0
    last = t0
    stop = False
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot, cnt = 0.0, 0
        for a in range(0, n - B + 1, B):
            sel = torch.as_tensor(perm[a:a + B], device="cuda")
            xg.view(B, V * 5).copy_(Xp.index_select(0, sel))
            yg.view(B, V * 5).copy_(Yp.index_select(0, sel))
            if augment:
                sym = torch.as_tensor(rng.integers(0, 48, B).astype(np.int32), device="cuda")
                eng.cube_sym(xg, B, S, 5, 2, sym, xa)
                eng.cube_sym(yg, B, S, 5, 2, sym, ya)
                src_x, src_y = xa, ya
            else:
                src_x, src_y = xg, yg
            sur.standardize(src_x, "in", out_bf16=xb)
            sur.standardize(src_y, "out", out_f32=yb)
            loss = net.train_step(xb, yb, lr=lr)
            tot += loss
            cnt += 1
            step += 1
            now = time.perf_counter()
            if now - last > 30:
                log(f"epoch {ep} step {step} train mse {tot / cnt:.4f} ({now - t0:.0f} s)")
                last = now
            if now - t0 > seconds:
                stop = True
                break
        val = evaluate_mse(sur, Xt, Yt)
        if val < best[0]:
            best = (val, net.w32.clone(), ep)
        hist.append({"epoch": ep, "steps": step, "train_mse": tot / max(cnt, 1), "val_mse": val,
                     "seconds": time.perf_counter() - t0})
        log(f"epoch {ep}: train mse {tot / max(cnt, 1):.4f} val mse {val:.4f}")
        if stop:
            break
    if best[1] is not None:
        net.w32.copy_(best[1])
        eng.f32_to_bf16(net.w32, net.wbf)
        log(f"kept the weights of epoch {best[2]} (val mse {best[0]:.4f})")
    return hist


def evaluate_mse(sur: Surrogate, Xt, Yt):
    """Mean standardized-channel MSE over held-out pairs."""
    net = sur.net
    B, V = net.B, sur.V
    n = Xt.shape[0]
    tot = 0.0
    for a in range(0, n, B):
        b = min(B, n - a)
        net.Bcur = b
        pred = net.forward(Xt[a:a + b].reshape(-1))
        tot += b * sur.eng.mse(pred, 16, Yt[a:a + b].reshape(-1), sur.nc, b * V)
    net.Bcur = B
    return tot / n


def bench_training(a):
    """Training throughput of the network alone (random standardized inputs
    and targets; forward, MSE, backward, Adam per step)."""
    import torch
    from .unet import flops_forward
    eng = Engine(0)
    sur = Surrogate(eng, batch=a.batch, base=a.base, levels=a.levels, grid=a.grid, seed=1,
                    encoding=a.encoding)
    V, nc = a.grid ** 3, sur.nc
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    xb = torch.zeros(a.batch * V * 8, dtype=torch.float32, device="cuda")
    xb.view(-1, 8)[:, :nc] = torch.randn(a.batch * V, nc, device="cuda", generator=g)
    xb = xb.to(torch.bfloat16)
    yb = torch.randn(a.batch * V * nc, device="cuda", generator=g)
    for _ in range(3):
        sur.net.train_step(xb, yb, lr=a.lr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.bench_steps):
        sur.net.train_step(xb, yb, lr=a.lr)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.bench_steps
    fl = 3 * flops_forward(a.grid, a.base, a.levels) * a.batch
    out = {"batch": a.batch, "grid": a.grid, "encoding": a.encoding, "ms_per_step": dt * 1e3,
           "samples_per_s": a.batch / dt, "tflops_3x_forward": fl / dt / 1e12,
           "frac_bf16_peak": fl / dt / 2.5e15}
    print(json.dumps(out), flush=True)
    eng.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=256)
    ap.add_argument("--n-test", type=int, default=64)
    ap.add_argument("--per-batch", type=int, default=64)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--grid", type=int, default=GRID)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--train-seconds", type=float, default=600)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--init", default=None, help="surrogate.npz to continue from")
    ap.add_argument("--no-augment", action="store_true",
                    help="train without the random cube symmetries")
    ap.add_argument("--out", default="sn_out")
    ap.add_argument("--export", default=None,
                    help="also write the inference weights (BF16) to this file")
    ap.add_argument("--encoding", choices=("5ch", "8cube"), default="5ch",
                    help="network channels: five physical ones or the paper's eight cubes")
    ap.add_argument("--resampler", choices=("cdf", "gibbs"), default="cdf")
    ap.add_argument("--sweeps", type=int, default=4, help="Gibbs sweeps per particle")
    ap.add_argument("--eval-resamplers", default="cdf,gibbs",
                    help="resamplers compared in the held-out replacement check")
    ap.add_argument("--bench-steps", type=int, default=0,
                    help="only time this many training steps on random data and exit")
    a = ap.parse_args(argv)
    import torch
    if a.bench_steps > 0:
        return bench_training(a)
    os.makedirs(a.out, exist_ok=True)
    log = _log_fn(os.path.join(a.out, "log.txt"))
    eng = Engine(0)
    V = a.grid ** 3
    metrics = {"config": vars(a)}
    train_seeds = list(range(a.seed0, a.seed0 + a.n_train))
    test_seeds = list(range(a.seed0 + a.n_train, a.seed0 + a.n_train + a.n_test))

    # 1. data
    t0 = time.perf_counter()
    Xp, Yp, order, infos = generate_set(eng, train_seeds, a.per_batch, log, grid=a.grid)
    metrics["train_generation_s"] = time.perf_counter() - t0
    Xtp, Ytp, torder, tinfos = generate_set(eng, test_seeds, a.per_batch, log, grid=a.grid)
    metrics["test_plain_sph"] = tinfos

    # 2. statistics and standardized copies
    sur = Surrogate(eng, batch=a.batch, base=a.base, levels=a.levels, grid=a.grid, seed=1,
                    encoding=a.encoding, resampler=a.resampler, sweeps=a.sweeps)
    nc = sur.nc
    if a.init:
        sur.load(a.init)
    else:
        si = torch.zeros(2 * nc, dtype=torch.float64, device="cuda")
        so = torch.zeros(2 * nc, dtype=torch.float64, device="cuda")
        sur.channel_sums(Xp, si)
        sur.channel_sums(Yp, so)
        sp = None
        if nc != 5:
            sp = torch.zeros(10, dtype=torch.float64, device="cuda")
            eng.chan_stats(Yp.view(-1), 5, 5, sp)
        sur.set_stats(si, so, Xp.shape[0] * V, sums_phys=sp)
    metrics["stats"] = {k: getattr(sur, k).cpu().tolist()
                        for k in ("mean_in", "std_in", "mean_out", "std_out", "mean_phys",
                                  "std_phys")}

    def std_pair(X, Y):
        Xs = torch.empty((X.shape[0], V * 8), dtype=torch.bfloat16, device="cuda")
        Ys = torch.empty((Y.shape[0], V * nc), dtype=torch.float32, device="cuda")
        sur.standardize(X.view(-1), "in", out_bf16=Xs.view(-1))
        sur.standardize(Y.view(-1), "out", out_f32=Ys.view(-1))
        return Xs, Ys

    Xts, Yts = std_pair(Xtp, Ytp)
    log(f"dataset: {Xp.shape[0]} train / {Xts.shape[0]} test cubes")

    # 3. training
    from .unet import flops_forward
    t0 = time.perf_counter()
    hist = []
    if Xp.shape[0] >= a.batch and a.epochs > 0:
        hist = train(sur, Xp, Yp, Xts, Yts, a.epochs, a.train_seconds, a.lr, log,
                     augment=not a.no_augment)
    del Xp, Yp
    ttrain = time.perf_counter() - t0
    steps = hist[-1]["steps"] if hist else 0
    metrics["training"] = {"history": hist, "seconds": ttrain, "steps": steps,
                           "samples_per_s": steps * a.batch / max(ttrain, 1e-9),
                           "tflops_est": 3 * flops_forward(a.grid, a.base, a.levels) * steps * a.batch
                           / max(ttrain, 1e-9) / 1e12}
    sur.save(os.path.join(a.out, "surrogate.npz"))
    if a.export:
        sur.export(a.export)

    # 4. held-out evaluation (physical channels)
    n_t = Xtp.shape[0]
    pred = torch.empty(n_t * V * 5, dtype=torch.float32, device="cuda")
    sur.infer(Xts.view(-1), n_t, pred)
    metrics["surrogate_vs_sph"] = summarize(pred, Ytp)
    metrics["persistence_vs_sph"] = summarize(Xtp, Ytp)
    # the same comparison in the standardized target channels the loss uses
    pers = torch.empty(n_t * V * nc, dtype=torch.float32, device="cuda")
    sur.standardize(Xtp.view(-1), "out", out_f32=pers)
    metrics["mse_standardized"] = {
        "surrogate": evaluate_mse(sur, Xts, Yts),
        "persistence": sur.eng.mse(pers, nc, Yts.reshape(-1), nc, n_t * V)}
    del pers
    _, Yc, _, cinfos = generate_set(eng, test_seeds, a.per_batch, log, dt_fixed_myr=DT_GLOBAL_MYR,
                                    grid=a.grid)
    metrics["coarse_dt_sph_vs_sph"] = summarize(Yc, Ytp)
    metrics["coarse_dt_sph"] = cinfos
    del Yc

    # replacement particles: resample, density, voxelize again; and timings,
    # for each resampler compared
    import ics
    cfg = SPHConfig()
    metrics["replaced_particles_vs_sph"] = {}
    metrics["timing_by_resampler"] = {}
    plain_s = sum(i["seconds"] for i in tinfos)
    for rs in [r for r in a.eval_resamplers.split(",") if r]:
        sur.resampler = rs
        rt, sur_s, nreg = [], 0.0, 0
        k = 0
        for bs in batches_by_size(test_seeds, a.per_batch):
            sb = SNBatch(eng, ics.sn_batch(bs), cfg)
            sb.voxelize(grid=a.grid)            # kernel sizes of the pre-explosion state
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            off, idx, new, _ = sur.regions(sb.p, sb.g, sb.centers, cap=sb.n)
            torch.cuda.synchronize()
            sur_s += time.perf_counter() - t1
            nreg += len(bs)
            m = sb.p.m.index_select(0, idx.long())
            q = ParticleSet(x=new["x"], y=new["y"], z=new["z"], vx=new["vx"], vy=new["vy"],
                            vz=new["vz"], m=m, eps2=sb.p.eps2[:m.shape[0]])
            g = GasState.zeros(q.n, u=new["u"])
            eng.tree_build(q, GX_TREE_GAS, cfg.n_leaf, cfg.n_group)
            eng.sph_density(q, g, cfg.n_ngb, cfg.gamma, cfg.h_tol, cfg.max_iter, allow_noconv=True)
            vox = torch.zeros(len(bs) * V * 5, dtype=torch.float32, device="cuda")
            eng.sn_voxelize(q, g.u, g.H, sb.centers, SIDE, a.grid, 1.0 / U_PER_K, sb.ambient(),
                            out_f32=vox)
            rt.append((vox, k, len(bs)))
            k += len(bs)
        # truth rows follow the same size-sorted order as generate_set produced
        ref = torch.cat([Ytp[kk:kk + nb].reshape(-1) for _, kk, nb in rt])
        metrics["replaced_particles_vs_sph"][rs] = summarize(torch.cat([v for v, _, _ in rt]), ref)
        metrics["timing_by_resampler"][rs] = {
            "regions": nreg, "plain_sph_s": plain_s, "surrogate_s": sur_s,
            "speedup": plain_s / max(sur_s, 1e-12), "plain_sph_s_per_64": plain_s / nreg * 64,
            "surrogate_s_per_64": sur_s / nreg * 64}
        del rt, ref
    sur.resampler = a.resampler
    metrics["timing"] = metrics["timing_by_resampler"].get(
        a.resampler, next(iter(metrics["timing_by_resampler"].values()), {}))
    log(json.dumps({k: metrics[k] for k in ("mse_standardized", "surrogate_vs_sph", "persistence_vs_sph",
                                             "coarse_dt_sph_vs_sph", "replaced_particles_vs_sph",
                                             "timing")}))
    with open(os.path.join(a.out, "metrics.json"), "w") as f:
        json.dump(metrics, f, indent=1)
    eng.close()
    return metrics


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
