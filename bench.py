#!/usr/bin/env python3
"""Benchmark of the GN-Krylov registration hot path on one MI355X.

Workload (the paper's method on a 256^3 FP32 problem): a periodic Voronoi
phantom (120 seeds, Gaussian-smoothed with sigma = 2 cells, rescaled to
[0, 1]) as template, transported by a smooth random velocity (Gaussian-
filtered white noise, Leray-projected, max |v| = 0.15 * 2 pi) to make the
reference; H1-div regularisation with beta_v = 5e-3, beta_w = 1; nt = 4,
tricubic interpolation, spectral preconditioner, GN-Krylov to relative
gradient 5e-2.  Inputs are synthetic and seeded; they are generated and
uploaded before any timed region.

One step = one full GN-Krylov solve from v = 0 (departure points, state,
objective, adjoint, gradient, PCG with Hessian matvecs, line search).
value = Hessian matvecs per second of the whole job: matvecs performed in
the K timed solves divided by their wall time.  The matvec-only rate (median
of 5 runs of 100 matvecs at the generating velocity, eager and replayed from
a captured HIP graph), the per-kernel breakdown (HIP events on the library stream) and the dominant
kernel's HBM roofline are reported beside it, and the FP64 CPU oracle is
timed on a bounded sample of the same recipe as the CPU baseline.  The
FP16-storage variant (FP32 arithmetic, adjoint and incremental fields held in
FP16) is timed on the same inputs and reported in "precision_variant".
"two_level" repeats the timed solves with the two-level coarse-grid
preconditioner (coarse grid 128^3, nested CG to kappa times the PCG
tolerance; kappa 0.1 as in the paper, and 0.5).
"batched" solves the uneven batch -- 16 pairs at 64^3, 16 at 96^3, 12 at
128^3 and 4 at 160^3 -- with four concurrent streams, graph-captured matvecs
and autotuned tiles, against one stream without either, and in lockstep
(all 48 pairs in one mireg batch: one launch per transport step across the
pairs, one launch per Krylov pass per grid size).
"warm_start" compares solves of held-out 128^3 pairs from v = 0 and from the
trained network's prediction (paper_1808_04487_amd/weights) to the same
absolute gradient tolerance.  "analytic_32" gives the time to tolerance of
the paper's analytic problem at 32^3 in FP64, on the GPU and (with the CPU
baseline) by the FP64 oracle on the host cores, with their iteration
counters.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, vendor figure
TWO_PI = 2.0 * math.pi


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed GN solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed GN solves")
    ap.add_argument("--n", type=int, default=256, help="grid size per axis")
    ap.add_argument("--matvecs", type=int, default=100,
                    help="matvecs per timed run of the matvec-only timing (median of 5 runs)")
    ap.add_argument("--cpu-n", type=int, default=256,
                    help="grid of the CPU-oracle sample (the workload's own size by default: no scaling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-variant", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--no-two-level", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: PCG replays its matvecs (and the nested coarse CG's) from captured HIP graphs")
    ap.add_argument("--warm-pairs", type=int, default=16, help="held-out pairs of the warm-start comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before the timed region, run a fill and a multiply over 1 GiB (known "
                         "traffic) as the reference for memory-traffic counters")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(ctx, n, torch):
    """Config recipe on the GPU with the library's own operators."""
    from paper_1808_04487_amd import synth

    dev = ctx.device
    raw = torch.from_numpy(synth.voronoi_phantom((n, n, n), nseeds=120, seed=1)).to(dev, torch.float32)
    mT = ctx.op("rescale01", ctx.op("gauss", raw, 2.0))
    sig = n / 8.0  # physical sigma pi/4 in cells

    def smooth_velocity(seed):
        noise = torch.from_numpy(synth.white_noise((n, n, n), seed=seed)).to(dev, torch.float32)
        sm = torch.stack([ctx.op("gauss", noise[c].contiguous(), sig) for c in range(3)]).contiguous()
        return ctx.op("scale_maxnorm", ctx.op("leray", sm), 0.15 * TWO_PI)

    v_true = smooth_velocity(2)
    probe = smooth_velocity(3)
    ctx.set_velocity(v_true)
    mR = ctx.op("transport_state", mT)
    ctx.set_velocity(torch.zeros_like(v_true))
    return mT, mR, v_true, probe


def cpu_baseline(args):
    """FP64 oracle on the host cores: per-velocity setup (departure points,
    state history, state gradients, adjoint), then one Hessian matvec on the
    workload itself at the default --cpu-n = 256; a smaller --cpu-n times two
    matvecs there and scales their rate by the point count (the matvec is
    O(N) transport work), and the unit says so."""
    import numpy as np

    from oracle import core, prep
    from paper_1808_04487_amd import synth

    m = args.cpu_n
    n = (m, m, m)
    g = core.Grid(n)
    raw = synth.voronoi_phantom(n, nseeds=120, seed=1)
    mT = prep.smooth_rescale(g, raw, 2.0)
    v_true = prep.smooth_velocity(g, synth.white_noise(n, seed=2), math.pi / 4, 0.15 * TWO_PI)
    probe = prep.smooth_velocity(g, synth.white_noise(n, seed=3), math.pi / 4, 0.15 * TWO_PI)
    mR = prep.transport(g, mT, v_true)
    p = core.Params(n, nt=4, order=3, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=5e-3, beta_w=1.0)
    R = core.Registration(p, mT, mR)
    R.set_velocity(v_true)
    t0 = time.perf_counter()
    R.gradient()  # builds X, Y, state history, grad m, div v
    t_setup = time.perf_counter() - t0
    reps = 1 if m >= args.n else 2
    t0 = time.perf_counter()
    for _ in range(reps):
        R.hessian_matvec(probe)
    t_mv = (time.perf_counter() - t0) / reps
    scale = (m ** 3) / float(args.n ** 3)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    unit = ("Hessian matvecs/s at %d^3" % args.n if m == args.n else
            "Hessian matvecs/s at %d^3 (scaled from %d^3 by point count)" % (args.n, m))
    return {
        "value": round(scale / t_mv, 6),
        "unit": unit,
        "cores": cores,
        "kind": "oracle",
        "sample": "FP64 oracle, %d^3 same recipe: setup (state, adjoint, gradient caches) %.2f s, "
                  "%d GN Hessian matvec%s at %.2f s each" % (m, t_setup, reps, "" if reps == 1 else "s", t_mv),
    }


OPTS = dict(grad_rtol=5e-2, grad_atol=1e-6, max_gn=50, max_pcg=100)
ANALYTIC_OPTS = dict(grad_rtol=1e-2, grad_atol=1e-6, max_gn=50, max_pcg=100)
ANALYTIC_KEYS = ("status", "gn_iters", "matvecs", "pde_solves", "ls_trials")


def analytic_gpu(args, torch, mireg):
    """The paper's analytic problem at 32^3 in FP64 (H1-div, beta_v = 1e-2,
    beta_w = 1, nt = 4, tricubic, relative gradient 1e-2): the reference is
    the template transported by the library; median time to tolerance of 5
    solves from v = 0 after one untimed."""
    from paper_1808_04487_amd import synth

    n = (32, 32, 32)
    ctx = mireg.Context(n, nt=4, order=3, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=1e-2, beta_w=1.0,
                        dtype=torch.float64)
    mT = torch.from_numpy(synth.trig_template(n)).to(ctx.device)
    ctx.set_velocity(torch.from_numpy(synth.trig_velocity(n)).to(ctx.device))
    mR = ctx.op("transport_state", mT)
    ctx.set_velocity(torch.zeros((3,) + n, dtype=torch.float64, device=ctx.device))
    ctx.set_images(mT, mR)
    ctx.gn_solve(**ANALYTIC_OPTS)
    ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = ctx.gn_solve(**ANALYTIC_OPTS)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ctx.close()
    out = {k: rep[k] for k in ANALYTIC_KEYS + ("mismatch_rel", "gnorm_rel")}
    out["time_to_tol_s"] = round(sorted(ts)[2], 5)
    return out


def analytic_cpu(args):
    """The same problem solved by the FP64 oracle on the host cores (its own
    reference image), for the CPU baseline."""
    import numpy as np

    from oracle import core, prep, solver
    from paper_1808_04487_amd import synth

    n = (32, 32, 32)
    g = core.Grid(n)
    mT = synth.trig_template(n)
    mR = prep.transport(g, mT, synth.trig_velocity(n))
    p = core.Params(n, nt=4, order=3, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=1e-2, beta_w=1.0)
    R = core.Registration(p, mT, mR)
    t0 = time.perf_counter()
    _, rep = solver.gn_solve(R, np.zeros((3,) + n), **ANALYTIC_OPTS)
    t = time.perf_counter() - t0
    out = {k: getattr(rep, k) for k in ANALYTIC_KEYS + ("mismatch_rel",)}
    out["time_to_tol_s"] = round(t, 4)
    return out


def timed_solves(args, ctx, torch, warmup, steps):
    """GN solves from v = 0: `warmup` untimed, then `steps` timed back to back."""
    for w in range(warmup):
        _, rep = ctx.gn_solve(**OPTS)
        log(args, "warmup solve %d: %s" % (w, rep))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(steps):
        _, rep = ctx.gn_solve(**OPTS)
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k, rep in enumerate(reps):
        log(args, "timed solve %d: %s" % (k, rep))
    return reps, wall


def matvec_ms(args, ctx, torch, v, probe, graphs=False):
    """Matvec-only time at velocity v with the probe direction: 10 untimed
    matvecs, then the median over 5 runs of `matvecs` matvecs (events on the
    library stream); graphs: the entry point replays a captured graph."""
    ctx.set_velocity(v)
    ctx.set_graphs(graphs)
    out = ctx.empty(3)
    for _ in range(10):
        ctx.hessian_matvec(probe, out)
    runs = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.matvecs):
            ctx.hessian_matvec(probe, out)
        e1.record(ctx.stream)
        e1.synchronize()
        runs.append(e0.elapsed_time(e1) / args.matvecs)
    ctx.set_graphs(bool(args.graphs))
    ms = sorted(runs)[2]
    log(args, "matvec-only (%s, %s): %.3f ms (%.1f matvecs/s)" % (ctx.dtype_name, "graph" if graphs else "eager",
                                                                   ms, 1000.0 / ms))
    return ms


def precision_variant(args, torch, mireg, n, mT, mR, v_true, probe, plain):
    """The same workload with FP16 storage of the adjoint and incremental
    fields: one warm-up and `steps` timed solves, the matvec-only rate, and
    the final mismatch against the plain FP32 solve's."""
    ctx = mireg.Context((n, n, n), nt=4, order=3, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=5e-3,
                        beta_w=1.0, dtype="f32h16")
    ctx.set_images(mT, mR)
    reps, wall = timed_solves(args, ctx, torch, 1, args.steps)
    ms = matvec_ms(args, ctx, torch, v_true, probe)
    ctx.close()
    rep = reps[-1]
    return {
        "dtype": "f32 compute, f16 storage of lambda, mt, lt",
        "time_to_tol_s": round(wall / max(1, args.steps), 4),
        "matvecs_per_s": round(sum(r["matvecs"] for r in reps) / wall, 3),
        "matvec_only_per_s": round(1000.0 / ms, 2),
        "matvec_ms": round(ms, 4),
        "solve": {k: rep[k] for k in ("status", "gn_iters", "matvecs", "mismatch_rel", "gnorm_rel")},
        "mismatch_rel_change_vs_plain": round(abs(rep["mismatch_rel"] - plain["mismatch_rel"])
                                              / plain["mismatch_rel"], 6),
    }


def batched_eval(args, torch, mireg):
    """Uneven batch: sequential (one stream, eager) vs batched (4 streams,
    graphs, autotuner) vs hybrid (the same, with the 64^3 pairs in lockstep
    groups of 8) vs lockstep (all pairs in one batch: one launch per
    transport step across them); each configuration runs once untimed first."""
    from paper_1808_04487_amd import batch

    sizes = batch.UNEVEN_BATCH
    pairs = batch.make_pairs(sizes)
    out = {"workload": "16 pairs at 64^3, 16 at 96^3, 12 at 128^3, 4 at 160^3, seeds (100+2p, 101+2p), "
                       "amplitude U[0.05, 0.2] 2 pi; H1-div beta_v=5e-3, eps_g=5e-2", "pairs": len(sizes),
           "points": int(sum(n ** 3 for n in sizes))}
    for key, kw in (("sequential", dict(workers=1, graphs=False, autotune=False)),
                    ("batched", dict(workers=4, graphs=True, autotune=True)),
                    ("hybrid", dict(workers=4, graphs=True, autotune=True, lockstep={64: 8}))):
        bs = batch.BatchSolver(**kw)
        bs.solve(pairs, grad_rtol=5e-2)
        res, wall = bs.solve(pairs, grad_rtol=5e-2)
        bs.close()
        mv = sum(r[1]["matvecs"] for r in res)
        out[key] = {"wall_s": round(wall, 4), "pairs_per_s": round(len(sizes) / wall, 2),
                    "matvecs": mv, "points_matvecs_per_s": round(sum(r[1]["matvecs"] * p[0].numel()
                                                                   for r, p in zip(res, pairs)) / wall, 1)}
        log(args, "%s: %.3f s for %d pairs" % (key, wall, len(sizes)))
    out["speedup"] = round(out["sequential"]["wall_s"] / out["batched"]["wall_s"], 3)
    out["hybrid"]["speedup"] = round(out["sequential"]["wall_s"] / out["hybrid"]["wall_s"], 3)
    # lockstep: one context per pair on one stream; each transport step of the
    # Hessian matvec is one launch across all running pairs, each Krylov pass
    # one launch per grid size, one PCG read-back per iteration for all
    ctxs = [mireg.Context(tuple(p[0].shape), dtype=torch.float32, **batch.SOLVER) for p in pairs]
    for c, (mT, mR) in zip(ctxs, pairs):
        c.set_images(mT, mR)
    B = mireg.Batch(ctxs)
    B.gn_solve(grad_rtol=5e-2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, reps = B.gn_solve(grad_rtol=5e-2)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.close()
    for c in ctxs:
        c.close()
    out["lockstep"] = {"wall_s": round(wall, 4), "pairs_per_s": round(len(sizes) / wall, 2),
                       "matvecs": sum(r["matvecs"] for r in reps),
                       "points_matvecs_per_s": round(sum(r["matvecs"] * p[0].numel()
                                                         for r, p in zip(reps, pairs)) / wall, 1)}
    log(args, "lockstep: %.3f s for %d pairs" % (wall, len(sizes)))
    return out


def warm_start_eval(args, torch):
    """Plain vs warm-started GN-Krylov solves of held-out 128^3 pairs (seeds
    3000000 on, disjoint from training and from the recorded evaluation)."""
    from paper_1808_04487_amd import warmstart

    path = os.path.join(warmstart.WEIGHTS_DIR, "warmstart_128.npz")
    net = warmstart.WarmStartNet.load(path)
    ctx = warmstart.registration_context(net.n)
    mT, mR, _, _, _ = warmstart.make_pair(net, ctx, 2999999, solve=False)
    warmstart.solve_pair(ctx, mT, mR, net)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(5):
        net.forward(mT, mR)
    e1.record(net.stream)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    rows = []
    for s in range(3000000, 3000000 + args.warm_pairs):
        mT, mR, _, _, _ = warmstart.make_pair(net, ctx, s, solve=False)
        r = warmstart.solve_pair(ctx, mT, mR, net)
        (p, tp), (w, tw, used) = r["plain"], r["warm"]
        rows.append((p["gn_iters"], w["gn_iters"], p["matvecs"], w["matvecs"], tp, tw, p["mismatch_rel"],
                     w["mismatch_rel"], float(used)))
    ctx.close()
    net.close()
    import numpy as np
    a = np.array(rows)
    m = a.mean(axis=0)
    log(args, "warm start: plain %.2f GN %.1f ms, warm %.2f GN %.1f ms" % (m[0], 1e3 * m[4], m[1], 1e3 * m[5]))
    return {"workload": "held-out 128^3 Voronoi pairs, velocity amplitude U[0.05, 0.15] 2 pi, H1-div "
                        "beta_v=5e-3, same absolute gradient tolerance (5e-2 |g(0)|)",
            "pairs": len(rows), "plain_time_to_tol_s": round(m[4], 5), "warm_time_to_tol_s": round(m[5], 5),
            "speedup": round(m[4] / m[5], 3), "plain_gn_iters": round(m[0], 3), "warm_gn_iters": round(m[1], 3),
            "plain_matvecs": round(m[2], 2), "warm_matvecs": round(m[3], 2),
            "plain_mismatch_rel": round(m[6], 6), "warm_mismatch_rel": round(m[7], 6),
            "prediction_used_fraction": round(m[8], 3), "network_forward_ms": round(fwd_ms, 3)}


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    import torch

    from paper_1808_04487_amd import mireg

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    n = args.n
    ctx = mireg.Context((n, n, n), nt=4, order=3, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=5e-3,
                        beta_w=1.0, dtype=torch.float32)
    ctx.set_graphs(bool(args.graphs))
    log(args, "context %d^3, workspace %.2f GB" % (n, ctx.workspace_bytes() / 1e9))
    t0 = time.perf_counter()
    mT, mR, v_true, probe = make_inputs(ctx, n, torch)
    ctx.set_images(mT, mR)
    torch.cuda.synchronize()
    log(args, "inputs ready in %.1f s" % (time.perf_counter() - t0))
    if args.copy_calibration:
        # fill: writes 1 GiB; multiply: reads 1 GiB and writes 1 GiB
        a = torch.ones(1 << 28, dtype=torch.float32, device=ctx.device)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

    reps, wall = timed_solves(args, ctx, torch, args.warmup, args.steps)
    total_mv = sum(r["matvecs"] for r in reps)
    value = total_mv / wall
    mv_ms = matvec_ms(args, ctx, torch, v_true, probe)
    mv_graph_ms = matvec_ms(args, ctx, torch, v_true, probe, graphs=True)
    out = ctx.empty(3)

    # per-kernel event timing over a separate run of matvecs
    ctx.kernel_stats(enable=True, reset=True)
    for _ in range(args.matvecs):
        ctx.hessian_matvec(probe, out)
    stats = ctx.kernel_stats(enable=False, reset=True)
    per_mv = {k: (v[1] / args.matvecs, v[0] / args.matvecs, v[1] / v[0], v[2]) for k, v in stats.items()}
    dom = max(per_mv, key=lambda k: per_mv[k][0])
    avg_ms, bytes_launch = per_mv[dom][2], per_mv[dom][3]
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    kernels = {k: {"ms_per_matvec": round(v[0], 4), "launches_per_matvec": v[1],
                   "avg_ms": round(v[2], 4), "GBps": round(v[3] / (v[2] * 1e-3) / 1e9, 1),
                   "hbm_frac": round(v[3] / (v[2] * 1e-3) / 1e9 / PEAK_HBM_GBS, 3)}
               for k, v in sorted(per_mv.items(), key=lambda kv: -kv[1][0])}
    # the per-kernel goal of half the HBM roofline, stated next to the solve rate
    below = {k: v["hbm_frac"] for k, v in kernels.items() if v["hbm_frac"] < 0.5}
    kernel_target = {"target_frac": 0.5, "met": not below, "kernels_below": below}
    for k, v in kernels.items():
        log(args, "kernel %-18s %s" % (k, v))
    fft_ms = sum(v[0] for k, v in per_mv.items() if k.startswith("fft"))
    sl_ms = sum(v[0] for k, v in per_mv.items() if k.startswith("sl_"))

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            from paper_1808_04487_amd import build as hb

            t = json.load(open(tpath))
            if t.get("source_sha") == hb.source_sha():
                traffic = t.get("bytes_per_launch", {}).get(dom)
        except Exception:
            traffic = None

    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "bytes_per_launch": bytes_launch, "avg_launch_ms": round(avg_ms, 5)}

    two = None
    if not args.no_two_level:
        two = {"coarse_grid": [n // 2] * 3, "max_inner": 50}
        for kappa, key in ((0.1, "kappa_0.1"), (0.5, "kappa_0.5")):
            log(args, "two-level preconditioner, kappa %.1f" % kappa)
            ctx.set_precond("two_level", kappa=kappa, max_inner=50)
            treps, twall = timed_solves(args, ctx, torch, 1, args.steps)
            tr = treps[-1]
            two[key] = {"time_to_tol_s": round(twall / max(1, args.steps), 4),
                        "speedup_vs_spectral": round(wall / twall, 3),
                        "solve": {k: tr[k] for k in ("status", "gn_iters", "matvecs", "coarse_matvecs",
                                                     "mismatch_rel", "gnorm_rel")}}
        ctx.set_precond("spectral")

    bat = None
    if not args.no_batched:
        log(args, "batched uneven solves")
        bat = batched_eval(args, torch, mireg)

    warm = None
    if not args.no_warm_start:
        log(args, "warm-start comparison")
        warm = warm_start_eval(args, torch)

    prec = None
    if not args.no_precision_variant:
        log(args, "FP16-storage variant")
        prec = precision_variant(args, torch, mireg, n, mT, mR, v_true, probe, reps[-1])

    log(args, "analytic problem, 32^3 FP64")
    analytic = {"workload": "the paper's analytic problem (Sec. 4.2) at 32^3 FP64, H1-div beta_v=1e-2 beta_w=1, "
                            "nt=4 tricubic, spectral PC, relative gradient 1e-2",
                "gpu": analytic_gpu(args, torch, mireg)}

    cpu = None
    if not args.no_cpu_baseline:
        log(args, "timing the CPU oracle sample")
        cpu = cpu_baseline(args)
        analytic["cpu_oracle"] = analytic_cpu(args)
        analytic["same_counters"] = all(analytic["gpu"][k] == analytic["cpu_oracle"][k] for k in ANALYTIC_KEYS)

    solve_s = wall / max(1, args.steps)
    line = {
        "metric": "Hessian matvecs/s at 256^3 (whole GN-Krylov solve), time-to-tol, fraction of HBM BW",
        "value": round(value, 3),
        "unit": "Hessian matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * solve_s, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "voronoi-phantom registration %d^3 FP32, H1-div beta_v=5e-3 beta_w=1, "
                               "nt=4 tricubic, spectral PC, eps_g=5e-2" % n,
                   "grid": [n, n, n], "nt": 4, "parallelism": "single-gpu"},
        "time_to_tol_s": round(solve_s, 4),
        "per_kernel_hbm_target": kernel_target,
        "solve": {k: reps[-1][k] for k in ("status", "gn_iters", "matvecs", "pde_solves", "ls_trials",
                                            "mismatch_rel", "gnorm_rel")},
        "matvec_only_per_s": round(1000.0 / mv_ms, 2),
        "matvec_ms": round(mv_ms, 4),
        "matvec_graph_per_s": round(1000.0 / mv_graph_ms, 2),
        "matvec_graph_ms": round(mv_graph_ms, 4),
        "fft_ms_per_matvec": round(fft_ms, 4),
        "interp_ms_per_matvec": round(sl_ms, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_variant": prec,
        "two_level": two,
        "batched": bat,
        "warm_start": warm,
        "analytic_32": analytic,
        "kernels": kernels,
    }
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
