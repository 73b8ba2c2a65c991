"""Train the warm-start network on pairs the solver generates, then compare
warm-started and zero-initialised solves on held-out pairs.

  python -m paper_1808_04487_amd.train_warmstart --n 128 --pairs 768 --steps 3000 \
      --out paper_1808_04487_amd/weights/warmstart_128.npz

Pairs use seeds 0..pairs-1; held-out pairs use seeds from 1000000 on.  One
line of progress is printed at least every few seconds.  With --init WEIGHTS
and --steps 0 only the held-out evaluation of those weights runs:

  python -m paper_1808_04487_amd.train_warmstart --init paper_1808_04487_amd/weights/warmstart_128.npz \
      --pairs 0 --steps 0 --eval 256 --report eval.json

With --sizes (a comma list of training-set sizes) the pairs are generated
once, for the largest size, and a fresh network is trained on the first
`size` of them for each size (same steps, learning rate and seed) and
evaluated on the same held-out pairs; no weights are saved:

  python -m paper_1808_04487_amd.train_warmstart --sizes 256,1024,3072 --steps 6000 --eval 128 \
      --report sizes.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1808_04487_amd import warmstart  # noqa: E402
else:
    from . import warmstart

HELD_OUT_SEED = 1000000


def log(*a):
    print("[train]", *a, flush=True)


def generate(net, ctx, seeds, solve=True):
    pairs, t0, last = [], time.perf_counter(), time.perf_counter()
    for k, s in enumerate(seeds):
        mT, mR, vt, _, rep = warmstart.make_pair(net, ctx, int(s), solve=solve)
        pairs.append((mT, mR, vt))
        if time.perf_counter() - last > 10 or k == len(seeds) - 1:
            last = time.perf_counter()
            log("pairs %d/%d (%.1f s)%s" % (k + 1, len(seeds), last - t0,
                                           " gn %d matvecs %d" % (rep["gn_iters"], rep["matvecs"]) if rep else ""))
    return pairs


def evaluate(net, ctx, seeds):
    rows = []
    for s in seeds:
        mT, mR, _, _, _ = warmstart.make_pair(net, ctx, int(s), solve=False)
        r = warmstart.solve_pair(ctx, mT, mR, net)
        p, tp = r["plain"]
        w, tw, used = r["warm"]
        rows.append({"seed": int(s), "plain_gn": p["gn_iters"], "plain_matvecs": p["matvecs"], "plain_s": tp,
                     "plain_mismatch": p["mismatch_rel"], "plain_gnorm": p["gnorm"], "warm_gn": w["gn_iters"],
                     "warm_matvecs": w["matvecs"], "warm_s": tw, "warm_mismatch": w["mismatch_rel"],
                     "warm_gnorm": w["gnorm"], "used": bool(used), "warm_status": w["status"]})
        log("eval seed %d: plain %d GN %.3f s mismatch %.4f | warm %d GN %.3f s mismatch %.4f%s" % (
            s, p["gn_iters"], tp, p["mismatch_rel"], w["gn_iters"], tw, w["mismatch_rel"],
            "" if used else " (fallback)"))
    return rows


def summary(rows):
    f = lambda k: float(np.mean([r[k] for r in rows]))
    return {"pairs": len(rows), "plain_gn_mean": f("plain_gn"), "warm_gn_mean": f("warm_gn"),
            "plain_matvecs_mean": f("plain_matvecs"), "warm_matvecs_mean": f("warm_matvecs"),
            "plain_s_mean": f("plain_s"), "warm_s_mean": f("warm_s"),
            "plain_mismatch_mean": f("plain_mismatch"), "warm_mismatch_mean": f("warm_mismatch"),
            "fallbacks": int(sum(not r["used"] for r in rows))}


def train(net, pairs, steps, batch, lr0, seed):
    t0 = last = time.perf_counter()
    rng = np.random.default_rng(seed)
    loss = float("nan")
    for s in range(steps):
        lr = lr0 * 0.5 * (1.0 + np.cos(np.pi * s / steps))  # cosine decay
        idx = rng.choice(len(pairs), size=batch, replace=False)
        loss = net.train_step([pairs[i] for i in idx], lr)
        if time.perf_counter() - last > 10 or s == steps - 1:
            last = time.perf_counter()
            log("step %d/%d loss %.4e lr %.2e (%.1f s)" % (s + 1, steps, loss, lr, last - t0))
    return loss, time.perf_counter() - t0


def size_study(args, ctx):
    sizes = sorted(int(x) for x in args.sizes.split(","))
    net = warmstart.WarmStartNet(args.n)
    t0 = time.perf_counter()
    pairs = generate(net, ctx, range(sizes[-1]))
    t_gen = time.perf_counter() - t0
    out = {"args": vars(args), "generate_s": t_gen, "sizes": []}
    for size in sizes:
        net.set_params(warmstart.init_params(warmstart.CHANNELS, args.seed))
        log("training on %d pairs" % size)
        loss, t_train = train(net, pairs[:size], args.steps, args.batch, args.lr, args.seed)
        rows = evaluate(net, ctx, range(HELD_OUT_SEED, HELD_OUT_SEED + args.eval))
        summ = summary(rows)
        summ.update({"train_pairs": size, "final_train_loss": loss, "train_s": t_train,
                     "gn_ratio": summ["plain_gn_mean"] / summ["warm_gn_mean"],
                     "matvec_ratio": summ["plain_matvecs_mean"] / summ["warm_matvecs_mean"],
                     "time_ratio": summ["plain_s_mean"] / summ["warm_s_mean"]})
        log("size %d: %s" % (size, json.dumps(summ)))
        out["sizes"].append(summ)
    if args.report:
        json.dump(out, open(args.report, "w"), indent=1)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--pairs", type=int, default=768)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval", type=int, default=16, help="held-out pairs")
    ap.add_argument("--out", default=os.path.join(warmstart.WEIGHTS_DIR, "warmstart_128.npz"))
    ap.add_argument("--report", default=None, help="JSON file for the evaluation")
    ap.add_argument("--init", default=None, help="start from these weights (with --steps 0: evaluate them only)")
    ap.add_argument("--sizes", default=None, help="comma list of training-set sizes to compare (no weights saved)")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.sizes:
        ctx = warmstart.registration_context(args.n)
        return size_study(args, ctx)
    if args.init:
        net = warmstart.WarmStartNet.load(args.init)
        if net.n != args.n:
            raise SystemExit("weights are for n = %d, not %d" % (net.n, args.n))
    else:
        net = warmstart.WarmStartNet(args.n)
        net.set_params(warmstart.init_params(warmstart.CHANNELS, args.seed))
    ctx = warmstart.registration_context(args.n)
    log("network %d parameters, n = %d" % (net.param_count, args.n))
    pairs = generate(net, ctx, range(args.pairs))
    if args.steps > 0:
        train(net, pairs, args.steps, args.batch, args.lr, args.seed)
    if args.steps > 0:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        net.save(args.out)
        log("saved", args.out)
    del pairs
    rows = evaluate(net, ctx, range(HELD_OUT_SEED, HELD_OUT_SEED + args.eval))
    summ = summary(rows)
    log(json.dumps(summ))
    if args.report:
        json.dump({"summary": summ, "rows": rows, "args": vars(args)}, open(args.report, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
