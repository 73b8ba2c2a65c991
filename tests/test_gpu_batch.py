"""Batched solves of pairs of uneven sizes, graph-captured matvecs and the
tile-shape autotuner: none of them may change a result bit."""
import numpy as np
import pytest
import torch

from oracle import core, prep
from paper_1808_04487_amd import batch, mireg, synth

from gpu_util import as_input, need_gpu, smooth_vector

pytestmark = pytest.mark.gpu


def synthetic_ctx(n, dtype=torch.float32):
    g = core.Grid(n)
    mT = synth.trig_template(n)
    vs = synth.trig_velocity(n)
    mT_t, _ = as_input(mT, dtype)
    mR_t, _ = as_input(prep.transport(g, mT, vs), dtype)
    ctx = mireg.Context(n, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=1e-2, beta_w=1.0, dtype=dtype)
    ctx.set_images(mT_t, mR_t)
    return g, ctx, vs


def test_graph_replays_match_eager():
    """PCG with its matvec replayed from a captured graph equals eager PCG,
    bit for bit, across velocity changes and with eager work between."""
    need_gpu()
    n = (64, 64, 64)
    g, ctx, vs = synthetic_ctx(n)
    rhs = torch.from_numpy(smooth_vector(g, 91)).float().cuda()
    probe = torch.from_numpy(smooth_vector(g, 92)).float().cuda()
    for scale in (0.5, 0.8, 0.8):
        ctx.set_velocity(torch.from_numpy(scale * vs).float().cuda())
        ctx.set_graphs(False)
        x0, it0, _ = ctx.pcg(rhs, rtol=1e-6, maxit=12)
        h0 = ctx.hessian_matvec(probe)
        ctx.set_graphs(True)
        x1, it1, _ = ctx.pcg(rhs, rtol=1e-6, maxit=12)      # capture, then replays
        h1 = ctx.hessian_matvec(probe)                        # eager call between replays
        torch.cuda.synchronize()
        x2, it2, _ = ctx.pcg(rhs, rtol=1e-6, maxit=12)      # replays of the same graph
        print("velocity scale", scale, "iterations", it0, it1, it2, flush=True)
        assert it0 == it1 == it2 >= 3
        assert torch.equal(x0, x1) and torch.equal(x0, x2) and torch.equal(h0, h1)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_matvec_entry_graph_replays_match_eager(dtype):
    """The matvec entry point replayed from a captured graph equals the eager
    matvec bit for bit on every replay, with eager library and torch work and
    synchronisations between replays; new input buffers, a new velocity and
    PCG's own graph in between each force a re-capture."""
    need_gpu()
    n = (64, 64, 64)
    g, ctx, vs = synthetic_ctx(n, dtype)
    probes = [torch.from_numpy(smooth_vector(g, s)).to(dtype).cuda() for s in (94, 95)]
    rhs = torch.from_numpy(smooth_vector(g, 96)).to(dtype).cuda()
    out = ctx.empty(3)
    for scale in (0.6, 0.9):
        ctx.set_velocity(torch.from_numpy(scale * vs).to(dtype).cuda())
        ctx.set_graphs(False)
        ref = [ctx.hessian_matvec(p).clone() for p in probes]
        ctx.set_graphs(True)
        for rep in range(3):
            for k, p in enumerate(probes):
                ctx.hessian_matvec(p, out)                      # capture for this (vt, Hvt), then replay
                torch.cuda.synchronize()
                assert torch.equal(out, ref[k]), (scale, rep, k)
                ctx.hessian_matvec(p, out)                      # replay of the same graph
                torch.cuda.synchronize()
                assert torch.equal(out, ref[k]), (scale, rep, k)
                ctx.op("grad", probes[0][0])                    # eager library work
                (probes[1] * 2.0).sum().item()                  # eager torch work and a sync
            if rep == 1:
                ctx.pcg(rhs, rtol=1e-3, maxit=5)                # PCG's spectral graph in between
        print("velocity scale", scale, "replays equal", flush=True)
    ctx.set_graphs(False)
    assert torch.equal(ctx.hessian_matvec(probes[1]), ref[1])
    ctx.close()


def test_autotune_keeps_results():
    need_gpu()
    n = (64, 64, 64)
    g, ctx, vs = synthetic_ctx(n)
    ctx.set_velocity(torch.from_numpy(0.7 * vs).float().cuda())
    probe = torch.from_numpy(smooth_vector(g, 93)).float().cuda()
    before = ctx.hessian_matvec(probe)
    shape, ms = ctx.autotune(reps=2)
    print("autotune", shape, ms, flush=True)
    assert shape in (0, 1, 2) and all(m > 0 for m in ms)
    assert ms[shape] == min(ms)
    assert torch.equal(ctx.hessian_matvec(probe), before)


def test_autotune_krylov_width_at_256():
    """FP32 256^3: the Krylov x1 passes in 16-column workgroups give the
    same PCG as the default 32 (same iterations; the FP64 partial sums of
    <s, Hs> are grouped differently, so the iterates agree to rounding), the
    matvec entry point is bit for bit the same, and the autotuner, which
    times both widths with every tile shape, leaves the matvec unchanged."""
    need_gpu()
    n = 256
    (mT, mR), = batch.make_pairs([n])
    ctx = mireg.Context((n, n, n), dtype=torch.float32, **batch.SOLVER)
    ctx.set_images(mT, mR)
    noise = torch.randn((3, n, n, n), generator=torch.Generator().manual_seed(5)).cuda()
    sm = torch.stack([ctx.op("gauss", noise[c].contiguous(), n / 8.0) for c in range(3)]).contiguous()
    ctx.set_velocity(ctx.op("scale_maxnorm", ctx.op("leray", sm), 0.5))
    probe = ctx.op("leray", torch.stack([ctx.op("gauss", noise[c].flip(0).contiguous(), 16.0) for c in range(3)]))
    assert ctx.tuning() == (1, 0)
    before = ctx.hessian_matvec(probe).clone()
    xw, itw, _ = ctx.pcg(probe, rtol=1e-3, maxit=40)
    ctx.set_tuning(1, 1)
    assert ctx.tuning() == (1, 1)
    assert torch.equal(ctx.hessian_matvec(probe), before)
    xn, itn, _ = ctx.pcg(probe, rtol=1e-3, maxit=40)
    e = ((xn - xw).norm() / xw.norm()).item()
    print("pcg 32 vs 16 columns: iterations %d / %d, rel diff %.2e" % (itw, itn, e), flush=True)
    assert itw == itn and e < 1e-5
    shape, ms = ctx.autotune(reps=2)
    print("autotune", shape, ms, ctx.tuning(), flush=True)
    assert ctx.tuning()[0] == shape and ms[shape] == min(ms)
    assert torch.equal(ctx.hessian_matvec(probe), before)
    with pytest.raises(mireg.MiregError):
        ctx.set_tuning(3, 0)
    ctx.close()


def test_batched_solves_equal_sequential():
    need_gpu()
    sizes = [32, 96, 48, 64, 48, 32, 16]  # power-of-two and radix-3 grids
    pairs = batch.make_pairs(sizes)
    seq = batch.BatchSolver(workers=1, graphs=False, autotune=False)
    rs, ts = seq.solve(pairs, grad_rtol=5e-2)
    par = batch.BatchSolver(workers=3, graphs=True, autotune=True)
    rp, tp = par.solve(pairs, grad_rtol=5e-2)
    print("sequential %.3f s, batched %.3f s" % (ts, tp), flush=True)
    for (vs_, a), (vp_, b) in zip(rs, rp):
        for k in ("status", "gn_iters", "matvecs", "ls_trials", "mismatch_rel", "gnorm"):
            assert a[k] == b[k], (k, a[k], b[k])
        assert torch.equal(vs_, vp_)
    assert all(r[1]["status"] == mireg.CONVERGED_REL for r in rp)
    seq.close()
    par.close()


REPORT_KEYS = ("status", "gn_iters", "matvecs", "pde_solves", "pcg_iters", "ls_trials", "neg_curv", "J0", "J",
               "mismatch_rel", "gnorm0", "gnorm", "gnorm_rel")  # printed in the oracle comparison


def test_hybrid_batch_matches_single_solves():
    """Worker streams with same-size pairs grouped into lockstep batches
    (here the 32^3 pairs in groups of 3, the rest one pair per job) against
    the pairs solved one by one: single-pair jobs bit for bit, grouped pairs
    to the FP32 lockstep bounds (same status and J0, iterations within one,
    J and relative mismatch within 1e-2)."""
    need_gpu()
    sizes = [32, 48, 32, 32, 16, 32, 32, 32]
    pairs = batch.make_pairs(sizes)
    seq = batch.BatchSolver(workers=1, graphs=False, autotune=False)
    ref, _ = seq.solve(pairs, grad_rtol=5e-2)
    seq.close()
    hyb = batch.BatchSolver(workers=2, graphs=True, autotune=False, lockstep={32: 3})
    assert sorted(len(j) for j in hyb._jobs(pairs)) == [1, 1, 3, 3]
    got, _ = hyb.solve(pairs, grad_rtol=5e-2)
    hyb.close()
    for n, (v, rep), (vr, rr) in zip(sizes, got, ref):
        print("hybrid", n, rep["gn_iters"], rep["J"], "single", rr["gn_iters"], rr["J"], flush=True)
        assert rep["status"] == rr["status"] == mireg.CONVERGED_REL
        if n != 32:
            assert torch.equal(v, vr) and rep["J"] == rr["J"] and rep["matvecs"] == rr["matvecs"]
        else:
            assert abs(rep["gn_iters"] - rr["gn_iters"]) <= 1
            assert rep["J0"] == rr["J0"]
            for k in ("J", "mismatch_rel"):
                assert abs(rep[k] - rr[k]) <= 1e-2 * abs(rr[k]), k


def _lockstep_contexts(sizes, dtype):
    """Contexts of the given grid sizes on the current stream, each with a
    synthetic pair of its own (the paper's analytic problem at that size)."""
    out = []
    for k, n in enumerate(sizes):
        g, ctx, vs = synthetic_ctx(n, dtype)
        out.append((g, ctx, vs))
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_lockstep_pcg_matches_single_problem_pcg(dtype):
    """Lockstep PCG over problems of uneven sizes (one transport launch per
    matvec step across them, one launch per Krylov pass per grid size)
    against the single-problem PCG of each problem, also when problems stop
    at different iterations and one has a zero right-hand side: the same
    iterations and status, relative residual and iterate to rounding (the
    multi-problem kernels are separate instantiations whose operation
    contraction may differ)."""
    need_gpu()
    sizes = [(16, 16, 16), (48, 48, 48), (32, 16, 64), (16, 32, 16), (64, 16, 16), (64, 64, 64)]
    probs = _lockstep_contexts(sizes, dtype)
    rhs, ref = [], []
    for k, (g, ctx, vs) in enumerate(probs):
        ctx.set_velocity(torch.from_numpy((0.4 + 0.1 * k) * vs).to(dtype).cuda())
        r = torch.from_numpy(smooth_vector(g, 200 + k)).to(dtype).cuda()
        if k == 3:
            r.zero_()
        rhs.append(r)
    rtols = [0.3, 0.1, 0.03, 1e-3, 1e-2, 1e-2]
    for (g, ctx, vs), r, rt in zip(probs, rhs, rtols):
        ref.append(ctx.pcg(r, rtol=rt, maxit=40, with_status=True))
    B = mireg.Batch([p[1] for p in probs])
    xs, its, rels, sts = B.pcg(rhs, rtol=rtols, maxit=40)
    print("lockstep pcg", dtype, "iterations", its, "single", [r[1] for r in ref], flush=True)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for x, it, rel, st, (xr, itr, relr, str_) in zip(xs, its, rels, sts, ref):
        assert (it, st) == (itr, str_)
        assert abs(rel - relr) <= tol * max(relr, 1e-30) or rel == relr
        d = (x - xr).abs().max().item()
        scale = xr.abs().max().item()
        print("  iterate max diff %.2e of max %.2e" % (d, scale), flush=True)
        assert d <= tol * max(scale, 1e-30) * (1 if dtype == torch.float64 else 50)
    assert len(set(its)) > 2  # the problems stop at different iterations
    B.close()
    for p in probs:
        p[1].close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_lockstep_gn_matches_single_problem_gn(dtype):
    """Lockstep GN-Krylov over pairs of uneven sizes (power-of-two and
    radix-3 grids) against each pair's single-problem solve: in FP64 every
    counter identical and J, mismatch and gradient norms to 1e-10 (the FP64
    lockstep iterates equal the single ones bit for bit); in FP32, where a
    few ulps of difference in the Krylov passes steer the iterates of a
    solve stopped at a 20-fold gradient reduction, the same status,
    iterations within one, the same J0, and J and the relative mismatch
    within 1e-2 (measured: 7e-4 and 2e-3 on the 64^3 pair)."""
    need_gpu()
    sizes = [32, 48, 64, 32, 16]
    pairs = batch.make_pairs(sizes)
    if dtype == torch.float64:
        pairs = [(a.double(), b.double()) for a, b in pairs]
    ctxs = [mireg.Context((n, n, n), dtype=dtype, **batch.SOLVER) for n in sizes]
    singles = []
    for ctx, (mT, mR) in zip(ctxs, pairs):
        ctx.set_images(mT, mR)
        singles.append(ctx.gn_solve(grad_rtol=5e-2))
    B = mireg.Batch(ctxs)
    vs, reps = B.gn_solve(grad_rtol=5e-2)
    print("lockstep gn", dtype, [(r["gn_iters"], r["matvecs"], r["J"]) for r in reps], flush=True)
    print("single gn", dtype, [(r["gn_iters"], r["matvecs"], r["J"]) for _, r in singles], flush=True)
    for v, rep, (vr, rr) in zip(vs, reps, singles):
        assert rep["status"] == rr["status"] == mireg.CONVERGED_REL
        if dtype == torch.float64:
            for k in ("gn_iters", "matvecs", "pde_solves", "pcg_iters", "ls_trials", "neg_curv"):
                assert rep[k] == rr[k], k
            for k in ("J0", "J", "mismatch_rel", "gnorm0", "gnorm"):
                assert abs(rep[k] - rr[k]) <= 1e-10 * abs(rr[k]), k
        else:
            assert abs(rep["gn_iters"] - rr["gn_iters"]) <= 1
            assert rep["J0"] == rr["J0"]
            for k in ("J", "mismatch_rel"):
                assert abs(rep[k] - rr[k]) <= 1e-2 * abs(rr[k]), k
    B.close()
    for c in ctxs:
        c.close()


@pytest.mark.timeout(900)
def test_lockstep_gn_matches_oracle_on_batch_pairs():
    """Two pairs of the uneven batch recipe, the first 64^3 and the first
    96^3 one, prepared by the oracle on the host in FP64 (its own reference
    images) and solved together by the lockstep GN in FP64: status,
    iterations, matvecs, PDE solves and trials equal the oracle's solves,
    J, mismatch and gradient norms agree to 1e-10."""
    need_gpu()
    import math

    from oracle import solver

    amp = np.random.default_rng(7).uniform(0.05, 0.2, len(batch.UNEVEN_BATCH)) * 2 * math.pi
    picks = [batch.UNEVEN_BATCH.index(64), batch.UNEVEN_BATCH.index(96)]
    ctxs, oracle_reps = [], []
    for p in picks:
        n = (batch.UNEVEN_BATCH[p],) * 3
        g = core.Grid(n)
        mT = prep.smooth_rescale(g, synth.voronoi_phantom(n, nseeds=120, seed=100 + 2 * p), 2.0)
        v = prep.smooth_velocity(g, synth.white_noise(n, seed=101 + 2 * p), math.pi / 4, float(amp[p]))
        mR = prep.transport(g, mT, v)
        print("oracle solve", n, flush=True)
        prm = core.Params(n, nt=4, order=3, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=5e-3, beta_w=1.0)
        _, rep = solver.gn_solve(core.Registration(prm, mT, mR), np.zeros((3,) + n), grad_rtol=5e-2)
        oracle_reps.append(rep)
        ctx = mireg.Context(n, dtype=torch.float64, **batch.SOLVER)
        ctx.set_images(torch.from_numpy(mT).cuda(), torch.from_numpy(mR).cuda())
        ctxs.append(ctx)
    B = mireg.Batch(ctxs)
    _, reps = B.gn_solve(grad_rtol=5e-2)
    for rep, ro in zip(reps, oracle_reps):
        print("lockstep", {k: rep[k] for k in REPORT_KEYS}, "oracle", ro.as_dict(), flush=True)
        for k in ("status", "gn_iters", "matvecs", "pde_solves", "ls_trials", "neg_curv"):
            assert rep[k] == getattr(ro, k), k
        for k in ("J0", "J", "mismatch_rel", "gnorm0", "gnorm"):
            assert abs(rep[k] - getattr(ro, k)) <= 1e-10 * abs(getattr(ro, k)), k
    B.close()
    for c in ctxs:
        c.close()


def test_batch_rejects_mismatched_contexts():
    need_gpu()
    a = mireg.Context((16, 16, 16), dtype=torch.float32)
    b = mireg.Context((16, 16, 16), dtype=torch.float64)
    c = mireg.Context((16, 16, 16), dtype=torch.float32, nt=2)
    for bad in ([a, b], [a, c], [a, a]):
        with pytest.raises(mireg.MiregError):
            mireg.Batch(bad)
    B = mireg.Batch([a])
    with pytest.raises(mireg.MiregError):  # no images
        B.gn_solve()
    B.close()
    for x in (a, b, c):
        x.close()
