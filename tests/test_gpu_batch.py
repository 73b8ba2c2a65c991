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
