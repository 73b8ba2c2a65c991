"""Two-level coarse-grid preconditioner (Sec. 2.3.3) on the GPU against the
oracle (oracle/twolevel.py): the preconditioner itself, its reduction to the
spectral preconditioner without data term, PCG and the GN-Krylov solve (FP64,
same iteration path), and an FP32 solve that needs fewer fine matvecs than
with the spectral preconditioner."""
import numpy as np
import pytest
import torch

from oracle import core, prep, solver, twolevel
from paper_1808_04487_amd import mireg, synth

from gpu_util import as_input, need_gpu, rel_err, rel_err_l2, smooth_vector

pytestmark = pytest.mark.gpu


def problem(n, dtype, const_template=False):
    g = core.Grid(n)
    mT = np.full(n, 0.3) if const_template else synth.trig_template(n)
    vs = synth.trig_velocity(n)
    mT_t, mT = as_input(mT, dtype)
    mR_t, mR = as_input(prep.transport(g, synth.trig_template(n), vs), dtype)
    ctx = mireg.Context(n, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=1e-2, beta_w=1.0, dtype=dtype)
    ctx.set_images(mT_t, mR_t)
    ctx.set_precond("two_level", kappa=0.1, max_inner=50)
    p = core.Params(n, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=1e-2, beta_w=1.0)
    return g, ctx, core.Registration(p, mT, mR), vs


@pytest.mark.parametrize("n", [(32, 32, 32), (32, 16, 64)])
def test_two_level_apply_matches_oracle(n):
    need_gpu()
    dt = torch.float64
    g, ctx, R, vs = problem(n, dt)
    v_t, v = as_input(0.7 * vs + smooth_vector(g, 81, amp=0.1), dt)
    ctx.set_velocity(v_t)
    R.set_velocity(v)
    r_t, r = as_input(smooth_vector(g, 82) + 0.1 * np.random.default_rng(83).standard_normal((3,) + n), dt)
    z = ctx.precond(r_t)
    T = twolevel.TwoLevel(R, kappa=0.1, max_inner=50)
    zo = T.apply(r, 1.0)
    e = rel_err(z, zo)
    print("two-level apply", n, "coarse matvecs", T.coarse_matvecs, "err %.2e" % e, flush=True)
    assert e < 1e-11


def test_reduces_to_spectral_without_data_term():
    need_gpu()
    n = (32, 32, 32)
    g, ctx, _, vs = problem(n, torch.float64, const_template=True)
    ctx.set_velocity(torch.from_numpy(0.5 * vs).cuda())
    r = np.random.default_rng(84).standard_normal((3,) + n)
    r -= r.mean(axis=(1, 2, 3), keepdims=True)
    r_t = torch.from_numpy(r).cuda()
    z = ctx.precond(r_t)
    zs = ctx.op("precond", r_t)
    assert rel_err(z, zs.cpu().numpy()) < 1e-12


def test_pcg_and_gn_solve_match_oracle():
    need_gpu()
    n = (32, 32, 32)
    dt = torch.float64
    g, ctx, R, vs = problem(n, dt)
    v_t, v = as_input(0.6 * vs, dt)
    ctx.set_velocity(v_t)
    R.set_velocity(v)
    rhs = -R.gradient()
    x, its, rel = ctx.pcg(torch.from_numpy(rhs).cuda(), rtol=1e-3, maxit=100)
    T = twolevel.TwoLevel(R, kappa=0.1)
    xo, itso, relo = solver.pcg(R.hessian_matvec, lambda r: T.apply(r, 1e-3), rhs, 1e-3, 100, R.g.inner)
    print("PCG two-level GPU %d its rel %.3e, oracle %d its rel %.3e" % (its, rel, itso, relo), flush=True)
    assert its == itso and abs(rel - relo) < 1e-9
    assert rel_err(x, xo) < 1e-10
    # GN-Krylov solve from zero with the two-level preconditioner
    ctx.set_velocity(torch.zeros((3,) + n, dtype=dt, device="cuda"))
    vg, rep = ctx.gn_solve(grad_rtol=1e-2)
    T2 = twolevel.TwoLevel(R, kappa=0.1)
    vo, ro = solver.gn_solve(R, np.zeros((3,) + n), grad_rtol=1e-2, precond=T2)
    print("GN GPU", rep, "\nGN oracle", ro.as_dict(), flush=True)
    for k in ("status", "gn_iters", "matvecs", "pcg_iters", "ls_trials", "coarse_matvecs"):
        assert rep[k] == getattr(ro, k), k
    assert abs(rep["mismatch_rel"] - ro.mismatch_rel) < 1e-10
    assert rel_err(vg, vo) < 1e-9


def test_fp32_two_level_solve_needs_fewer_fine_matvecs():
    """The paper's synthetic problem at 128^3 in FP32: the two-level solve
    converges to the same tolerance with fewer fine-grid matvecs."""
    need_gpu()
    n = (128, 128, 128)
    _, ctx, _, _ = problem(n, torch.float32)
    ctx.set_precond("spectral")
    _, rs = ctx.gn_solve(grad_rtol=1e-2)
    ctx.set_precond("two_level", kappa=0.1)
    _, rt = ctx.gn_solve(grad_rtol=1e-2)
    print("spectral", rs, "\ntwo-level", rt, flush=True)
    assert rs["status"] == rt["status"] == mireg.CONVERGED_REL
    assert rt["matvecs"] < rs["matvecs"] and rt["coarse_matvecs"] > 0
    assert abs(rt["mismatch_rel"] - rs["mismatch_rel"]) < 0.05 * rs["mismatch_rel"]


def test_two_level_graph_replays_match_eager():
    """PCG with the two-level preconditioner, its fine and nested coarse
    matvecs replayed from captured graphs, equals the eager PCG bit for bit,
    over two velocities and repeated solves."""
    need_gpu()
    n = (32, 32, 32)
    dt = torch.float32
    g, ctx, R, vs = problem(n, dt)
    rhs = torch.from_numpy(smooth_vector(g, 84)).float().cuda()
    for scale in (0.5, 0.8):
        ctx.set_velocity(torch.from_numpy(scale * vs).float().cuda())
        ctx.set_graphs(False)
        x0, it0, _ = ctx.pcg(rhs, rtol=1e-4, maxit=30)
        ctx.set_graphs(True)
        x1, it1, _ = ctx.pcg(rhs, rtol=1e-4, maxit=30)
        torch.cuda.synchronize()
        x2, it2, _ = ctx.pcg(rhs, rtol=1e-4, maxit=30)
        print("two-level graphs: scale", scale, "iterations", it0, it1, it2, flush=True)
        assert it0 == it1 == it2 >= 2
        assert torch.equal(x0, x1) and torch.equal(x0, x2)
    ctx.set_graphs(False)
