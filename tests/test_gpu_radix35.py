"""Grids of 48, 80, 96 and 160 points per axis (3 and 5 times a power of two;
radix-3 and radix-5 transform stages, general-n index arithmetic in the
transport kernels) against the oracle: every spectral operator on grids that
use each new line length in each pass, departure points, interpolation and
transport through both gather paths, objective, gradient, Hessian matvec and
PCG, the two-level preconditioner with a 48^3 coarse grid, and the sizes the
library refuses."""
import numpy as np
import pytest
import torch

from oracle import core, prep, solver, twolevel
from paper_1808_04487_amd import mireg, synth

from gpu_util import (as_input, assert_close, assert_close_composite, need_gpu, rel_err,
                      smooth_scalar, smooth_vector)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
# x3 lines n3/2 in {24, 40, 48, 80}, strided lines n1, n2 in {48, 80, 96, 160},
# mixed with powers of two
GRIDS = [(48, 48, 48), (96, 80, 160), (80, 160, 96), (160, 96, 48), (48, 96, 80), (64, 48, 32)]


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_spectral_operators_radix35(n, dtype):
    need_gpu()
    g = core.Grid(n)
    bv, bw = 3e-2, 0.5
    ctx = mireg.Context(n, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=bv, beta_w=bw, dtype=dtype)
    u_t, u = as_input(smooth_scalar(g, 1, sigma=1.0) + 0.3 * np.random.default_rng(2).standard_normal(n), dtype)
    v_t, v = as_input(smooth_vector(g, 3, sigma=1.0) + 0.3 * np.random.default_rng(4).standard_normal((3,) + n), dtype)
    print("spectral ops", n, dtype, flush=True)
    assert_close(ctx.op("grad", u_t), core.grad(g, u), dtype, what="grad")
    assert_close(ctx.op("div", v_t), core.div(g, v), dtype, what="div")
    assert_close(ctx.op("laplace", u_t), core.laplacian(g, u), dtype, what="laplace")
    assert_close(ctx.op("apply_A", v_t), core.apply_A(g, v, core.REG_H1), dtype, what="A (H1)")
    assert_close(ctx.op("apply_K", v_t), core.apply_K(g, v, core.DIV_NEAR, bv, bw), dtype, what="K")
    assert_close(ctx.op("leray", v_t), core.apply_K(g, v, core.DIV_LERAY), dtype, what="Leray")
    assert_close(ctx.op("precond", v_t), core.apply_Hreg_inverse(g, v, core.REG_H1, bv), dtype, what="M^-1")
    assert_close(ctx.op("gauss", u_t, 1.7), core.gauss_smooth(g, u, 1.7), dtype, what="Gaussian")
    ctx.close()


@pytest.mark.parametrize("n", [(48, 96, 80), (96, 48, 160)])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("order", [3, 1])
@pytest.mark.parametrize("staging", ["lds", "global"])
def test_transport_radix35(n, dtype, order, staging, monkeypatch):
    need_gpu()
    g = core.Grid(n)
    if staging == "global":
        monkeypatch.setenv("MIREG_LDS_STENCIL", "0")
    ctx = mireg.Context(n, order=order, dtype=dtype)
    v_t, v = as_input(smooth_vector(g, 5, amp=1.5, sigma=3.0), dtype)
    print("transport", n, dtype, order, staging, flush=True)
    Xo = core.departure_points(g, v, 4, order, -1)
    assert_close(ctx.op("departure_X", v_t), Xo, dtype, what="X")
    assert_close(ctx.op("departure_Y", v_t), core.departure_points(g, v, 4, order, +1), dtype, what="Y")
    f_t, f = as_input(smooth_scalar(g, 6), dtype)
    d_t, d = as_input(Xo, dtype)
    arg = torch.cat([f_t.reshape(1, -1), d_t.reshape(3, -1)]).contiguous()
    assert_close(ctx.op("interp", arg), core.interp(g, f, d, order), dtype, what="interp")
    ctx.set_velocity(v_t)
    m1 = ctx.op("transport_state", f_t)
    assert_close(m1, prep.transport(g, f, v, nt=4, order=order), dtype, factor=4, what="state m(1)")
    ctx.close()


def problem(n, reg, div, bv, bw, dtype):
    g = core.Grid(n)
    mT_t, mT = as_input(synth.trig_template(n), dtype)
    vs = synth.trig_velocity(n)
    mR_t, mR = as_input(prep.transport(g, mT, vs, nt=4, order=3), dtype)
    p = core.Params(n, nt=4, order=3, reg=reg, div_mode=div, beta_v=bv, beta_w=bw)
    R = core.Registration(p, mT, mR)
    ctx = mireg.Context(n, nt=4, order=3, reg=reg, div=div, beta_v=bv, beta_w=bw, dtype=dtype)
    ctx.set_images(mT_t, mR_t)
    return g, R, ctx, vs


@pytest.mark.parametrize("case", [((48, 48, 48), core.REG_H1, core.DIV_NEAR, 1e-2, 1.0),
                                  ((96, 48, 80), core.REG_H2, core.DIV_NONE, 1e-3, 0.0)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_objective_gradient_matvec_pcg_radix35(case, dtype):
    need_gpu()
    n, reg, div, bv, bw = case
    g, R, ctx, vs = problem(n, reg, div, bv, bw, dtype)
    print("reduced ops", n, reg, div, dtype, flush=True)
    v_t, v = as_input(0.6 * vs + smooth_vector(g, 11, amp=0.2), dtype)
    ctx.set_velocity(v_t)
    R.set_velocity(v)
    J, mis, rg = ctx.objective()
    Jo, miso, rgo = R.objective()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert abs(mis - miso) <= 10 * tol * abs(miso)
    assert abs(rg - rgo) <= 10 * tol * abs(rgo)
    gr, gn = ctx.gradient()
    go = R.gradient()
    assert_close_composite(gr, go, dtype, what="gradient")
    vt_t, vt = as_input(smooth_vector(g, 12, amp=1.0), dtype)
    Ho = R.hessian_matvec(vt)
    assert_close_composite(ctx.hessian_matvec(vt_t), Ho, dtype, what="matvec")
    rhs_t, rhs = as_input(-go, dtype)
    x, it, rel = ctx.pcg(rhs_t, rtol=1e-3, maxit=50)
    xo, ito, relo = solver.pcg(R.hessian_matvec, R.precond, rhs, 1e-3, 50, g.inner)
    print("pcg iterations", it, ito, flush=True)
    assert it == ito
    assert_close(x, xo, dtype, factor=50 if dtype == torch.float32 else 10, what="pcg x")
    ctx.close()


def test_two_level_with_48_coarse_grid():
    """96^3 has the 48^3 coarse problem; the preconditioner matches the
    oracle.  48^3 itself has no supported coarse grid (24^3)."""
    need_gpu()
    n = (96, 96, 96)
    dt = torch.float64
    g, R, ctx, vs = problem(n, core.REG_H1, core.DIV_NEAR, 1e-2, 1.0, dt)
    ctx.set_precond("two_level", kappa=0.1, max_inner=50)
    v_t, v = as_input(0.7 * vs, dt)
    ctx.set_velocity(v_t)
    R.set_velocity(v)
    r_t, r = as_input(smooth_vector(g, 82) + 0.1 * np.random.default_rng(83).standard_normal((3,) + n), dt)
    z = ctx.precond(r_t)
    zo = twolevel.TwoLevel(R, kappa=0.1, max_inner=50).apply(r, 1.0)
    e = rel_err(z, zo)
    print("two-level 96^3 err %.2e" % e, flush=True)
    assert e < 1e-11
    ctx.close()
    small = mireg.Context((48, 48, 48), dtype=dt)
    with pytest.raises(mireg.MiregError) as exc:
        small.set_precond("two_level")
    assert exc.value.code == mireg.E_SHAPE
    small.close()


@pytest.mark.parametrize("n", [(72, 64, 64), (64, 112, 64), (64, 64, 40), (24, 64, 64)])
def test_unsupported_sizes_are_refused(n):
    need_gpu()
    with pytest.raises(mireg.MiregError) as exc:
        mireg.Context(n, dtype=torch.float32)
    assert exc.value.code == mireg.E_SHAPE
