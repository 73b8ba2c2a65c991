"""Pins for the two-level preconditioner oracle (oracle/twolevel.py, Sec.
2.3.3): spectral restriction and prolongation exact on band-limited fields
and adjoint to each other, F_L + F_H = I, the split factor squared equal to
the spectral preconditioner, reduction to the spectral preconditioner when
the data term vanishes, and PCG / GN solves that converge with fewer fine
Hessian matvecs than with the spectral preconditioner."""
import numpy as np
import pytest

from oracle import core, prep, solver, twolevel
from paper_1808_04487_amd import synth


def trig(shape, kmax, seed):
    """Random trigonometric polynomial with |k_a| <= kmax on every axis."""
    g = core.Grid(shape)
    x1, x2, x3 = g.coords()
    rng = np.random.default_rng(seed)
    u = np.zeros(shape)
    for _ in range(8):
        k = rng.integers(-kmax, kmax + 1, 3)
        ph = rng.uniform(0, 2 * np.pi)
        u += rng.standard_normal() * np.cos(k[0] * x1 + k[1] * x2 + k[2] * x3 + ph)
    return u


def test_resampling_is_exact_on_band_limited_fields():
    fine, coarse = (32, 16, 32), (16, 8, 16)
    u = trig(fine, 3, 1)                      # |k_a| <= 3 < 4 = n_coarse / 2 on every axis
    uc = twolevel.resample(u, coarse)
    assert np.abs(uc - trig(coarse, 3, 1)).max() < 1e-12
    assert np.abs(twolevel.resample(uc, fine) - u).max() < 1e-12


def test_restriction_is_the_adjoint_of_prolongation():
    fine, coarse = (32, 32, 16), (16, 16, 8)
    gf, gc = core.Grid(fine), core.Grid(coarse)
    rng = np.random.default_rng(2)
    u, w = rng.standard_normal((3,) + fine), rng.standard_normal((3,) + coarse)
    lhs = gc.inner(twolevel.resample(u, coarse), w)
    rhs = gf.inner(u, twolevel.resample(w, fine))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_low_and_high_parts_add_up():
    fine = (32, 32, 32)
    g = core.Grid(fine)
    u = np.random.default_rng(3).standard_normal(fine)
    low = twolevel.resample(twolevel.resample(u, (16, 16, 16)), fine)
    assert np.abs(low + twolevel.highpass(g, u) - u).max() < 1e-12
    # F_L is a projector onto |k_a| < 8
    assert np.abs(twolevel.highpass(g, low)).max() < 1e-12
    assert np.abs(twolevel.highpass(g, trig(fine, 7, 4))).max() < 1e-12


@pytest.mark.parametrize("reg", [core.REG_H1, core.REG_H2])
def test_split_factor_squares_to_the_spectral_preconditioner(reg):
    g = core.Grid((16, 16, 16))
    r = np.random.default_rng(5).standard_normal((3,) + g.n)
    z = twolevel.hreg_inv_sqrt(g, twolevel.hreg_inv_sqrt(g, r, reg, 3e-2), reg, 3e-2)
    assert np.abs(z - core.apply_Hreg_inverse(g, r, reg, 3e-2)).max() < 1e-12 * np.abs(z).max()


def test_reduces_to_the_spectral_preconditioner_without_data_term():
    """Constant template: H = beta_v A on both grids, so the coarse operator
    is the identity on zero-mean fields and M^{-1} = (beta_v A)^{-1}."""
    n = (32, 32, 32)
    g = core.Grid(n)
    p = core.Params(n, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=1e-2, beta_w=1.0)
    R = core.Registration(p, np.full(n, 0.3), synth.trig_template(n))
    R.set_velocity(0.5 * synth.trig_velocity(n))
    r = np.random.default_rng(6).standard_normal((3,) + n)
    r -= r.mean(axis=(1, 3, 2), keepdims=True)
    T = twolevel.TwoLevel(R, kappa=0.1)
    z = T.apply(r, 0.5)
    assert T.coarse_matvecs == 1
    zs = R.precond(r)
    assert np.abs(z - zs).max() < 1e-12 * np.abs(zs).max()


def synthetic(n):
    g = core.Grid(n)
    mT = synth.trig_template(n)
    vs = synth.trig_velocity(n)
    mR = prep.transport(g, mT, vs)
    p = core.Params(n, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=1e-2, beta_w=1.0)
    return core.Registration(p, mT, mR), vs


def test_pcg_with_two_level_reaches_the_true_residual():
    n = (16, 16, 16)
    R, vs = synthetic(n)
    R.set_velocity(0.7 * vs)
    rhs = -R.gradient()
    T = twolevel.TwoLevel(R, kappa=0.1)
    x, its, rel = solver.pcg(R.hessian_matvec, lambda r: T.apply(r, 1e-3), rhs, 1e-3, 100, R.g.inner)
    res = rhs - R.hessian_matvec(x)
    assert np.sqrt(R.g.inner(res, res)) <= 1.01e-3 * np.sqrt(R.g.inner(rhs, rhs))
    xs, its_s, _ = solver.pcg(R.hessian_matvec, R.precond, rhs, 1e-3, 100, R.g.inner)
    print("PCG iterations: spectral", its_s, "two-level", its, "coarse matvecs", T.coarse_matvecs)
    assert its < its_s


def test_gn_solve_with_two_level_needs_fewer_fine_matvecs():
    n = (32, 32, 32)
    R, _ = synthetic(n)
    v0 = np.zeros((3,) + n)
    _, rs = solver.gn_solve(R, v0, grad_rtol=1e-2)
    T = twolevel.TwoLevel(R, kappa=0.1)
    _, rt = solver.gn_solve(R, v0, grad_rtol=1e-2, precond=T)
    print("spectral", rs.as_dict(), "\ntwo-level", rt.as_dict())
    assert rs.status == rt.status == solver.CONVERGED_REL
    assert rt.matvecs < rs.matvecs and rt.coarse_matvecs > 0
    assert abs(rt.mismatch_rel - rs.mismatch_rel) < 0.05 * rs.mismatch_rel
