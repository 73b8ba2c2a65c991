"""Pins for the oracle's interpolation and semi-Lagrangian transport
(Sec. 2.3.1, Sec. 3.4) against closed forms, polynomial exactness,
convergence orders and conservation laws."""
import numpy as np
import pytest

from oracle import core, prep
from paper_1808_04487_amd import synth


def test_interpolation_exact_at_nodes_and_wraps():
    g = core.Grid((8, 6, 10))
    rng = np.random.default_rng(0)
    f = rng.standard_normal(g.n)
    shift = np.stack([np.full(g.n, s) for s in (3.0, -7.0, 12.0)])
    for order in (1, 3):
        out = core.interp(g, f, shift, order)
        assert np.array_equal(out, np.roll(f, (-3, 7, -12), axis=(0, 1, 2)))


@pytest.mark.parametrize("order,deg", [(3, 3), (1, 1)])
def test_interpolation_reproduces_tensor_polynomials(order, deg):
    """Lagrange interpolation of degree p reproduces every polynomial of
    degree <= p per axis inside a window that does not wrap."""
    g = core.Grid((16, 16, 16))
    rng = np.random.default_rng(1)
    i = np.arange(16.0)
    coef = rng.standard_normal((deg + 1, deg + 1, deg + 1))

    def poly(a, b, c):
        return sum(coef[p, q, r] * a ** p * b ** q * c ** r
                   for p in range(deg + 1) for q in range(deg + 1) for r in range(deg + 1))

    f = poly(i.reshape(-1, 1, 1), i.reshape(1, -1, 1), i.reshape(1, 1, -1))
    pts = rng.uniform(2.0, 12.0, size=(200, 3))  # stencils stay inside [1, 14]
    out = core.interp_points(g, f, pts, order)
    expect = poly(pts[:, 0], pts[:, 1], pts[:, 2])
    assert np.abs(out - expect).max() < 1e-9 * np.abs(expect).max()
    # one degree higher is not reproduced
    f2 = i.reshape(-1, 1, 1) ** (deg + 1) + 0 * i.reshape(1, -1, 1) + 0 * i.reshape(1, 1, -1)
    out2 = core.interp_points(g, f2, pts, order)
    assert np.abs(out2 - pts[:, 0] ** (deg + 1)).max() > 1e-3


@pytest.mark.parametrize("order,expect_order", [(3, 3.7), (1, 1.8)])
def test_interpolation_convergence_order(order, expect_order):
    rng = np.random.default_rng(2)
    errs = []
    for n in (16, 32, 64):
        g = core.Grid((n, n, n))
        x = g.coords()
        f = np.sin(x[0]) * np.cos(2 * x[1]) * np.sin(x[2] + 1.0)
        pts = rng.uniform(0, n, size=(4000, 3))
        out = core.interp_points(g, f, pts, order)
        P = pts * g.h[0]
        ex = np.sin(P[:, 0]) * np.cos(2 * P[:, 1]) * np.sin(P[:, 2] + 1.0)
        errs.append(np.abs(out - ex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > expect_order, (errs, rates)
    if order == 3:
        # textbook bound per axis: |f''''| max |(t+1)t(t-1)(t-2)|/24 h^4 = 9/16/24 h^4
        h = 2 * np.pi / 64
        bound = 3 * (4 ** 2 + 1 + 1) * (9.0 / 16.0) / 24.0 * h ** 4
        assert errs[-1] <= bound


@pytest.mark.parametrize("order", [1, 3])
def test_integer_shift_transport_is_a_roll(order):
    """Constant v = (h/dt) s with s integer: each step moves by s cells, so
    m(1) is mT rolled by nt*s."""
    n, nt = (12, 10, 14), 4
    g = core.Grid(n)
    s = (1, -2, 3)
    v = np.stack([np.full(n, s[a] * g.h[a] * nt) for a in range(3)])
    rng = np.random.default_rng(3)
    mT = rng.standard_normal(n)
    m1 = prep.transport(g, mT, v, nt=nt, order=order)
    expect = np.roll(mT, tuple(nt * s[a] for a in range(3)), axis=(0, 1, 2))
    assert np.abs(m1 - expect).max() < 1e-13


def test_constant_velocity_transport_order():
    """Constant non-integer v: exact solution mT(x - v), RK2 characteristics
    are exact, so all error is interpolation error (order about 4)."""
    c = np.array([0.37, -0.61, 0.23])
    errs = []
    for n in (16, 32, 64):
        g = core.Grid((n,) * 3)
        x = g.coords()
        v = np.stack([np.full(g.n, c[a]) for a in range(3)])
        mT = synth.trig_template(g.n)
        m1 = prep.transport(g, mT, v, nt=4)
        ex = (np.sin(x[0] - c[0]) ** 2 + np.sin(x[1] - c[1]) ** 2 + np.sin(x[2] - c[2]) ** 2) / 3
        errs.append(np.abs(m1 - ex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 3.5, (errs, rates)


def rk4_feet(g, vfun, steps=64):
    """Feet of the characteristics of dx/dt = v(x) over t in [0, 1], traced
    back from every grid point with classical RK4."""
    x = [np.broadcast_to(c, g.n).astype(np.float64) for c in g.coords()]
    dt = -1.0 / steps
    for _ in range(steps):
        k1 = vfun(*x)
        k2 = vfun(*[x[a] + 0.5 * dt * k1[a] for a in range(3)])
        k3 = vfun(*[x[a] + 0.5 * dt * k2[a] for a in range(3)])
        k4 = vfun(*[x[a] + dt * k3[a] for a in range(3)])
        x = [x[a] + dt / 6 * (k1[a] + 2 * k2[a] + 2 * k3[a] + k4[a]) for a in range(3)]
    return x


def test_variable_velocity_transport_against_rk4_characteristics():
    """The paper's synthetic velocity (scaled by 0.5): m(1, x) = mT(foot(x)).
    Error falls under refinement (space at nt = 16; time at 32^3)."""
    def vstar(a, b, c):
        return [0.5 * np.sin(c) * np.cos(b) * np.sin(b), 0.5 * np.sin(a) * np.cos(c) * np.sin(c),
                0.5 * np.sin(b) * np.cos(a) * np.sin(a)]

    def mfun(a, b, c):
        return (np.sin(a) ** 2 + np.sin(b) ** 2 + np.sin(c) ** 2) / 3

    errs = {}
    for n in (16, 32):
        g = core.Grid((n,) * 3)
        ex = mfun(*rk4_feet(g, vstar))
        v = synth.trig_velocity(g.n)
        mT = synth.trig_template(g.n)
        for nt in (4, 8, 16):
            errs[(n, nt)] = np.abs(prep.transport(g, mT, v, nt=nt) - ex).max()
    assert errs[(16, 16)] / errs[(32, 16)] > 6.0  # about order 3 in h
    assert errs[(32, 4)] < 1e-3
    assert errs[(32, 16)] < errs[(32, 4)]


def compressible_velocity(g, amp=0.3):
    """Pure gradient field v = amp grad(sin x1 + sin x2 + sin x3) (div v != 0)."""
    x1, x2, x3 = g.coords()
    return amp * np.stack(np.broadcast_arrays(np.cos(x1) + 0 * x2 + 0 * x3,
                                              np.cos(x2) + 0 * x1 + 0 * x3,
                                              np.cos(x3) + 0 * x1 + 0 * x2))


def test_adjoint_conserves_mass():
    """-dl/dt - div(l v) = 0 on a periodic domain conserves int l dx.  With a
    compressible v the drift of the discrete adjoint vanishes under
    refinement; pure transport (divergence source dropped) leaves an O(1)
    drift."""
    drift, plain = [], []
    for n in (16, 32):
        g = core.Grid((n,) * 3)
        v = compressible_velocity(g)
        x1, x2, x3 = g.coords()
        lam = np.exp(np.cos(x1 - 1) + np.cos(x2 + 0.5) + np.cos(x3) + 0 * x1)
        Y = core.departure_points(g, v, 4, 3, +1)
        d = core.div(g, v)
        l0, L = lam.copy(), lam.copy()
        for _ in range(4):
            lam = core.adjoint_step(g, lam, Y, d, 4, 3)
            L = core.interp(g, L, Y, 3)
        drift.append(abs(lam.sum() - l0.sum()) / l0.sum())
        plain.append(abs(L.sum() - l0.sum()) / l0.sum())
    assert drift[0] / drift[1] > 5.0
    assert drift[1] < 5e-4
    assert min(plain) > 2e-2


def test_departure_points_zero_velocity_and_sign():
    g = core.Grid((8, 8, 8))
    v0 = np.zeros((3,) + g.n)
    assert np.array_equal(core.departure_points(g, v0, 4, 3, -1), v0)
    c = np.array([0.3, -0.2, 0.1])
    v = np.stack([np.full(g.n, c[a]) for a in range(3)])
    X = core.departure_points(g, v, 4, 3, -1)
    Y = core.departure_points(g, v, 4, 3, +1)
    for a in range(3):
        assert np.allclose(X[a], -0.25 * c[a] / g.h[a], atol=1e-14)
        assert np.allclose(Y[a], 0.25 * c[a] / g.h[a], atol=1e-14)
