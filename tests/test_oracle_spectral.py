"""Pins for the oracle's pseudospectral operators (Sec. 2.2, 2.3.1) against
closed forms: exact derivatives of trigonometric polynomials, the Helmholtz
decomposition, the Gaussian symbol and the preconditioner's inverse."""
import numpy as np
import pytest

from oracle import core

N = (16, 12, 20)


def trig_poly(g, rng, nterms=6):
    """Random trigonometric polynomial with |k_a| < n_a/2 and its analytic
    first and second derivatives."""
    x = g.coords()
    f = np.zeros(g.n)
    df = [np.zeros(g.n) for _ in range(3)]
    lap = np.zeros(g.n)
    for _ in range(nterms):
        k = [int(rng.integers(-(g.n[a] // 2) + 1, g.n[a] // 2)) for a in range(3)]
        amp, ph = rng.normal(), rng.uniform(0, 2 * np.pi)
        arg = k[0] * x[0] + k[1] * x[1] + k[2] * x[2] + ph
        f += amp * np.cos(arg)
        for a in range(3):
            df[a] += -amp * k[a] * np.sin(arg)
        lap += -amp * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2) * np.cos(arg)
    return f, df, lap


def test_grad_div_laplacian_exact_on_trig_polynomials():
    g = core.Grid(N)
    rng = np.random.default_rng(0)
    f, df, lap = trig_poly(g, rng)
    gf = core.grad(g, f)
    for a in range(3):
        assert np.abs(gf[a] - df[a]).max() < 1e-11
    # div of a vector of trig polynomials
    comps = [trig_poly(g, rng) for _ in range(3)]
    v = np.stack([c[0] for c in comps])
    dv = comps[0][1][0] + comps[1][1][1] + comps[2][1][2]
    assert np.abs(core.div(g, v) - dv).max() < 1e-11
    assert np.abs(core.laplacian(g, f) - lap).max() < 1e-10


def test_regularisation_symbols_h1_h2():
    g = core.Grid(N)
    rng = np.random.default_rng(1)
    comps = [trig_poly(g, rng) for _ in range(3)]
    v = np.stack([c[0] for c in comps])
    lap = np.stack([c[2] for c in comps])
    # H1: A = -Lap ; H2: A = Lap^2 = Lap(Lap)
    assert np.abs(core.apply_A(g, v, core.REG_H1) + lap).max() < 1e-9
    lap2 = np.stack([core.laplacian(g, lap[a]) for a in range(3)])
    ref = np.abs(lap2).max()
    assert np.abs(core.apply_A(g, v, core.REG_H2) - lap2).max() < 1e-12 * ref * 100


def test_nyquist_rule():
    """Odd symbols vanish on the Nyquist mode, even symbols keep it."""
    g = core.Grid((8, 8, 8))
    x = g.coords()
    u = np.cos(4 * x[0]) + 0 * x[1] + 0 * x[2]  # pure Nyquist mode along x1
    assert np.abs(core.grad(g, u)).max() < 1e-13
    assert np.abs(core.laplacian(g, u) + 16 * u).max() < 1e-12
    G = core.gauss_smooth(g, u, 1.0)
    assert np.allclose(G, np.exp(-0.5 * (g.h[0] * 4) ** 2) * u, atol=1e-13)


def helmholtz_fields(g):
    """u = grad phi + curl psi with analytic phi, psi (zero-mean, no Nyquist)."""
    x1, x2, x3 = g.coords()
    gphi = [np.cos(x1) * np.sin(2 * x2) * np.cos(x3) * 1.0,
            2 * np.sin(x1) * np.cos(2 * x2) * np.cos(x3),
            -np.sin(x1) * np.sin(2 * x2) * np.sin(x3)]  # phi = sin x1 sin 2x2 cos x3
    # psi = (cos 2x3 sin x2, sin x1 cos x3, cos x2 sin 3x1)
    # curl psi = (d2 psi3 - d3 psi2, d3 psi1 - d1 psi3, d1 psi2 - d2 psi1)
    curl = [-np.sin(x2) * np.sin(3 * x1) + np.sin(x1) * np.sin(x3),
            -2 * np.sin(2 * x3) * np.sin(x2) - 3 * np.cos(x2) * np.cos(3 * x1),
            np.cos(x1) * np.cos(x3) - np.cos(2 * x3) * np.cos(x2)]
    shape = g.n
    gphi = np.stack([np.broadcast_to(c, shape) for c in gphi])
    curl = np.stack([np.broadcast_to(c, shape) for c in curl])
    return gphi, curl


def test_leray_projection_invariants():
    g = core.Grid(N)
    gphi, curl = helmholtz_fields(g)
    # analytic: div curl psi = 0
    assert np.abs(core.div(g, curl)).max() < 1e-12
    P = core.apply_K(g, gphi + curl, core.DIV_LERAY)
    assert np.abs(P - curl).max() < 1e-12  # P(grad phi + curl psi) = curl psi
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3,) + g.n)
    Pu = core.apply_K(g, u, core.DIV_LERAY)
    assert np.abs(core.div(g, Pu)).max() < 1e-11  # div P u = 0, Nyquist included
    PPu = core.apply_K(g, Pu, core.DIV_LERAY)
    assert np.abs(PPu - Pu).max() < 1e-12  # P^2 = P
    # P is self-adjoint in the trapezoidal inner product
    w = rng.standard_normal((3,) + g.n)
    Pw = core.apply_K(g, w, core.DIV_LERAY)
    assert abs(g.inner(Pu, w) - g.inner(u, Pw)) < 1e-10 * g.norm(u) * g.norm(w)


def test_near_incompressible_projection():
    g = core.Grid(N)
    gphi, curl = helmholtz_fields(g)
    bv, bw = 1e-2, 1.0
    # divergence-free fields pass unchanged
    K = core.apply_K(g, curl, core.DIV_NEAR, bv, bw)
    assert np.abs(K - curl).max() < 1e-12
    # a single-mode gradient field is scaled by 1 - c(k) = bv / (bv + bw(|k|^2+1))
    x1, x2, x3 = g.coords()
    phi_grad = np.stack(np.broadcast_arrays(-np.sin(x1 + 2 * x2) + 0 * x3,
                                            -2 * np.sin(x1 + 2 * x2) + 0 * x3,
                                            0 * x1 + 0 * x2 + 0 * x3))
    K = core.apply_K(g, phi_grad, core.DIV_NEAR, bv, bw)
    scale = bv / (bv + bw * (5.0 + 1.0))
    assert np.abs(K - scale * phi_grad).max() < 1e-12
    # K tends to the Leray projection as beta_w grows
    rng = np.random.default_rng(4)
    u = rng.standard_normal((3,) + g.n)
    P = core.apply_K(g, u, core.DIV_LERAY)
    K = core.apply_K(g, u, core.DIV_NEAR, bv, 1e8)
    assert np.abs(K - P).max() < 1e-8
    assert np.array_equal(core.apply_K(g, u, core.DIV_NONE), u)


def test_preconditioner_inverts_regularisation():
    g = core.Grid(N)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3,) + g.n)
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    for reg in (core.REG_H1, core.REG_H2):
        Au = 0.3 * core.apply_A(g, u, reg)
        back = core.apply_Hreg_inverse(g, Au, reg, 0.3)
        assert np.abs(back - u).max() < 1e-10
    # the zero singular value is set to one: constants pass unchanged
    c = np.ones((3,) + g.n) * np.array([1.0, -2.0, 0.5]).reshape(3, 1, 1, 1)
    assert np.allclose(core.apply_Hreg_inverse(g, c, core.REG_H1, 0.3), c, atol=1e-13)


def test_gaussian_symbol_on_single_mode():
    g = core.Grid(N)
    x1, x2, x3 = g.coords()
    k = (2, -3, 5)
    u = np.cos(k[0] * x1 + k[1] * x2 + k[2] * x3 + 0.4)
    s = 1.7
    expect = np.exp(-0.5 * sum((s * g.h[a] * k[a]) ** 2 for a in range(3))) * u
    assert np.abs(core.gauss_smooth(g, u, s) - expect).max() < 1e-13


@pytest.mark.parametrize("n", [(4, 4, 4), (6, 4, 8)])
def test_spectral_derivative_matches_brute_force_dft(n):
    """The library FFT step against an O(N^2) DFT written out directly."""
    g = core.Grid(n)
    rng = np.random.default_rng(6)
    u = rng.standard_normal(n)
    idx = np.indices(n).reshape(3, -1)
    kk = [np.fft.fftfreq(n[a], 1.0 / n[a]) for a in range(3)]
    kidx = np.indices(n).reshape(3, -1)
    kv = [kk[a][kidx[a]] for a in range(3)]
    phase = sum(np.outer(kv[a], idx[a]) * (2 * np.pi / n[a]) for a in range(3))
    F = np.exp(-1j * phase)  # forward DFT matrix
    U = F @ u.ravel()
    for a in range(3):
        kt = kv[a].copy()
        kt[kidx[a] == n[a] // 2] = 0.0
        d = (np.conj(F).T @ (1j * kt * U)).real / u.size
        assert np.abs(d.reshape(n) - core.grad(g, u)[a]).max() < 1e-12
