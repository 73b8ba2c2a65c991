"""Oracle core (TEST INFRASTRUCTURE ONLY): FP64 reference of the reduced-space
Gauss-Newton-Krylov gradient and Hessian matvec for a stationary velocity.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark use
this module.  Everything is computed the plain way, in the order the paper
gives it (arXiv 1808.04487):

* Problem (Sec. 2.1, eq. "varopt"): minimise
  1/2 ||m(1) - mR||^2 + beta_v/2 <B v, B v> [+ beta_w/2 (||grad w||^2 + ||w||^2)]
  subject to dm/dt + grad m . v = 0, m(0) = mT, div v = w.
* Adjoint (eq. "adj"): -dl/dt - div(l v) = 0, l(1) = mR - m(1).
* Reduced gradient (eq. "reduced-gradient"): g = beta_v A v + K[int_0^1 l grad m dt].
* Incremental state (eq. "inc-state") and incremental adjoint (eq. "inc-adj")
  in their Gauss-Newton form (Sec. 2.3.2: every term with l is dropped), and
  the Hessian matvec (eq. "hessian-matvec"):
  H vt = beta_v A vt + K[int_0^1 lt grad m dt].
* Discretisation (Sec. 2.3.1): periodic grid on (0, 2 pi)^3, pseudospectral
  derivatives (FFT, weights, inverse FFT), trapezoidal rule in space and
  time, nt + 1 nodal time slices, explicit RK2 semi-Lagrangian transport
  with cubic (or linear) Lagrange interpolation.

Readings where the paper is silent (kept identical on every implementation):

* Nyquist: odd derivative symbols (d/dx_i, grad, div, and the wavenumbers
  inside K) use kt_i = k_i with kt_i = 0 at the Nyquist index; even symbols
  (A, Gaussian) keep the Nyquist mode.
* K for the near-incompressible model is built from the odd symbols:
  K = I - c(k) kt kt^T / |kt|^2, c = beta_w(|kt|^2+1)/(beta_v + beta_w(|kt|^2+1)),
  K = I at kt = 0 (Leray: c = 1; no constraint: K = I).
* Characteristics: Heun's method.  X = x - dt/2 (v(x) + v(x - dt v(x))),
  Y = x + dt/2 (v(x) + v(x + dt v(x))), with v at the predictor interpolated
  with the same polynomial order as every other off-grid value.
* Adjoint step: l^j = L + dt/2 (S + (L + dt S) d) with L = I[l^{j+1}](Y),
  S = I[l^{j+1} d](Y), d = div v (explicit Heun for the source l div v).
* Incremental state step: mt^{j+1} = I[mt^j + dt/2 f^j](X) + dt/2 f^{j+1},
  f^j = -grad m^j . vt (trapezoidal rule along the characteristic).
* Time integrals use the trapezoidal weights a_0 = a_nt = dt/2, a_j = dt.
* Preconditioner: (beta_v A)^{-1} with the zero singular value (k = 0) set
  to one (Sec. 2.3.3, remark on H_reg).
"""
import ctypes
import os

import numpy as np
import scipy.fft as sfft

from . import build as _build

DIV_NONE, DIV_NEAR, DIV_LERAY = 0, 1, 2
REG_H1, REG_H2 = 1, 2

WORKERS = int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1)

_lib = None


def _clib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
            os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)
        ):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_interp_field.argtypes = [dp, ip, dp, ctypes.c_int, dp]
        lib.orc_interp_field.restype = None
        lib.orc_interp_points.argtypes = [dp, ip, dp, ctypes.c_long, ctypes.c_int, dp]
        lib.orc_interp_points.restype = None
        lib.orc_interp_point.argtypes = [dp, ip, dp, ctypes.c_int]
        lib.orc_interp_point.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Grid:
    """Regular periodic grid on (0, 2 pi)^3 (Sec. 2.3.1).

    Grid point index i_a in [0, n_a) sits at x_a = i_a h_a, h_a = 2 pi / n_a
    (the same points as the paper's -n_a/2+1 <= k_a <= n_a/2, modulo 2 pi).
    Arrays are C-ordered [n1][n2][n3] with x3 fastest; vector fields carry a
    leading component axis of length 3.
    """

    def __init__(self, n):
        self.n = tuple(int(x) for x in n)
        if len(self.n) != 3 or any(x < 2 or x % 2 for x in self.n):
            raise ValueError("grid sizes must be three even integers")
        self.h = tuple(2.0 * np.pi / x for x in self.n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.cell = self.h[0] * self.h[1] * self.h[2]  # trapezoidal weight
        # integer wavenumbers in FFT order (index n/2 is the Nyquist mode)
        k = [np.fft.fftfreq(x, 1.0 / x) for x in self.n]
        kt = []
        for a, x in enumerate(self.n):
            ka = k[a].copy()
            ka[x // 2] = 0.0  # odd symbols vanish at the Nyquist index
            kt.append(ka)
        shp = [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]
        self.k = [k[a].reshape(shp[a]) for a in range(3)]
        self.kt = [kt[a].reshape(shp[a]) for a in range(3)]
        self.ksq = self.k[0] ** 2 + self.k[1] ** 2 + self.k[2] ** 2
        self.ktsq = self.kt[0] ** 2 + self.kt[1] ** 2 + self.kt[2] ** 2

    def coords(self):
        """Physical coordinates x_a = i_a h_a, each broadcastable to the grid."""
        shp = [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]
        return [(np.arange(self.n[a]) * self.h[a]).reshape(shp[a]) for a in range(3)]

    def inner(self, a, b):
        """Trapezoidal L2 inner product h1 h2 h3 sum(a b) (Sec. 2.3.1)."""
        return float(self.cell * np.sum(a * b))

    def norm(self, a):
        return float(np.sqrt(self.inner(a, a)))


# ---------------------------------------------------------------------------
# Pseudospectral operators (Sec. 2.3.1: FFT, weights, inverse FFT)
# ---------------------------------------------------------------------------

def fft(u):
    return sfft.fftn(u, workers=WORKERS)


def ifft_real(U):
    return sfft.ifftn(U, workers=WORKERS).real


def grad(g, u):
    """grad u: symbol i kt_a per component."""
    U = fft(u)
    return np.stack([ifft_real(1j * g.kt[a] * U) for a in range(3)])


def div(g, v):
    """div v: symbol sum_a i kt_a."""
    S = 0
    for a in range(3):
        S = S + 1j * g.kt[a] * fft(v[a])
    return ifft_real(S)


def reg_symbol(g, reg):
    """Symbol of A = B*B: H1 seminorm B = grad gives A = -Lap (|k|^2);
    H2 seminorm B = -Lap gives A = Lap^2 (|k|^4) (Sec. 2.1, 2.2)."""
    if reg == REG_H1:
        return g.ksq
    if reg == REG_H2:
        return g.ksq ** 2
    raise ValueError("reg must be 1 (H1) or 2 (H2)")


def apply_A(g, v, reg):
    a = reg_symbol(g, reg)
    return np.stack([ifft_real(a * fft(v[c])) for c in range(3)])


def laplacian(g, u):
    """Lap u with the even symbol -|k|^2."""
    return ifft_real(-g.ksq * fft(u))


def k_weight(g, div_mode, beta_v, beta_w):
    """Longitudinal weight c(k) of the projection K (Sec. 2.2):
    K = I - grad (beta_v (beta_w(-Lap + I))^{-1} + I)^{-1} Lap^{-1} div,
    which per mode is I - c(k) kt kt^T/|kt|^2 with
    c = beta_w(|kt|^2+1)/(beta_v + beta_w(|kt|^2+1)); Leray has c = 1."""
    if div_mode == DIV_NONE:
        return np.zeros_like(g.ktsq)
    if div_mode == DIV_LERAY:
        return np.ones_like(g.ktsq)
    if div_mode == DIV_NEAR:
        t = beta_w * (g.ktsq + 1.0)
        return t / (beta_v + t)
    raise ValueError("unknown divergence model")


def apply_K(g, v, div_mode, beta_v=0.0, beta_w=0.0):
    """K v (Sec. 2.2): identity without constraint, Leray projection for the
    incompressible model, near-incompressible projection with beta_w."""
    if div_mode == DIV_NONE:
        return np.array(v, dtype=np.float64, copy=True)
    V = [fft(v[a]) for a in range(3)]
    c = k_weight(g, div_mode, beta_v, beta_w)
    safe = np.where(g.ktsq > 0, g.ktsq, 1.0)
    proj = c * (g.kt[0] * V[0] + g.kt[1] * V[1] + g.kt[2] * V[2]) / safe
    return np.stack([ifft_real(V[a] - g.kt[a] * proj) for a in range(3)])


def apply_Hreg_inverse(g, r, reg, beta_v):
    """Spectral preconditioner M^{-1} = (beta_v A)^{-1} with the zero singular
    value of the regularisation operator set to one (Sec. 2.3.3, remark)."""
    s = beta_v * reg_symbol(g, reg)
    s = np.where(g.ksq == 0, 1.0, s)
    return np.stack([ifft_real(fft(r[c]) / s) for c in range(3)])


def gauss_smooth(g, u, sigma_vox):
    """Spectral Gaussian smoothing (Sec. 2.3.1) with standard deviation
    sigma_vox grid cells per axis: symbol exp(-1/2 sum_a (sigma_vox h_a k_a)^2)."""
    G = np.exp(-0.5 * sum((sigma_vox * g.h[a] * g.k[a]) ** 2 for a in range(3)))
    return ifft_real(G * fft(u))


# ---------------------------------------------------------------------------
# Off-grid interpolation (Sec. 2.3.1, Sec. 3.4): C library, see interp.c
# ---------------------------------------------------------------------------

def interp(g, f, disp, order):
    """I[f](x + disp(x)) at every grid point; disp in cell units [3][n...]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    disp = np.ascontiguousarray(disp, dtype=np.float64)
    if f.shape != g.n or disp.shape != (3,) + g.n:
        raise ValueError("shape mismatch in interp")
    out = np.empty(g.n, dtype=np.float64)
    n = (ctypes.c_int * 3)(*g.n)
    _clib().orc_interp_field(_dptr(f), n, _dptr(disp), int(order), _dptr(out))
    return out


def interp_points(g, f, xi, order):
    """I[f] at arbitrary cell-unit positions xi of shape [M][3]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
    out = np.empty(xi.shape[0], dtype=np.float64)
    n = (ctypes.c_int * 3)(*g.n)
    _clib().orc_interp_points(_dptr(f), n, _dptr(xi), xi.shape[0], int(order), _dptr(out))
    return out


# ---------------------------------------------------------------------------
# Semi-Lagrangian transport (Sec. 2.3.1)
# ---------------------------------------------------------------------------

def time_weights(nt):
    """Trapezoidal weights of the nodal time grid t_j = j/nt."""
    a = np.full(nt + 1, 1.0 / nt)
    a[0] = a[-1] = 0.5 / nt
    return a


def departure_points(g, v, nt, order, sign):
    """Characteristic feet over one step dt = 1/nt by Heun's method (RK2).

    sign = -1: X, foot of dx/dt = v traced back (state and incremental state);
    sign = +1: Y, foot for the adjoint equations, which run backward in time
    along -v.  Returned as displacements in cell units, [3][n...].
    """
    dt = 1.0 / nt
    pred = np.stack([sign * dt * v[a] / g.h[a] for a in range(3)])
    vp = np.stack([interp(g, v[a], pred, order) for a in range(3)])
    return np.stack([sign * 0.5 * dt * (v[a] + vp[a]) / g.h[a] for a in range(3)])


def solve_state(g, mT, X, nt, order):
    """State equation (eq. "varopt" constraint) forward in time:
    m^0 = mT, m^{j+1}(x) = m^j(X(x)).  Returns [m^0, ..., m^nt]."""
    m = [np.array(mT, dtype=np.float64, copy=True)]
    for j in range(nt):
        m.append(interp(g, m[j], X, order))
    return m


def adjoint_step(g, lam_next, Y, d, nt, order):
    """One backward step of -dl/dt - div(l v) = 0 (eq. "adj"): along the
    characteristic the adjoint obeys dl/dtau = l div v; the source is
    integrated with explicit Heun."""
    dt = 1.0 / nt
    L = interp(g, lam_next, Y, order)
    S = interp(g, lam_next * d, Y, order)
    return L + 0.5 * dt * (S + (L + dt * S) * d)


class Params:
    """Problem parameters (Sec. 2.1-2.3, Table "claire-parameters")."""

    def __init__(self, n, nt=4, order=3, reg=REG_H1, div_mode=DIV_NONE, beta_v=1e-2, beta_w=0.0):
        self.n = tuple(n)
        self.nt = int(nt)
        self.order = int(order)
        self.reg = int(reg)
        self.div = int(div_mode)
        self.beta_v = float(beta_v)
        self.beta_w = float(beta_w)


class Registration:
    """Reduced-space operators at the current velocity v (Sec. 2.2).

    Caches what depends on v only (departure points, state history, state
    gradients, div v, adjoint) until the next set_velocity.
    """

    def __init__(self, params, mT, mR):
        self.p = params
        self.g = Grid(params.n)
        self.mT = np.array(mT, dtype=np.float64, copy=True)
        self.mR = np.array(mR, dtype=np.float64, copy=True)
        self.a = time_weights(params.nt)
        self.set_velocity(np.zeros((3,) + self.g.n))

    # -- velocity-dependent quantities --------------------------------------
    def set_velocity(self, v):
        self.v = np.array(v, dtype=np.float64, copy=True)
        self._X = self._Y = self._m = self._gradm = self._d = None

    @property
    def X(self):
        if self._X is None:
            self._X = departure_points(self.g, self.v, self.p.nt, self.p.order, -1)
        return self._X

    @property
    def Y(self):
        if self._Y is None:
            self._Y = departure_points(self.g, self.v, self.p.nt, self.p.order, +1)
        return self._Y

    @property
    def m(self):
        if self._m is None:
            self._m = solve_state(self.g, self.mT, self.X, self.p.nt, self.p.order)
        return self._m

    @property
    def gradm(self):
        if self._gradm is None:
            self._gradm = [grad(self.g, mj) for mj in self.m]
        return self._gradm

    @property
    def d(self):
        if self._d is None:
            self._d = div(self.g, self.v)
        return self._d

    # -- objective (eq. "varopt:objective") ---------------------------------
    def objective(self):
        """Returns (J, mismatch term, regularisation term).  For the
        near-incompressible model w = div v is eliminated, which leaves the
        penalty beta_w/2 (||grad div v||^2 + ||div v||^2)."""
        g, p = self.g, self.p
        r = self.m[-1] - self.mR
        mism = 0.5 * g.inner(r, r)
        reg = 0.5 * p.beta_v * g.inner(apply_A(g, self.v, p.reg), self.v)
        if p.div == DIV_NEAR:
            w = self.d
            gw = grad(g, w)
            reg += 0.5 * p.beta_w * (g.inner(gw, gw) + g.inner(w, w))
        return mism + reg, mism, reg

    def mismatch_rel(self):
        """||m(1) - mR||^2 / ||mT - mR||^2."""
        r1 = self.m[-1] - self.mR
        r0 = self.mT - self.mR
        return float(np.sum(r1 * r1) / np.sum(r0 * r0))

    # -- adjoint and reduced gradient (eqs. "adj", "reduced-gradient") ------
    def adjoint(self):
        """Adjoint history [l^0, ..., l^nt] with l^nt = mR - m^nt."""
        nt = self.p.nt
        lam = [None] * (nt + 1)
        lam[nt] = self.mR - self.m[nt]
        for j in range(nt - 1, -1, -1):
            lam[j] = adjoint_step(self.g, lam[j + 1], self.Y, self.d, nt, self.p.order)
        return lam

    def gradient(self):
        """g = beta_v A v + K[ int_0^1 l grad m dt ] (trapezoidal in time)."""
        g, p = self.g, self.p
        lam = self.adjoint()
        b = np.zeros((3,) + g.n)
        for j in range(p.nt + 1):
            b += self.a[j] * lam[j] * self.gradm[j]
        return p.beta_v * apply_A(g, self.v, p.reg) + apply_K(g, b, p.div, p.beta_v, p.beta_w)

    # -- Gauss-Newton Hessian matvec (eqs. "inc-state", "inc-adj", "hessian-matvec")
    def incremental_state(self, vt):
        """mt(1) from dmt/dt + grad mt . v + grad m . vt = 0, mt(0) = 0."""
        nt, dt = self.p.nt, 1.0 / self.p.nt
        f = [-np.sum(self.gradm[j] * vt, axis=0) for j in range(nt + 1)]
        mt = np.zeros(self.g.n)
        for j in range(nt):
            mt = interp(self.g, mt + 0.5 * dt * f[j], self.X, self.p.order) + 0.5 * dt * f[j + 1]
        return mt

    def hessian_matvec(self, vt):
        """H vt = beta_v A vt + K[ int_0^1 lt grad m dt ] with the GN incremental
        adjoint -dlt/dt - div(lt v) = 0, lt(1) = -mt(1)."""
        g, p = self.g, self.p
        vt = np.asarray(vt, dtype=np.float64)
        lt = -self.incremental_state(vt)
        b = self.a[p.nt] * lt * self.gradm[p.nt]
        for j in range(p.nt - 1, -1, -1):
            lt = adjoint_step(g, lt, self.Y, self.d, p.nt, p.order)
            b = b + self.a[j] * lt * self.gradm[j]
        return p.beta_v * apply_A(g, vt, p.reg) + apply_K(g, b, p.div, p.beta_v, p.beta_w)

    def precond(self, r):
        return apply_Hreg_inverse(self.g, r, self.p.reg, self.p.beta_v)
