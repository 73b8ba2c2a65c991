"""Oracle of the two-level coarse-grid preconditioner (TEST INFRASTRUCTURE
ONLY), Sec. 2.3.3 of the paper.

The preconditioned system is the regularisation split form
Hreg^{-1/2} H Hreg^{-1/2} w = Hreg^{-1/2} s with Hreg = beta_v A (its zero
singular value set to one).  Its preconditioner P keeps the high-frequency
part (F_H) unchanged and solves the low-frequency part on a grid of half the
size: u_L = Q_P Sc^{-1} Q_R F_L t with Sc = Hreg_c^{-1/2} H_c Hreg_c^{-1/2} the
direct (non-Galerkin) coarse discretisation, H_c the Gauss-Newton Hessian of
the coarse problem (restricted images, restricted velocity), inverted by CG
to the relative tolerance kappa eps_H ("PCG(kappa)", kappa = 0.1).  In terms
of the original system this is the preconditioner
M^{-1} = Hreg^{-1/2} P^{-1} Hreg^{-1/2} of PCG for H x = s.

Restriction Q_R and prolongation Q_P are spectral: the trigonometric
interpolant truncated to the modes both grids resolve below their Nyquist
(|k_a| < n_a / 4 for a fine grid of n_a points), sampled on the other grid.
F_L keeps exactly those modes, F_H = I - F_L.
"""
import numpy as np

from . import core


def resample(u, shape_out):
    """Spectral resampling of the scalar or vector field u (leading component
    axis allowed) to the grid ``shape_out``."""
    u = np.asarray(u, dtype=np.float64)
    lead = u.shape[:-3]
    ns = u.shape[-3:]
    nd = tuple(shape_out)
    U = np.fft.fftn(u, axes=(-3, -2, -1))
    idx_s, idx_d = [], []
    for a in range(3):
        c = min(ns[a], nd[a]) // 2
        w = np.arange(-c + 1, c)
        idx_s.append(w % ns[a])
        idx_d.append(w % nd[a])
    out = np.zeros(lead + nd, dtype=complex)
    out[(Ellipsis,) + np.ix_(*idx_d)] = U[(Ellipsis,) + np.ix_(*idx_s)]
    out *= float(np.prod(nd)) / float(np.prod(ns))
    return np.real(np.fft.ifftn(out, axes=(-3, -2, -1)))


def highpass(g, u):
    """F_H: zero on the modes with |k_a| < n_a / 4 on every axis."""
    low = np.ones(g.ksq.shape, dtype=bool)
    for a in range(3):
        low &= 4 * np.abs(g.k[a]) < g.n[a]
    U = core.fft(u)
    return core.ifft_real(np.where(low, 0.0, U))


def hreg_inv_sqrt(g, u, reg, beta_v):
    """(beta_v A)^{-1/2} with the k = 0 value set to one."""
    a = beta_v * core.reg_symbol(g, reg)
    s = np.where(g.ksq == 0, 1.0, 1.0 / np.sqrt(np.where(g.ksq == 0, 1.0, a)))
    return core.ifft_real(core.fft(u) * s)


class TwoLevel:
    """Two-level preconditioner for the GN Hessian of ``reg`` (a
    core.Registration on a grid with at least 16 points per axis)."""

    def __init__(self, reg, kappa=0.1, max_inner=50):
        self.R = reg
        p = reg.p
        self.nc = tuple(n // 2 for n in p.n)
        pc = core.Params(self.nc, nt=p.nt, order=p.order, reg=p.reg, div_mode=p.div, beta_v=p.beta_v,
                         beta_w=p.beta_w)
        self.C = core.Registration(pc, resample(reg.mT, self.nc), resample(reg.mR, self.nc))
        self.kappa, self.max_inner = float(kappa), int(max_inner)
        self.coarse_matvecs = 0
        self._v = None

    def _coarse_at_current_velocity(self):
        if self._v is None or not np.array_equal(self._v, self.R.v):
            self._v = self.R.v.copy()
            self.C.set_velocity(resample(self.R.v, self.nc))

    def coarse_operator(self, u):
        C, p = self.C, self.C.p
        w = hreg_inv_sqrt(C.g, u, p.reg, p.beta_v)
        self.coarse_matvecs += 1
        return hreg_inv_sqrt(C.g, C.hessian_matvec(w), p.reg, p.beta_v)

    def coarse_cg(self, b, tol_rel):
        """CG on the coarse split operator from 0, stopping when
        ||r|| <= tol_rel ||b||, after max_inner iterations or on
        non-positive curvature."""
        inner = self.C.g.inner
        u = np.zeros_like(b)
        r = b.copy()
        p = b.copy()
        rr = inner(r, r)
        tol = tol_rel * np.sqrt(rr)
        it = 0
        while it < self.max_inner and np.sqrt(rr) > tol:
            q = self.coarse_operator(p)
            pq = inner(p, q)
            if not pq > 0:
                break
            alpha = rr / pq
            u = u + alpha * p
            r = r - alpha * q
            rr_new = inner(r, r)
            it += 1
            if np.sqrt(rr_new) <= tol:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        return u

    def apply(self, r, eps_h=1.0):
        """z = M^{-1} r at the current velocity of the fine problem."""
        self._coarse_at_current_velocity()
        g, p = self.R.g, self.R.p
        t = hreg_inv_sqrt(g, r, p.reg, p.beta_v)
        u = self.coarse_cg(resample(t, self.nc), self.kappa * eps_h)
        return hreg_inv_sqrt(g, highpass(g, t) + resample(u, p.n), p.reg, p.beta_v)
