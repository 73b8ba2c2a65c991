"""Oracle solver loops (TEST INFRASTRUCTURE ONLY).

Preconditioned CG for the reduced Newton system H vt = -g (Algorithm "Newton
step (inner iterations)", Sec. 2.3.2) and the inexact Gauss-Newton-Krylov
outer loop with Armijo line search (Algorithm "Inexact Newton-Krylov method
(outer iterations)", Sec. 2.3.2).  Readings where the paper is silent:

* forcing: eps_H = min(0.5, sqrt(||g_k|| / ||g_0||)) and PCG stops once
  ||r|| <= eps_H ||r_0|| (a tolerance proportional to the gradient norm, as
  the text states, rather than the absolute test of the listing);
* PCG caps at max_pcg iterations and stops on non-positive curvature
  <s, H s> <= 0, returning the current iterate (M^{-1} rhs if it is the first);
  the matvec that found the curvature is counted, and the stop is reported
  (status NEG_CURV of the solve, a count in the GN report);
* GN stops when ||g_k|| <= eps_g ||g_0|| (the tables report ||g||/||g_0||
  just below eps_g, so the test is on the norm, not its square), or
  ||g_k|| <= grad_atol, or after max_gn iterations;
* Armijo: J(v + a vt) <= J(v) + c1 a <g, vt>, a = 1, 1/2, ..., at most max_ls
  trials, c1 = 1e-4; a failed search keeps v and ends the solve;
* norms and inner products are the trapezoidal L2 ones of the grid;
* PDE-solve counter in the convention of the paper's tables (Sec. 4.7: three
  GN iterations with three matvecs take 15 PDE solves; Table S3:
  #PDE = 2 #matvecs + 2 #iter + 3): 3 for the objective and gradient at the
  initial velocity (a state solve for each and the adjoint solve), 2 per
  matvec, 1 per line-search trial (a state solve) and 1 per accepted step
  (the adjoint solve of the new gradient, whose state the accepted trial
  computed).
"""
import math
import time

import numpy as np

CONVERGED_REL, CONVERGED_ABS, MAXIT, LS_FAIL, NEG_CURV = 1, 2, 3, 4, 5


def pcg(apply_H, apply_Minv, rhs, rtol, maxit, inner, info=None):
    """Solve H x = rhs approximately from x_0 = 0.  Returns (x, iters, relres);
    ``info`` (a dict, optional) receives "matvecs" (applications of H, the
    iterations plus one when the loop stops on non-positive curvature) and
    "status" (CONVERGED_REL, MAXIT or NEG_CURV)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    r0 = math.sqrt(inner(r, r))
    if info is not None:
        info["matvecs"], info["status"] = 0, CONVERGED_REL
    if r0 == 0.0:
        return x, 0, 0.0
    z = apply_Minv(r)
    s = z.copy()
    rz = inner(r, z)
    it = 0
    rnorm = r0
    status = MAXIT
    while it < maxit:
        Hs = apply_H(s)
        if info is not None:
            info["matvecs"] += 1
        sHs = inner(s, Hs)
        if sHs <= 0.0:
            if it == 0:
                x = z.copy()
            status = NEG_CURV
            break
        kappa = rz / sHs
        x = x + kappa * s
        r = r - kappa * Hs
        it += 1
        rnorm = math.sqrt(inner(r, r))
        if rnorm <= rtol * r0:
            status = CONVERGED_REL
            break
        z = apply_Minv(r)
        rz_new = inner(r, z)
        mu = rz_new / rz
        rz = rz_new
        s = z + mu * s
    if info is not None:
        info["status"] = status
    return x, it, rnorm / r0


class Report:
    def __init__(self):
        self.status = 0
        self.gn_iters = 0
        self.matvecs = 0
        self.pde_solves = 0
        self.pcg_iters = 0
        self.ls_trials = 0
        self.J0 = self.J = 0.0
        self.mismatch_rel = 0.0
        self.gnorm0 = self.gnorm = self.gnorm_rel = 0.0
        self.seconds = 0.0
        self.coarse_matvecs = 0
        self.neg_curv = 0
        self.history = []

    def as_dict(self):
        return {k: getattr(self, k) for k in (
            "status", "gn_iters", "matvecs", "pde_solves", "pcg_iters", "ls_trials", "J0", "J",
            "mismatch_rel", "gnorm0", "gnorm", "gnorm_rel", "seconds", "coarse_matvecs", "neg_curv")}


def gn_solve(reg, v0, grad_rtol=5e-2, grad_atol=1e-6, max_gn=50, max_pcg=100,
             armijo_c1=1e-4, max_ls=10, precond=None):
    """Inexact GN-Krylov solve for the registration problem ``reg``
    (an ``oracle.core.Registration``) from the initial velocity v0.
    ``precond``: None for the spectral preconditioner, else an object with
    ``apply(r, eps_h)`` (and a ``coarse_matvecs`` count) such as
    ``oracle.twolevel.TwoLevel``, applied at the current velocity."""
    t0 = time.perf_counter()
    g_ = reg.g
    inner = g_.inner
    rep = Report()
    v = np.array(v0, dtype=np.float64, copy=True)
    reg.set_velocity(v)
    J = reg.objective()[0]
    grad = reg.gradient()
    rep.pde_solves += 3  # the paper counts a state solve for J and for g, and the adjoint
    g0 = math.sqrt(inner(grad, grad))
    rep.J0, rep.gnorm0 = J, g0
    k = 0
    while True:
        gnorm = math.sqrt(inner(grad, grad))
        rep.history.append({"iter": k, "J": J, "gnorm": gnorm})
        if gnorm <= grad_rtol * g0:
            rep.status = CONVERGED_REL
            break
        if gnorm <= grad_atol:
            rep.status = CONVERGED_ABS
            break
        if k >= max_gn:
            rep.status = MAXIT
            break
        eps_h = min(0.5, math.sqrt(gnorm / g0))
        minv = reg.precond if precond is None else (lambda r, e=eps_h: precond.apply(r, e))
        info = {}
        vt, its, _ = pcg(reg.hessian_matvec, minv, -grad, eps_h, max_pcg, inner, info)
        rep.matvecs += info["matvecs"]
        rep.pcg_iters += its
        rep.pde_solves += 2 * info["matvecs"]
        rep.neg_curv += info["status"] == NEG_CURV
        slope = inner(grad, vt)
        alpha = 1.0
        accepted = False
        for _ in range(max_ls):
            vtrial = v + alpha * vt
            reg.set_velocity(vtrial)
            Jt = reg.objective()[0]
            rep.ls_trials += 1
            rep.pde_solves += 1
            if Jt <= J + armijo_c1 * alpha * slope:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            reg.set_velocity(v)
            rep.status = LS_FAIL
            break
        v, J = vtrial, Jt
        grad = reg.gradient()
        rep.pde_solves += 1
        k += 1
    rep.gn_iters = k
    rep.coarse_matvecs = precond.coarse_matvecs if precond is not None else 0
    rep.J = J
    rep.gnorm = math.sqrt(inner(grad, grad))
    rep.gnorm_rel = rep.gnorm / g0 if g0 > 0 else 0.0
    rep.mismatch_rel = reg.mismatch_rel()
    rep.seconds = time.perf_counter() - t0
    return v, rep
