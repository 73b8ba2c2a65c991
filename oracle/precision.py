"""Oracle model of reduced-precision storage (TEST INFRASTRUCTURE ONLY).

The paper runs its solver in FP32 or FP64 throughout and finds the
Gauss-Newton-Krylov iteration counts unchanged in single precision
(Sec. 4.4, the FP32 vs FP64 runs).  This module models one step further:
FP64 arithmetic everywhere, except that chosen fields are rounded to IEEE
binary16 at the points where they are stored between transport steps.

It repeats the steps of ``core.Registration.gradient`` and
``core.Registration.hessian_matvec`` in the same order, with a store hook:

* ``lam``   - the adjoint history l^nt .. l^1 (l^0 is formed in registers
              and used at once, never stored);
* ``inc``   - the incremental state slices mt^0 .. mt^{nt-1} (stored as the
              step source q^j = mt^j + dt/2 f^j) and the incremental adjoint
              lt^nt .. lt^1;
* ``state`` - the state history m^0 .. m^nt, its gradients taken from the
              stored values.

Rounding is numpy's conversion to float16 (round to nearest even).  With no
field selected the results equal ``core``'s exactly.
"""
import numpy as np

from . import core


def round16(x):
    """Store and reload through IEEE binary16."""
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def _keep(x):
    return x


class StoredRegistration:
    """Gradient and GN matvec of ``core.Registration`` with the fields named
    in ``fields`` (a subset of {"lam", "inc", "state"}) rounded to FP16 where
    they are stored."""

    def __init__(self, reg, fields):
        unknown = set(fields) - {"lam", "inc", "state"}
        if unknown:
            raise ValueError("unknown fields %s" % sorted(unknown))
        self.R = reg
        self.s_lam = round16 if "lam" in fields else _keep
        self.s_inc = round16 if "inc" in fields else _keep
        self.s_state = round16 if "state" in fields else _keep
        self._m = self._gm = None

    def _state(self):
        """State history m^0..m^nt (each slice stored, and transported from
        its stored value) and the gradients of the stored slices."""
        if self._m is None:
            R = self.R
            m = [self.s_state(R.mT)]
            for _ in range(R.p.nt):
                m.append(self.s_state(core.interp(R.g, m[-1], R.X, R.p.order)))
            self._m = m
            self._gm = [core.grad(R.g, mj) for mj in m]
        return self._m, self._gm

    def _backward(self, l_end, gm, store):
        """Adjoint sweep from l^nt (already stored) down to l^0 with the
        trapezoidal time integral b = sum_j a_j l^j grad m^j."""
        R = self.R
        nt = R.p.nt
        lam = l_end
        b = R.a[nt] * lam * gm[nt]
        for j in range(nt - 1, -1, -1):
            lam = core.adjoint_step(R.g, lam, R.Y, R.d, nt, R.p.order)
            if j > 0:
                lam = store(lam)
            b = b + R.a[j] * lam * gm[j]
        return b

    def gradient(self):
        """g = beta_v A v + K[int l grad m dt] with the stored fields."""
        R, p = self.R, self.R.p
        m, gm = self._state()
        b = self._backward(self.s_lam(R.mR - m[-1]), gm, self.s_lam)
        return p.beta_v * core.apply_A(R.g, R.v, p.reg) + core.apply_K(R.g, b, p.div, p.beta_v, p.beta_w)

    def hessian_matvec(self, vt):
        """GN matvec with the stored incremental fields."""
        R, p = self.R, self.R.p
        nt, dt = p.nt, 1.0 / p.nt
        _, gm = self._state()
        vt = np.asarray(vt, dtype=np.float64)
        f = [-np.sum(gm[j] * vt, axis=0) for j in range(nt + 1)]
        # q^j = mt^j + dt/2 f^j is what one step transports
        q = self.s_inc(0.5 * dt * f[0])
        for j in range(nt - 1):
            q = self.s_inc(core.interp(R.g, q, R.X, p.order) + dt * f[j + 1])
        lt = self.s_inc(-(core.interp(R.g, q, R.X, p.order) + 0.5 * dt * f[nt]))
        b = self._backward(lt, gm, self.s_inc)
        return p.beta_v * core.apply_A(R.g, vt, p.reg) + core.apply_K(R.g, b, p.div, p.beta_v, p.beta_w)
