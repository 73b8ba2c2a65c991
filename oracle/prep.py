"""Oracle input preparation (TEST INFRASTRUCTURE ONLY).

Turns the raw seeded draws of ``paper_1808_04487_amd.synth`` into solver
inputs with the oracle's own operators:

* images are smoothed with the spectral Gaussian and rescaled to [0, 1]
  (Sec. 2.3.1);
* smooth random velocities are Gaussian-filtered white noise, Leray projected
  and scaled to a prescribed maximum pointwise Euclidean norm;
* the reference image is the template transported by a velocity with the
  state equation (Sec. 4.2 builds its synthetic reference that way).
"""
import numpy as np

from . import core


def smooth_rescale(g, raw, sigma_vox):
    u = core.gauss_smooth(g, raw, sigma_vox)
    lo, hi = float(u.min()), float(u.max())
    return (u - lo) / (hi - lo)


def smooth_velocity(g, noise, sigma_phys, vmax):
    """Gaussian filter of physical width sigma_phys (sigma_phys / h_a cells per
    axis; the grids used here are cubic), Leray projection, then scaling so
    that max_x |v(x)|_2 = vmax."""
    sig = sigma_phys / g.h[0]
    v = np.stack([core.gauss_smooth(g, noise[a], sig) for a in range(3)])
    v = core.apply_K(g, v, core.DIV_LERAY)
    peak = float(np.sqrt(np.max(np.sum(v * v, axis=0))))
    return v * (vmax / peak)


def transport(g, mT, v, nt=4, order=3):
    """m(1) for the state equation with initial condition mT."""
    X = core.departure_points(g, v, nt, order, -1)
    return core.solve_state(g, mT, X, nt, order)[-1]
