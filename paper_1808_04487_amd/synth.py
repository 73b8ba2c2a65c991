"""Seeded synthetic inputs (FP64 numpy arrays on the host).

This module only draws random numbers and evaluates closed-form input
fields; it holds none of the registration method's arithmetic (no
smoothing, projection, transport or spectral operator).  Both the HIP path
and the CPU oracle start from these arrays and turn them into solver inputs
with their own operators.

Grid convention: n = (n1, n2, n3), point (i1, i2, i3) at x_a = 2 pi i_a / n_a,
arrays C-ordered [n1][n2][n3] (x3 fastest), vector fields [3][n1][n2][n3].
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def coords(n):
    shp = [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]
    return [(np.arange(n[a]) * (TWO_PI / n[a])).reshape(shp[a]) for a in range(3)]


def trig_template(n):
    """Template of the paper's synthetic problem (Sec. 4.2):
    m_T(x) = (sin^2 x1 + sin^2 x2 + sin^2 x3) / 3."""
    x1, x2, x3 = coords(n)
    return ((np.sin(x1) ** 2 + np.sin(x2) ** 2 + np.sin(x3) ** 2) / 3.0).astype(np.float64)


def trig_velocity(n, amplitude=0.5):
    """Velocity of the paper's synthetic problem (Sec. 4.2), scaled by
    ``amplitude``: v1 = sin x3 cos x2 sin x2, v2 = sin x1 cos x3 sin x3,
    v3 = sin x2 cos x1 sin x1."""
    x1, x2, x3 = coords(n)
    shape = tuple(n)
    v = np.empty((3,) + shape, dtype=np.float64)
    v[0] = np.broadcast_to(np.sin(x3) * np.cos(x2) * np.sin(x2), shape)
    v[1] = np.broadcast_to(np.sin(x1) * np.cos(x3) * np.sin(x3), shape)
    v[2] = np.broadcast_to(np.sin(x2) * np.cos(x1) * np.sin(x1), shape)
    return amplitude * v


def voronoi_phantom(n, nseeds=120, seed=1):
    """Piecewise-constant periodic Voronoi image: nseeds points uniform on
    [0, 2 pi)^3 and one intensity U[0,1] per region, drawn in that order from
    numpy's PCG64 generator with ``seed``; each grid point takes the intensity
    of its nearest seed in the periodic (torus) distance."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, TWO_PI, size=(nseeds, 3))
    vals = rng.uniform(0.0, 1.0, size=nseeds)
    tree = cKDTree(np.mod(pts, TWO_PI), boxsize=TWO_PI)
    x1 = np.arange(n[0]) * (TWO_PI / n[0])
    x2, x3 = np.meshgrid(np.arange(n[1]) * (TWO_PI / n[1]),
                         np.arange(n[2]) * (TWO_PI / n[2]), indexing="ij")
    q = np.empty((n[1] * n[2], 3), dtype=np.float64)
    q[:, 1] = x2.ravel()
    q[:, 2] = x3.ravel()
    out = np.empty(tuple(n), dtype=np.float64)
    for i in range(n[0]):  # slab by slab to bound memory
        q[:, 0] = x1[i]
        _, lab = tree.query(q, workers=-1)
        out[i] = vals[lab].reshape(n[1], n[2])
    return out


def white_noise(n, seed, ncomp=3):
    """Independent N(0,1) samples, shape [ncomp][n1][n2][n3]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ncomp,) + tuple(n))


def uniform_field(n, seed, lo=-1.0, hi=1.0, ncomp=None):
    """Independent U[lo, hi) samples (ncomp=None gives a scalar field)."""
    rng = np.random.default_rng(seed)
    shape = tuple(n) if ncomp is None else (ncomp,) + tuple(n)
    return rng.uniform(lo, hi, size=shape)
