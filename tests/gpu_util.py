"""Helpers for the GPU parity tests (oracle vs the HIP library)."""
import numpy as np
import pytest
import torch

from oracle import core

# FP64 fields: the two sides differ only by rounding order (FFT algorithm,
# summation order of the 64-node stencil).  FP32 fields: inputs are rounded
# to FP32 before both sides see them, so the bound covers FP32 arithmetic in
# the kernels (unit roundoff 6e-8) amplified by FFT depth (log2 N ~ 24) and
# the chained transport steps.
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def as_input(a, dtype):
    """Round an FP64 array to the test dtype; return (tensor on GPU, FP64
    numpy copy of exactly the values the GPU sees)."""
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dtype)
    return t.cuda(), t.double().numpy()


def rel_err(got, ref):
    got = got.detach().double().cpu().numpy() if isinstance(got, torch.Tensor) else np.asarray(got)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        return float(np.abs(got).max())
    return float(np.abs(got - ref).max() / scale)


def rel_err_l2(got, ref):
    got = got.detach().double().cpu().numpy() if isinstance(got, torch.Tensor) else np.asarray(got)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def assert_close(got, ref, dtype, factor=1.0, what=""):
    e = rel_err(got, ref)
    tol = TOL[dtype] * factor
    if what:
        print("  %s: max rel %.2e (bound %.0e)" % (what, e, tol), flush=True)
    assert e <= tol, "%s: max rel error %.3e > %.1e" % (what, e, tol)
    return e


def assert_close_composite(got, ref, dtype, what=""):
    """Composite operators (gradient, matvec): FP64 max-relative 5 TOL
    (rounding of a few hundred chained operations); FP32 the field tolerance
    1e-5 itself, both in the L2-relative and the max-relative sense."""
    if dtype == torch.float64:
        return assert_close(got, ref, dtype, factor=5, what=what)
    tol = TOL[dtype]
    e2 = rel_err_l2(got, ref)
    e = rel_err(got, ref)
    print("%s: L2 rel %.2e, max rel %.2e (bound %.0e)" % (what, e2, e, tol), flush=True)
    assert e2 <= tol, "%s: L2 rel error %.3e > %.1e" % (what, e2, tol)
    assert e <= tol, "%s: max rel error %.3e > %.1e" % (what, e, tol)
    return e


def smooth_vector(g, seed, amp=1.0, sigma=2.0):
    rng = np.random.default_rng(seed)
    v = np.stack([core.gauss_smooth(g, rng.standard_normal(g.n), sigma) for _ in range(3)])
    return amp * v / np.abs(v).max()


def smooth_scalar(g, seed, sigma=1.5):
    rng = np.random.default_rng(seed)
    u = core.gauss_smooth(g, rng.standard_normal(g.n), sigma)
    return u / np.abs(u).max()
