"""The allocation-free interpolation entry point (mireg_interp_noalloc),
called through the C-ABI, against the context's interpolation op on the
same inputs: two calls in a row, the second on a smaller grid (the shared
scratch keeps the first call's tile boxes), both dtypes and orders, with
the oracle's tolerance as a second check."""
import ctypes

import pytest
import torch

from oracle import core
from paper_1808_04487_amd import mireg

from gpu_util import TOL, as_input, need_gpu, rel_err, smooth_scalar, smooth_vector

pytestmark = pytest.mark.gpu


def _case(n, dtype, order, seed):
    g = core.Grid(n)
    f_t, f = as_input(smooth_scalar(g, seed), dtype)
    d_t, d = as_input(smooth_vector(g, seed + 1, amp=5.0, sigma=max(1.5, n[0] / 16)), dtype)
    ctx = mireg.Context(n, order=order, dtype=dtype)
    arg = torch.cat([f_t.reshape(1, -1), d_t.reshape(3, -1)]).contiguous()
    ref = ctx.op("interp", arg)
    torch.cuda.synchronize()
    ctx.close()
    return g, f_t, d_t, ref, core.interp(g, f, d, order)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("order", [3, 1])
def test_noalloc_interp_matches_the_context_op(dtype, order):
    need_gpu()
    print("noalloc interp", dtype, order, flush=True)
    for n, seed in (((64, 64, 64), 71), ((32, 16, 48), 81)):
        g, f_t, d_t, ref, oracle = _case(n, dtype, order, seed)
        out = torch.full_like(f_t, float("nan"))
        mireg.interp_noalloc(f_t, d_t, out, order=order)
        torch.cuda.synchronize()
        print("  grid", n, "bitwise", torch.equal(out, ref), "oracle max rel %.2e" % rel_err(out, oracle),
              flush=True)
        assert torch.equal(out, ref)
        assert rel_err(out, oracle) <= TOL[dtype]


def test_noalloc_interp_errors():
    need_gpu()
    f = torch.zeros((16, 16, 16), device="cuda")
    d = torch.zeros((3, 16, 16, 16), device="cuda")
    lib = mireg.load_library()
    int3 = ctypes.c_int * 3
    rc = lib.mireg_interp_noalloc(int3(16, 16, 1024), 3, mireg.F32, f.data_ptr(), d.data_ptr(), f.data_ptr(), None)
    assert rc == mireg.E_SHAPE and b"1024" in lib.mireg_last_error(None)
    rc = lib.mireg_interp_noalloc(int3(16, 16, 16), 2, mireg.F32, f.data_ptr(), d.data_ptr(),
                                  f.data_ptr(), None)
    assert rc == mireg.E_ARG
    rc = lib.mireg_interp_noalloc(int3(16, 16, 16), 3, mireg.F32, None, d.data_ptr(), f.data_ptr(), None)
    assert rc == mireg.E_ARG
