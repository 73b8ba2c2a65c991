"""Python binding of the mireg C-ABI (include/mireg.h).

Argument marshalling only: tensors are checked (device, dtype, shape,
contiguity) and their device pointers handed to libmireg.so, which runs
every step on the GPU.  There is no fallback: if the library is missing
this module raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmireg.so")

OK, E_ARG, E_SHAPE, E_STATE, E_HIP, E_NOMEM, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
F32, F64, F32_H16 = 0, 1, 2
H1, H2 = 1, 2
DIV_NONE, DIV_NEAR, DIV_LERAY = 0, 1, 2
CONVERGED_REL, CONVERGED_ABS, MAXIT, LS_FAIL, NEG_CURV = 1, 2, 3, 4, 5
PC_SPECTRAL, PC_TWO_LEVEL = 0, 1

OPS = {
    "grad": 1, "div": 2, "laplace": 3, "apply_A": 4, "apply_K": 5, "leray": 6, "precond": 7,
    "gauss": 8, "departure_X": 9, "departure_Y": 10, "transport_state": 11, "interp": 12,
    "rescale01": 13, "scale_maxnorm": 14, "transport_adjoint": 15,
}
# (input components, output components); interp takes f and a displacement (1 + 3)
_OP_SHAPES = {
    "grad": (1, 3), "div": (3, 1), "laplace": (1, 1), "apply_A": (3, 3), "apply_K": (3, 3),
    "leray": (3, 3), "precond": (3, 3), "gauss": (1, 1), "departure_X": (3, 3),
    "departure_Y": (3, 3), "transport_state": (1, 1), "interp": (4, 1), "rescale01": (1, 1),
    "scale_maxnorm": (3, 3), "transport_adjoint": (1, 1),
}


class MiregError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mireg error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("nt", ctypes.c_int), ("interp_order", ctypes.c_int),
                ("reg", ctypes.c_int), ("div", ctypes.c_int), ("beta_v", ctypes.c_double),
                ("beta_w", ctypes.c_double), ("dtype", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("grad_rtol", ctypes.c_double), ("grad_atol", ctypes.c_double),
                ("max_gn", ctypes.c_int), ("max_pcg", ctypes.c_int),
                ("armijo_c1", ctypes.c_double), ("max_ls", ctypes.c_int),
                ("log_level", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("gn_iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("pde_solves", ctypes.c_int), ("pcg_iters", ctypes.c_int),
                ("ls_trials", ctypes.c_int), ("J0", ctypes.c_double), ("J", ctypes.c_double),
                ("mismatch_rel", ctypes.c_double), ("gnorm0", ctypes.c_double),
                ("gnorm", ctypes.c_double), ("gnorm_rel", ctypes.c_double),
                ("seconds", ctypes.c_double), ("coarse_matvecs", ctypes.c_int),
                ("neg_curv", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Timers(ctypes.Structure):
    _fields_ = [("fft_ms", ctypes.c_double), ("interp_ms", ctypes.c_double),
                ("other_ms", ctypes.c_double), ("launches", ctypes.c_long)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_long), ("total_ms", ctypes.c_double),
                ("bytes_per_launch", ctypes.c_double)]


# exported symbols and their signatures (argtypes, restype)
_vp, _ip, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "mireg_default_params": ([ctypes.POINTER(Params)], None),
    "mireg_default_solve_opts": ([ctypes.POINTER(SolveOpts)], None),
    "mireg_create": ([ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "mireg_destroy": ([_vp], ctypes.c_int),
    "mireg_last_error": ([_vp], ctypes.c_char_p),
    "mireg_workspace_bytes": ([_vp], ctypes.c_size_t),
    "mireg_set_images": ([_vp, _vp, _vp], ctypes.c_int),
    "mireg_set_velocity": ([_vp, _vp], ctypes.c_int),
    "mireg_get_velocity": ([_vp, _vp], ctypes.c_int),
    "mireg_objective": ([_vp, _dp, _dp, _dp], ctypes.c_int),
    "mireg_gradient": ([_vp, _vp, _dp], ctypes.c_int),
    "mireg_hessian_matvec": ([_vp, _vp, _vp], ctypes.c_int),
    "mireg_precond_apply": ([_vp, _vp, _vp], ctypes.c_int),
    "mireg_pcg_solve": ([_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _ip, _dp, _ip], ctypes.c_int),
    "mireg_gn_solve": ([_vp, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(Report)], ctypes.c_int),
    "mireg_op": ([_vp, ctypes.c_int, _vp, _vp, ctypes.c_double], ctypes.c_int),
    "mireg_set_precond": ([_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "mireg_set_graphs": ([_vp, ctypes.c_int], ctypes.c_int),
    "mireg_set_log_jsonl": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "mireg_get_tuning": ([_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "mireg_set_tuning": ([_vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "mireg_autotune": ([_vp, ctypes.c_int, _dp, _ip], ctypes.c_int),
    "mireg_timers_enable": ([_vp, ctypes.c_int], ctypes.c_int),
    "mireg_kernel_stats_enable": ([_vp, ctypes.c_int], ctypes.c_int),
    "mireg_kernel_stats_read": ([_vp, ctypes.POINTER(KernelStat), ctypes.c_int, _ip, ctypes.c_int], ctypes.c_int),
    "mireg_timers_read": ([_vp, ctypes.POINTER(Timers), ctypes.c_int], ctypes.c_int),
    "mireg_interp_noalloc": ([ctypes.c_int * 3, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp], ctypes.c_int),
    "mireg_batch_create": ([ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
    "mireg_batch_destroy": ([_vp], ctypes.c_int),
    "mireg_batch_last_error": ([_vp], ctypes.c_char_p),
    "mireg_batch_pcg_solve": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp, ctypes.c_int, _ip, _dp, _ip],
                              ctypes.c_int),
    "mireg_batch_gn_solve": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(SolveOpts), ctypes.POINTER(Report)],
                             ctypes.c_int),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libmireg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MiregError(E_STATE, "%s is missing: build it with __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _torch_dtype(dtype):
    """(boundary torch dtype, library code); "f32h16" is FP32 arithmetic with
    FP16 storage of the adjoint history and the incremental fields."""
    if dtype in (torch.float32, "f32", "float32", F32):
        return torch.float32, F32
    if dtype in (torch.float64, "f64", "float64", F64):
        return torch.float64, F64
    if dtype in ("f32h16", F32_H16):
        return torch.float32, F32_H16
    raise ValueError("dtype must be float32, float64 or 'f32h16'")


class Context:
    """One registration problem on the current CUDA (HIP) device.

    n: grid (n1, n2, n3); nt: time steps; order: 3 (tricubic) or 1
    (trilinear); reg: H1 or H2; div: DIV_NONE / DIV_NEAR / DIV_LERAY.
    All work runs on the torch stream current at creation.
    """

    def __init__(self, n, nt=4, order=3, reg=H1, div=DIV_NONE, beta_v=1e-2, beta_w=0.0,
                 dtype=torch.float32, device=None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise MiregError(E_STATE, "no HIP device available")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.dtype, code = _torch_dtype(dtype)
        self.dtype_name = {F32: "f32", F64: "f64", F32_H16: "f32h16"}[code]
        self.n = tuple(int(x) for x in n)
        p = Params()
        self.lib.mireg_default_params(ctypes.byref(p))
        p.n[0], p.n[1], p.n[2] = self.n
        p.nt, p.interp_order, p.reg, p.div = int(nt), int(order), int(reg), int(div)
        p.beta_v, p.beta_w, p.dtype = float(beta_v), float(beta_w), code
        self.params = p
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            rc = self.lib.mireg_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise MiregError(rc, "mireg_create failed for n=%s" % (self.n,))
        self.h = h
        self.N = self.n[0] * self.n[1] * self.n[2]

    # -- helpers ------------------------------------------------------------
    def _check(self, rc):
        if rc != OK:
            raise MiregError(rc, self.lib.mireg_last_error(self.h).decode())

    def _arg(self, t, comps, name):
        shape = self.n if comps == 1 else (comps,) + self.n
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device or t.dtype != self.dtype:
            raise ValueError("%s must be %s on %s" % (name, self.dtype, self.device))
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError("%s must be a contiguous tensor of shape %s" % (name, shape))
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, comps=1):
        shape = self.n if comps == 1 else (comps,) + self.n
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mireg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- C-ABI mirrors ------------------------------------------------------
    def workspace_bytes(self):
        return int(self.lib.mireg_workspace_bytes(self.h))

    def set_images(self, mT, mR):
        self._check(self.lib.mireg_set_images(self.h, self._arg(mT, 1, "mT"), self._arg(mR, 1, "mR")))

    def set_velocity(self, v):
        self._check(self.lib.mireg_set_velocity(self.h, self._arg(v, 3, "v")))

    def get_velocity(self, out=None):
        out = self.empty(3) if out is None else out
        self._check(self.lib.mireg_get_velocity(self.h, self._arg(out, 3, "out")))
        return out

    def objective(self):
        J, mis, reg = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.mireg_objective(self.h, ctypes.byref(J), ctypes.byref(mis), ctypes.byref(reg)))
        return J.value, mis.value, reg.value

    def gradient(self, out=None):
        out = self.empty(3) if out is None else out
        gn = ctypes.c_double()
        self._check(self.lib.mireg_gradient(self.h, self._arg(out, 3, "g"), ctypes.byref(gn)))
        return out, gn.value

    def hessian_matvec(self, vt, out=None):
        out = self.empty(3) if out is None else out
        self._check(self.lib.mireg_hessian_matvec(self.h, self._arg(vt, 3, "vt"), self._arg(out, 3, "Hvt")))
        return out

    def set_graphs(self, on=True):
        self._check(self.lib.mireg_set_graphs(self.h, int(bool(on))))

    def set_log_jsonl(self, path=None):
        """Append one JSON line per GN iteration of gn_solve to `path`
        (None closes the log)."""
        self._check(self.lib.mireg_set_log_jsonl(self.h, path.encode() if path else None))

    def autotune(self, reps=3):
        """Pick the fastest transport tile shape (and Krylov x1 width where
        there are two); returns (shape, ms per PCG iteration per shape)."""
        ms = (ctypes.c_double * 3)()
        sh = ctypes.c_int()
        self._check(self.lib.mireg_autotune(self.h, int(reps), ms, ctypes.byref(sh)))
        return sh.value, list(ms)

    def tuning(self):
        """(transport tile shape, Krylov x1 width: 1 for 16 columns)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.mireg_get_tuning(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_tuning(self, shape, narrow=0):
        self._check(self.lib.mireg_set_tuning(self.h, int(shape), int(narrow)))

    def set_precond(self, kind, kappa=0.1, max_inner=50):
        """PC_SPECTRAL or PC_TWO_LEVEL (coarse CG to kappa times the PCG tolerance)."""
        k = {"spectral": PC_SPECTRAL, "two_level": PC_TWO_LEVEL}.get(kind, kind)
        self._check(self.lib.mireg_set_precond(self.h, int(k), float(kappa), int(max_inner)))

    def precond(self, r, out=None):
        out = self.empty(3) if out is None else out
        self._check(self.lib.mireg_precond_apply(self.h, self._arg(r, 3, "r"), self._arg(out, 3, "z")))
        return out

    def pcg(self, rhs, rtol=1e-3, maxit=100, out=None, with_status=False):
        """Returns (x, iterations, relative residual[, status])."""
        out = self.empty(3) if out is None else out
        it, rel, st = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        self._check(self.lib.mireg_pcg_solve(self.h, self._arg(rhs, 3, "rhs"), self._arg(out, 3, "x"),
                                             float(rtol), int(maxit), ctypes.byref(it), ctypes.byref(rel),
                                             ctypes.byref(st)))
        return (out, it.value, rel.value, st.value) if with_status else (out, it.value, rel.value)

    def gn_solve(self, v0=None, grad_rtol=5e-2, grad_atol=1e-6, max_gn=50, max_pcg=100,
                 armijo_c1=1e-4, max_ls=10, log_level=0):
        """Returns (v, report dict); v0 (warm start) defaults to zero."""
        v = torch.zeros((3,) + self.n, dtype=self.dtype, device=self.device) if v0 is None else v0.clone()
        o = SolveOpts(float(grad_rtol), float(grad_atol), int(max_gn), int(max_pcg), float(armijo_c1),
                      int(max_ls), int(log_level))
        rep = Report()
        self._check(self.lib.mireg_gn_solve(self.h, self._arg(v, 3, "v"), ctypes.byref(o), ctypes.byref(rep)))
        return v, rep.as_dict()

    def op(self, name, x, arg=0.0, out=None):
        cin, cout = _OP_SHAPES[name]
        if name == "interp":
            if not (isinstance(x, torch.Tensor) and x.numel() == 4 * self.N and x.is_contiguous()):
                raise ValueError("interp takes a contiguous [4][n...] tensor (f then displacement)")
            ptr = self._arg(x.view((4,) + self.n), 4, "x")
        else:
            ptr = self._arg(x, cin, "x")
        out = self.empty(cout) if out is None else out
        self._check(self.lib.mireg_op(self.h, OPS[name], ptr, self._arg(out, cout, "out"), float(arg)))
        return out

    def kernel_stats(self, enable=None, reset=False):
        """Per-kernel event timing: {name: (launches, total_ms, bytes_per_launch)}."""
        if enable is not None:
            self._check(self.lib.mireg_kernel_stats_enable(self.h, int(bool(enable))))
        buf = (KernelStat * 64)()
        cnt = ctypes.c_int()
        self._check(self.lib.mireg_kernel_stats_read(self.h, buf, 64, ctypes.byref(cnt), int(bool(reset))))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].bytes_per_launch)
                for i in range(cnt.value)}

    def timers(self, enable=None, reset=False):
        if enable is not None:
            self._check(self.lib.mireg_timers_enable(self.h, int(bool(enable))))
        t = Timers()
        self._check(self.lib.mireg_timers_read(self.h, ctypes.byref(t), int(bool(reset))))
        return {"fft_ms": t.fft_ms, "interp_ms": t.interp_ms, "other_ms": t.other_ms, "launches": t.launches}


def interp_noalloc(f, disp, out, order=3):
    """out = I[f](x + disp) through the allocation-free entry point (no
    context; f, disp, out contiguous CUDA tensors of one dtype, shapes
    [n1, n2, n3], [3, n1, n2, n3], [n1, n2, n3]); enqueued on the current
    torch stream, not synchronised."""
    lib = load_library()
    n = tuple(f.shape)
    if len(n) != 3 or tuple(disp.shape) != (3,) + n or tuple(out.shape) != n:
        raise ValueError("shapes must be [n1, n2, n3], [3, n1, n2, n3], [n1, n2, n3]")
    if not (f.dtype == disp.dtype == out.dtype) or f.dtype not in (torch.float32, torch.float64):
        raise ValueError("f, disp and out must share dtype float32 or float64")
    for t in (f, disp, out):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("tensors must be contiguous CUDA tensors")
    code = F32 if f.dtype == torch.float32 else F64
    stream = torch.cuda.current_stream(f.device).cuda_stream
    rc = lib.mireg_interp_noalloc((ctypes.c_int * 3)(*n), int(order), code, f.data_ptr(), disp.data_ptr(),
                                  out.data_ptr(), stream)
    if rc != OK:
        raise MiregError(rc, lib.mireg_last_error(None).decode())
    return out


class Batch:
    """Lockstep solves of several contexts (any grid sizes; the same dtype,
    nt, order, stream and tile shape): one transport launch per matvec step
    across the problems, one PCG read-back per iteration for all of them."""

    def __init__(self, ctxs):
        self.lib = load_library()
        self.ctxs = list(ctxs)
        arr = (_vp * len(self.ctxs))(*[c.h for c in self.ctxs])
        h = _vp()
        rc = self.lib.mireg_batch_create(arr, len(self.ctxs), ctypes.byref(h))
        if rc != OK:
            raise MiregError(rc, "mireg_batch_create: contexts do not match or allocation failed")
        self.h = h

    def _check(self, rc):
        if rc != OK:
            raise MiregError(rc, self.lib.mireg_batch_last_error(self.h).decode())

    def _ptrs(self, tensors, comps, name):
        return (_vp * len(tensors))(*[c._arg(t, comps, name) for c, t in zip(self.ctxs, tensors)])

    def pcg(self, rhs, rtol=1e-3, maxit=100):
        """Returns ([x], [iterations], [relative residual], [status])."""
        P = len(self.ctxs)
        xs = [c.empty(3) for c in self.ctxs]
        rt = (ctypes.c_double * P)(*([float(rtol)] * P if not isinstance(rtol, (list, tuple)) else rtol))
        it, rel, st = (ctypes.c_int * P)(), (ctypes.c_double * P)(), (ctypes.c_int * P)()
        self._check(self.lib.mireg_batch_pcg_solve(self.h, self._ptrs(rhs, 3, "rhs"), self._ptrs(xs, 3, "x"), rt,
                                                   int(maxit), it, rel, st))
        return xs, list(it), list(rel), list(st)

    def gn_solve(self, v0=None, grad_rtol=5e-2, grad_atol=1e-6, max_gn=50, max_pcg=100, armijo_c1=1e-4,
                 max_ls=10, log_level=0):
        """Returns ([v], [report dict]); v0 (warm starts) defaults to zeros."""
        vs = [torch.zeros((3,) + c.n, dtype=c.dtype, device=c.device) if v0 is None else v0[i].clone()
              for i, c in enumerate(self.ctxs)]
        o = SolveOpts(float(grad_rtol), float(grad_atol), int(max_gn), int(max_pcg), float(armijo_c1),
                      int(max_ls), int(log_level))
        reps = (Report * len(self.ctxs))()
        self._check(self.lib.mireg_batch_gn_solve(self.h, self._ptrs(vs, 3, "v"), ctypes.byref(o), reps))
        return vs, [r.as_dict() for r in reps]

    def close(self):
        if getattr(self, "h", None):
            self.lib.mireg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
