"""Learned warm start for the GN-Krylov solver: Python binding of
include/mireg_net.h, training-data generation with the solver itself, the
training loop and the warm-started solve.

Everything numeric runs in libmireg.so (the network's forward and backward
passes, Adam, the phantom labels, the solver); this module marshals device
pointers, draws the seeded random numbers and keeps the bookkeeping.

Training pairs (128^3 by default): a periodic Voronoi phantom (120 seeds,
values U[0, 1], spectral Gaussian of 2 cells, rescaled to [0, 1]) as
template, a smooth random velocity (white noise, Gaussian of physical width
pi/4, Leray projection, max |v| drawn from U[0.05, 0.15] 2 pi) transports it
to the reference, and the plain GN-Krylov solve from v = 0 of that pair
(H1-div, beta_v = 5e-3, beta_w = 1, nt = 4, relative gradient 5e-2) is the
network's target.
"""
import ctypes
import math
import os
import time

import numpy as np
import torch

from . import mireg

TWO_PI = 2.0 * math.pi
CHANNELS = (16, 32, 64, 128)
SKIP_SIGMA = 4.0
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


class NetConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("channels", ctypes.c_int * 4), ("skip_sigma", ctypes.c_double)]


_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_vpp = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "mireg_net_create": ([ctypes.POINTER(NetConfig), _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "mireg_net_destroy": ([_vp], ctypes.c_int),
    "mireg_net_last_error": ([_vp], ctypes.c_char_p),
    "mireg_net_param_count": ([_vp], ctypes.c_longlong),
    "mireg_net_set_params": ([_vp, _vp], ctypes.c_int),
    "mireg_net_get_params": ([_vp, _vp], ctypes.c_int),
    "mireg_net_forward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "mireg_net_loss_grad": ([_vp, _vp, _vp, _vp, _dp, _vp], ctypes.c_int),
    "mireg_net_train_step": ([_vp, ctypes.c_int, _vpp, _vpp, _vpp, ctypes.c_double, _dp], ctypes.c_int),
    "mireg_net_voronoi": ([_vp, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
}


def _lib():
    lib = mireg.load_library()
    if not getattr(lib, "_net_bound", False):
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        lib._net_bound = True
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class WarmStartNet:
    """The network on one device: predict, train, save and load parameters."""

    def __init__(self, n, channels=CHANNELS, skip_sigma=SKIP_SIGMA, device=None):
        self.lib = _lib()
        if not torch.cuda.is_available():
            raise mireg.MiregError(mireg.E_STATE, "no HIP device available")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.n, self.channels, self.skip_sigma = int(n), tuple(int(c) for c in channels), float(skip_sigma)
        cfg = NetConfig()
        cfg.n = self.n
        for i, c in enumerate(self.channels):
            cfg.channels[i] = c
        cfg.skip_sigma = self.skip_sigma
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            rc = self.lib.mireg_net_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != mireg.OK:
            raise mireg.MiregError(rc, "mireg_net_create failed for n=%d channels=%s" % (self.n, self.channels))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mireg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != mireg.OK:
            raise mireg.MiregError(rc, self.lib.mireg_net_last_error(self.h).decode())

    def _field(self, t, comps, name):
        shape = (self.n,) * 3 if comps == 1 else (comps,) + (self.n,) * 3
        if t.device != self.device or t.dtype != torch.float32 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError("%s must be a contiguous float32 %s tensor on %s" % (name, shape, self.device))
        return _ptr(t)

    @property
    def param_count(self):
        return int(self.lib.mireg_net_param_count(self.h))

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.size != self.param_count:
            raise ValueError("expected %d parameters, got %d" % (self.param_count, theta.size))
        self._check(self.lib.mireg_net_set_params(self.h, theta.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        out = np.empty(self.param_count, dtype=np.float32)
        self._check(self.lib.mireg_net_get_params(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def forward(self, mT, mR, out=None):
        out = torch.empty((3,) + (self.n,) * 3, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.mireg_net_forward(self.h, self._field(mT, 1, "mT"), self._field(mR, 1, "mR"),
                                               self._field(out, 3, "v")))
        return out

    def loss_grad(self, mT, mR, vt):
        loss = ctypes.c_double()
        g = np.empty(self.param_count, dtype=np.float32)
        self._check(self.lib.mireg_net_loss_grad(self.h, self._field(mT, 1, "mT"), self._field(mR, 1, "mR"),
                                                 self._field(vt, 3, "v_target"), ctypes.byref(loss),
                                                 g.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, g

    def train_step(self, batch, lr):
        """batch: list of (mT, mR, v_target) device tensors; returns the mean loss."""
        B = len(batch)
        arr = lambda k, c, nm: (ctypes.c_void_p * B)(*[self._field(p[k], c, nm) for p in batch])
        loss = ctypes.c_double()
        self._check(self.lib.mireg_net_train_step(self.h, B, arr(0, 1, "mT"), arr(1, 1, "mR"), arr(2, 3, "v_target"),
                                                  float(lr), ctypes.byref(loss)))
        return loss.value

    def voronoi(self, seeds, values, out=None):
        seeds = np.ascontiguousarray(seeds, dtype=np.float32).reshape(-1, 3)
        values = np.ascontiguousarray(values, dtype=np.float32).ravel()
        out = torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.mireg_net_voronoi(self.h, len(values), seeds.ctypes.data_as(ctypes.c_void_p),
                                               values.ctypes.data_as(ctypes.c_void_p), self._field(out, 1, "out")))
        return out

    def save(self, path):
        np.savez(path, params=self.get_params(), n=self.n, channels=np.array(self.channels),
                 skip_sigma=self.skip_sigma)

    @classmethod
    def load(cls, path, device=None):
        with np.load(path, allow_pickle=False) as z:
            net = cls(int(z["n"]), tuple(int(c) for c in z["channels"]), float(z["skip_sigma"]), device=device)
            net.set_params(z["params"])
        return net


def init_params(channels, seed):
    """He-scaled normal weights and zero biases (flat layout of mireg_net.h);
    the two output maps start at zero, so the untrained network predicts 0."""
    rng = np.random.default_rng(seed)
    c0, c1, c2, c3 = channels
    layers = [(2, c0, 27), (c0, c1, 27), (c1, c2, 27), (c2, c3, 27), (c3, c2, 27), (c2, c1, 27), (c1, c0, 27),
              (c0, 3, 0), (c3, 3, 0)]
    parts = []
    for ci, co, t in layers:
        if t == 0:
            parts += [np.zeros(co * ci), np.zeros(co)]
        else:
            parts += [rng.standard_normal(co * t * ci) * math.sqrt(2.0 / (t * ci)), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


# ---- training data ----
def registration_context(n, device=None):
    """The solver configuration that labels the training pairs and evaluates the warm start."""
    return mireg.Context((n, n, n), nt=4, order=3, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=5e-3, beta_w=1.0,
                         dtype=torch.float32, device=device)


def make_pair(net, ctx, seed, solve=True):
    """(mT, mR, v_target, v_true, report) for one seeded pair; the target is the
    plain GN-Krylov solution from v = 0 (or v_true when solve is False)."""
    n = net.n
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, TWO_PI, (120, 3))
    values = rng.uniform(0.0, 1.0, 120)
    raw = net.voronoi(seeds, values)
    mT = ctx.op("rescale01", ctx.op("gauss", raw, 2.0))
    noise = torch.from_numpy(rng.standard_normal((3, n, n, n)).astype(np.float32)).to(net.device)
    sm = torch.stack([ctx.op("gauss", noise[c].contiguous(), n / 8.0) for c in range(3)]).contiguous()
    amp = rng.uniform(0.05, 0.15) * TWO_PI
    v_true = ctx.op("scale_maxnorm", ctx.op("leray", sm), amp)
    ctx.set_velocity(v_true)
    mR = ctx.op("transport_state", mT)
    rep = None
    if solve:
        ctx.set_images(mT, mR)
        vt, rep = ctx.gn_solve(grad_rtol=5e-2)
    else:
        vt = v_true
    return mT, mR, vt.contiguous(), v_true, rep


def train(net, pairs, steps, lr=1e-3, batch=4, seed=0, log=None):
    """Adam on random mini-batches of the stored pairs; returns the losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for s in range(steps):
        idx = rng.choice(len(pairs), size=batch, replace=False)
        losses.append(net.train_step([pairs[i][:3] for i in idx], lr))
        if log and (s % 50 == 0 or s == steps - 1):
            log("step %d loss %.4e" % (s, losses[-1]))
    return losses


# ---- warm-started solve ----
def solve_pair(ctx, mT, mR, net=None, grad_rtol=5e-2):
    """GN-Krylov solve of one pair from v = 0, and, with a network, from its
    prediction to the same absolute gradient tolerance (grad_rtol times the
    gradient norm at v = 0).  The plain start is the fallback: the predicted
    velocity is used only if its objective is below the objective at v = 0.
    The warm timing is standalone: it includes the objective and gradient at
    v = 0 (state and adjoint solves) that set its tolerance and fallback, not
    the plain solve's values.
    Returns {"plain": (report, seconds), "warm": (report, seconds, used)}."""
    ctx.set_images(mT, mR)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep0 = ctx.gn_solve(grad_rtol=grad_rtol)
    torch.cuda.synchronize()
    out = {"plain": (rep0, time.perf_counter() - t0)}
    if net is None:
        return out
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_velocity(torch.zeros((3,) + ctx.n, dtype=ctx.dtype, device=ctx.device))
    J_zero = ctx.objective()[0]
    _, g_zero = ctx.gradient()
    atol = grad_rtol * g_zero
    v0 = net.forward(mT, mR)
    ctx.set_velocity(v0)
    J_pred = ctx.objective()[0]
    used = J_pred < J_zero
    _, rep = ctx.gn_solve(v0=v0 if used else None, grad_rtol=0.0 if used else grad_rtol, grad_atol=atol)
    torch.cuda.synchronize()
    out["warm"] = (rep, time.perf_counter() - t0, used)
    return out
