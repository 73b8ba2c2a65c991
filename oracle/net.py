"""Oracle of the learned warm start (TEST INFRASTRUCTURE ONLY): FP64 forward
pass, hand-written backward pass and loss of the velocity-predicting network.

The paper has no learning component; its solver starts each Gauss-Newton
solve from a given velocity (v = 0, or the previous solution during the
beta_v continuation, Sec. 3.6).  The network maps an image pair (mT, mR) on
the periodic n^3 grid to such an initial velocity:

  x  = (mT, mR)                                     2 channels, n^3
  e0 = relu(C(x))                                   c0 channels, n^3
  e1 = relu(C(P e0)), e2 = relu(C(P e1)), e3 = relu(C(P e2))   n/2, n/4, n/8
  d2 = relu(C(U e3) + e2), d1 = relu(C(U d2) + e1), d0 = relu(C(U d1) + e0)
  y  = H d0                                         3 channels, n^3
  s  = G_sigma(U8 H3 e3)                            3 channels, n^3 (spectral skip)
  v  = Leray(y + s)

C is a periodic 3x3x3 convolution with bias, P the 2x2x2 mean, U nearest
upsampling by 2 (U8 by 8), H and H3 pointwise (1x1x1) maps, G_sigma the
spectral Gaussian of the core oracle, Leray the projection of the core
oracle.  Loss: L = |v - v_target|^2 / (2 * 3 n^3).

Parameters are one flat vector: for each layer in LAYERS order, W[Cout][T][Cin]
(T = 27 taps, or 1) then b[Cout].  Tap t = 9 (d1+1) + 3 (d2+1) + (d3+1) reads
the input at x + (d1, d2, d3) (periodic).

``bf16=True`` rounds (round to nearest even) where a BF16 implementation
stores values: the inputs, the weights of the 3x3x3 layers, every activation
e*, p*, d*, and the masked gradients fed to the 3x3x3 layers' adjoints (data,
weight and bias gradients); the skip connections carry the unrounded masked
gradients.  Accumulation stays FP64.
"""
import numpy as np

from . import core

TAPS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]


def layers(ch):
    """(name, Cin, Cout, taps) of every layer for level channels ch = (c0..c3)."""
    c0, c1, c2, c3 = ch
    return [("enc0", 2, c0, 27), ("enc1", c0, c1, 27), ("enc2", c1, c2, 27), ("enc3", c2, c3, 27),
            ("dec2", c3, c2, 27), ("dec1", c2, c1, 27), ("dec0", c1, c0, 27),
            ("head", c0, 3, 1), ("head3", c3, 3, 1)]


def param_count(ch):
    return sum(co * t * ci + co for _, ci, co, t in layers(ch))


def unpack(theta, ch):
    """Flat vector -> {name: (W[Cout][T][Cin], b[Cout])}."""
    out, o = {}, 0
    for name, ci, co, t in layers(ch):
        W = theta[o:o + co * t * ci].reshape(co, t, ci)
        o += co * t * ci
        out[name] = (W, theta[o:o + co])
        o += co
    assert o == theta.size
    return out


def pack(grads, ch):
    return np.concatenate([np.concatenate([grads[name][0].ravel(), grads[name][1].ravel()])
                           for name, _, _, _ in layers(ch)])


def round_bf16(x):
    """IEEE float32 -> bfloat16 (round to nearest even) -> float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(ch, seed):
    """He-scaled normal weights, zero biases; the two output maps start at
    zero, so the untrained network predicts v = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co, t in layers(ch):
        if name in ("head", "head3"):
            W = np.zeros((co, t, ci))
        else:
            W = rng.standard_normal((co, t, ci)) * np.sqrt(2.0 / (t * ci))
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts)


# ---- building blocks and their adjoints (arrays are [n1][n2][n3][C]) ----
def conv(x, W, b):
    """Periodic 3x3x3 (or 1x1x1) convolution: out[v] = sum_t W[:, t, :] x[v + off_t] + b."""
    T = W.shape[1]
    offs = TAPS if T == 27 else [(0, 0, 0)]
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, o in enumerate(offs):
        out += np.roll(x, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2)) @ W[:, t, :].T
    return out + b


def conv_adjoint(dz, x, W):
    """Adjoints of conv: (dx, dW, db) for upstream gradient dz."""
    T = W.shape[1]
    offs = TAPS if T == 27 else [(0, 0, 0)]
    dx = np.zeros(x.shape)
    dW = np.zeros(W.shape)
    dzf = dz.reshape(-1, dz.shape[-1])
    for t, o in enumerate(offs):
        xs = np.roll(x, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))
        dW[:, t, :] = dzf.T @ xs.reshape(-1, x.shape[-1])
        dx += np.roll(dz @ W[:, t, :], shift=(o[0], o[1], o[2]), axis=(0, 1, 2))
    return dx, dW, dzf.sum(axis=0)


def pool(x):
    n1, n2, n3, c = x.shape
    return x.reshape(n1 // 2, 2, n2 // 2, 2, n3 // 2, 2, c).mean(axis=(1, 3, 5))


def pool_adjoint(dy):
    return up(dy, 2) / 8.0


def up(x, f=2):
    return np.repeat(np.repeat(np.repeat(x, f, axis=0), f, axis=1), f, axis=2)


def up_adjoint(dy, f=2):
    n1, n2, n3, c = dy.shape
    return dy.reshape(n1 // f, f, n2 // f, f, n3 // f, f, c).sum(axis=(1, 3, 5))


def relu(z):
    return np.maximum(z, 0.0)


class Net:
    """Forward pass with the intermediates the backward pass needs."""

    def __init__(self, n, ch, sigma):
        self.n, self.ch, self.sigma = int(n), tuple(ch), float(sigma)
        self.g = core.Grid((self.n,) * 3)

    def forward(self, theta, mT, mR, bf16=False):
        r = round_bf16 if bf16 else (lambda a: a)
        P = {k: (r(W) if W.shape[1] == 27 else W, b)
             for k, (W, b) in unpack(np.asarray(theta, np.float64), self.ch).items()}
        c = {"x": r(np.stack([mT, mR], axis=-1))}
        c["e0"] = r(relu(conv(c["x"], *P["enc0"])))
        c["p0"] = r(pool(c["e0"]))
        c["e1"] = r(relu(conv(c["p0"], *P["enc1"])))
        c["p1"] = r(pool(c["e1"]))
        c["e2"] = r(relu(conv(c["p1"], *P["enc2"])))
        c["p2"] = r(pool(c["e2"]))
        c["e3"] = r(relu(conv(c["p2"], *P["enc3"])))
        c["u3"] = up(c["e3"])
        c["d2"] = r(relu(conv(c["u3"], *P["dec2"]) + c["e2"]))
        c["u2"] = up(c["d2"])
        c["d1"] = r(relu(conv(c["u2"], *P["dec1"]) + c["e1"]))
        c["u1"] = up(c["d1"])
        c["d0"] = r(relu(conv(c["u1"], *P["dec0"]) + c["e0"]))
        y = conv(c["d0"], *P["head"])
        h3 = conv(c["e3"], *P["head3"])
        s = np.stack([core.gauss_smooth(self.g, up(h3, 8)[..., k], self.sigma) for k in range(3)])
        w = np.moveaxis(y, -1, 0) + s
        v = core.apply_K(self.g, w, core.DIV_LERAY)
        c["P"] = P
        self.cache = c
        return v

    def loss(self, v, vt):
        N = float(self.n) ** 3
        return float(np.sum((v - vt) ** 2) / (2.0 * 3.0 * N))

    def backward(self, v, vt, bf16=False):
        """Gradient of the loss with respect to the flat parameter vector
        (after forward on the same inputs)."""
        r = round_bf16 if bf16 else (lambda a: a)
        c, P = self.cache, self.cache["P"]
        N = float(self.n) ** 3
        dv = (v - vt) / (3.0 * N)
        dw = core.apply_K(self.g, dv, core.DIV_LERAY)          # Leray is self-adjoint
        dy = np.moveaxis(dw, 0, -1)
        G = {}
        dd0, G["head"] = self._pointwise_adjoint(dy, c["d0"], P["head"])
        ds = np.stack([core.gauss_smooth(self.g, dw[k], self.sigma) for k in range(3)], axis=-1)
        dh3 = up_adjoint(ds, 8)
        de3, G["head3"] = self._pointwise_adjoint(dh3, c["e3"], P["head3"])
        # decoder: dz = upstream gradient masked by the layer's ReLU; the
        # convolution adjoints take it rounded, the skip paths unrounded
        dz = dd0 * (c["d0"] > 0)
        de0 = dz
        du1, *G["dec0"] = conv_adjoint(r(dz), c["u1"], P["dec0"][0])
        dz = up_adjoint(du1) * (c["d1"] > 0)
        de1 = dz
        du2, *G["dec1"] = conv_adjoint(r(dz), c["u2"], P["dec1"][0])
        dz = up_adjoint(du2) * (c["d2"] > 0)
        de2 = dz
        du3, *G["dec2"] = conv_adjoint(r(dz), c["u3"], P["dec2"][0])
        de3 = de3 + up_adjoint(du3)
        # encoder
        dz = de3 * (c["e3"] > 0)
        dp2, *G["enc3"] = conv_adjoint(r(dz), c["p2"], P["enc3"][0])
        dz = (de2 + pool_adjoint(dp2)) * (c["e2"] > 0)
        dp1, *G["enc2"] = conv_adjoint(r(dz), c["p1"], P["enc2"][0])
        dz = (de1 + pool_adjoint(dp1)) * (c["e1"] > 0)
        dp0, *G["enc1"] = conv_adjoint(r(dz), c["p0"], P["enc1"][0])
        dz = (de0 + pool_adjoint(dp0)) * (c["e0"] > 0)
        _, *G["enc0"] = conv_adjoint(r(dz), c["x"], P["enc0"][0])
        return pack({k: tuple(v) for k, v in G.items()}, self.ch)

    @staticmethod
    def _pointwise_adjoint(dy, x, Wb):
        W, _ = Wb
        dx, dW, db = conv_adjoint(dy, x, W)
        return dx, (dW, db)
