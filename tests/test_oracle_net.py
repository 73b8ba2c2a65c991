"""Pins for the warm-start network oracle (oracle/net.py): the convolution
against its definition written as loops, every adjoint by the dot-product
test, the whole backward pass against central finite differences, the
initial network's zero output, the divergence-free output, and the BF16
rounding model against torch's conversion."""
import numpy as np
import pytest
import torch

from oracle import core, net

CH = (8, 8, 8, 8)


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_loops():
    n, ci, co = 4, 2, 3
    x = rand((n, n, n, ci), 1)
    W = rand((co, 27, ci), 2)
    b = rand(co, 3)
    out = net.conv(x, W, b)
    ref = np.zeros((n, n, n, co))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for t, (a, bb, c) in enumerate(net.TAPS):
                    ref[i, j, k] += W[:, t, :] @ x[(i + a) % n, (j + bb) % n, (k + c) % n]
                ref[i, j, k] += b
    assert np.abs(out - ref).max() < 1e-12


@pytest.mark.parametrize("taps", [27, 1])
def test_conv_adjoint_dot_products(taps):
    n, ci, co = 4, 3, 5
    x = rand((n, n, n, ci), 4)
    W = rand((co, taps, ci), 5)
    dz = rand((n, n, n, co), 6)
    dx, dW, db = net.conv_adjoint(dz, x, W)
    zero = np.zeros(co)
    # linear in x and in W: <dz, C(x)> = <dx, x> = <dW, W>
    lhs = np.sum(dz * net.conv(x, W, zero))
    assert abs(lhs - np.sum(dx * x)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(dW * W)) < 1e-10 * abs(lhs)
    assert np.allclose(db, dz.reshape(-1, co).sum(0))


def test_pool_and_upsample_adjoints():
    x = rand((8, 8, 8, 3), 7)
    y = rand((4, 4, 4, 3), 8)
    assert abs(np.sum(net.pool(x) * y) - np.sum(x * net.pool_adjoint(y))) < 1e-12
    assert abs(np.sum(net.up(y) * x) - np.sum(y * net.up_adjoint(x))) < 1e-12
    z = rand((1, 1, 1, 3), 9)
    assert abs(np.sum(net.up(z, 8) * x) - np.sum(z * net.up_adjoint(x, 8))) < 1e-12
    # mean of a constant and nearest upsampling of a constant
    assert np.allclose(net.pool(np.ones((4, 4, 4, 1))), 1.0)
    assert np.allclose(net.up(np.full((2, 2, 2, 1), 3.0)), 3.0)


def problem(n=16, seed=11):
    rng = np.random.default_rng(seed)
    theta = net.init_params(CH, seed)
    theta += 0.05 * rng.standard_normal(theta.size)   # the output maps must be non-zero
    mT, mR = rng.random((n,) * 3), rng.random((n,) * 3)
    vt = 0.1 * rng.standard_normal((3,) + (n,) * 3)
    return net.Net(n, CH, 2.0), theta, mT, mR, vt


def test_backward_matches_finite_differences():
    N, theta, mT, mR, vt = problem()
    v = N.forward(theta, mT, mR)
    g = N.backward(v, vt)
    # one index in the weights and one in the bias of every layer
    idx, o = [], 0
    for name, ci, co, t in net.layers(CH):
        idx += [o + (co * t * ci) // 2, o + co * t * ci + co - 1]
        o += co * t * ci + co
    h = 1e-5
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (N.loss(N.forward(theta + e, mT, mR), vt) - N.loss(N.forward(theta - e, mT, mR), vt)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g).max() + 1e-6 * abs(fd), (i, fd, g[i])


def test_initial_network_predicts_zero_and_output_is_divergence_free():
    N, theta, mT, mR, _ = problem()
    v0 = N.forward(net.init_params(CH, 3), mT, mR)
    assert np.abs(v0).max() == 0.0
    v = N.forward(theta, mT, mR)
    assert np.abs(v).max() > 1e-3
    assert np.abs(core.div(N.g, v)).max() < 1e-10 * np.abs(v).max()


def test_round_bf16_matches_torch_and_ties_to_even():
    x = np.random.default_rng(12).standard_normal(100000) * 10.0 ** np.random.default_rng(13).integers(-8, 8, 100000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(net.round_bf16(x), ref)
    one = 1.0
    u = 2.0 ** -7  # bfloat16 spacing in [1, 2)
    assert net.round_bf16(np.array([one + u / 2]))[0] == one
    assert net.round_bf16(np.array([one + 1.5 * u]))[0] == one + 2 * u


def test_bf16_model_stays_close_to_fp64():
    N, theta, mT, mR, vt = problem()
    v = N.forward(theta, mT, mR)
    g = N.backward(v, vt)
    v16 = N.forward(theta, mT, mR, bf16=True)
    g16 = N.backward(v16, vt, bf16=True)
    assert np.linalg.norm(v16 - v) < 3e-2 * np.linalg.norm(v)
    assert np.linalg.norm(g16 - g) < 5e-2 * np.linalg.norm(g)
