"""What the trained warm start gains over the plain method: on held-out
pairs (seeds never used in training or in the recorded evaluation), solves
from the network's prediction reach the same absolute gradient tolerance as
solves from v = 0 with fewer GN iterations, fewer Hessian matvecs and less
wall time, at no worse relative mismatch."""
import os

import numpy as np
import pytest
import torch

from paper_1808_04487_amd import mireg, warmstart

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(warmstart.WEIGHTS_DIR, "warmstart_128.npz")


def test_trained_warm_start_beats_zero_init():
    need_gpu()
    net = warmstart.WarmStartNet.load(WEIGHTS)
    assert net.n == 128 and net.channels == warmstart.CHANNELS
    ctx = warmstart.registration_context(128)
    # one untimed pair warms up both paths
    mT, mR, _, _, _ = warmstart.make_pair(net, ctx, 2000000, solve=False)
    warmstart.solve_pair(ctx, mT, mR, net)
    rows = []
    for s in range(2000001, 2000013):
        mT, mR, _, _, _ = warmstart.make_pair(net, ctx, s, solve=False)
        r = warmstart.solve_pair(ctx, mT, mR, net)
        (p, tp), (w, tw, used) = r["plain"], r["warm"]
        print("seed %d plain %d GN %d mv %.1f ms %.4f | warm %d GN %d mv %.1f ms %.4f used=%s" % (
            s, p["gn_iters"], p["matvecs"], 1e3 * tp, p["mismatch_rel"], w["gn_iters"], w["matvecs"], 1e3 * tw,
            w["mismatch_rel"], used), flush=True)
        assert w["status"] in (mireg.CONVERGED_ABS, mireg.CONVERGED_REL)
        rows.append((p["gn_iters"], w["gn_iters"], p["matvecs"], w["matvecs"], tp, tw, p["mismatch_rel"],
                     w["mismatch_rel"], used))
    a = np.array(rows, dtype=np.float64)
    assert a[:, 8].all()                          # the prediction was always used
    assert a[:, 1].mean() < a[:, 0].mean() - 1.0  # at least one GN iteration fewer on average
    assert a[:, 3].sum() < 0.7 * a[:, 2].sum()    # 30% fewer matvecs
    assert a[:, 5].sum() < 0.85 * a[:, 4].sum()   # 15% less wall time
    assert np.median(a[:, 7] / a[:, 6]) <= 1.05   # mismatch no worse


@pytest.mark.timeout(600)
def test_trained_network_at_128_matches_oracle():
    """The production configuration: trained weights on a phantom pair at
    128^3 (block-tiled convolutions on the two finest levels), against the
    oracle's BF16 storage model and plain FP64.  A trained network is far
    less sensitive to BF16 rounding ties than a randomly initialised one, so
    the model bound of the smaller parity cases holds here."""
    need_gpu()
    from oracle import net as onet

    net = warmstart.WarmStartNet.load(WEIGHTS)
    theta = net.get_params().astype(np.float64)
    ctx = warmstart.registration_context(128)
    mT, mR, _, _, _ = warmstart.make_pair(net, ctx, 3000001, solve=False)
    v = net.forward(mT, mR).double().cpu().numpy()
    ctx.close()
    O = onet.Net(128, net.channels, net.skip_sigma)
    a, b = mT.cpu().numpy(), mR.cpu().numpy()
    print("oracle forward at 128^3 (BF16 model, then FP64)", flush=True)
    v16 = O.forward(theta, a, b, bf16=True)
    v64 = O.forward(theta, a, b)
    e16 = np.linalg.norm(v - v16) / np.linalg.norm(v16)
    e64 = np.linalg.norm(v - v64) / np.linalg.norm(v64)
    print("trained network 128^3: vs BF16 model %.2e, vs FP64 %.2e" % (e16, e64), flush=True)
    assert e16 < 2e-3 and e64 < 3e-2
