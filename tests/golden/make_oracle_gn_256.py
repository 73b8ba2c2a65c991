"""Writes oracle_gn_256.json: the oracle's FP64 GN-Krylov solve of the 256^3
benchmark workload (inputs rounded to FP32 exactly as the GPU tests prepare
them), with its per-iteration objective and gradient norm.  Calls only the
oracle; takes about half an hour on 8 host cores.

  python tests/golden/make_oracle_gn_256.py
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import core, prep, solver  # noqa: E402
from paper_1808_04487_amd import synth  # noqa: E402


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def main():
    n = (256, 256, 256)
    g = core.Grid(n)
    t0 = time.perf_counter()
    mT = f32(prep.smooth_rescale(g, synth.voronoi_phantom(n, nseeds=120, seed=1), 2.0))
    v = f32(prep.smooth_velocity(g, synth.white_noise(n, seed=2), math.pi / 4, 0.15 * 2 * math.pi))
    mR = f32(prep.transport(g, mT, v))
    p = core.Params(n, nt=4, order=3, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=5e-3, beta_w=1.0)
    R = core.Registration(p, mT, mR)
    print("inputs %.1f s" % (time.perf_counter() - t0), flush=True)
    _, rep = solver.gn_solve(R, np.zeros((3,) + n), grad_rtol=5e-2, grad_atol=1e-6, max_gn=50, max_pcg=100)
    out = rep.as_dict()
    out["history"] = rep.history
    out["recipe"] = ("256^3 Voronoi phantom (120 seeds, seed 1), Gaussian sigma 2 cells, rescaled to [0, 1]; "
                     "velocity from white noise seed 2, Gaussian of physical width pi/4, Leray, max |v| 0.15 2 pi; "
                     "mR = mT transported (nt 4, tricubic); mT, v and mR rounded to FP32; H1-div beta_v 5e-3 "
                     "beta_w 1, spectral preconditioner, relative gradient 5e-2, from v = 0")
    with open(os.path.join(HERE, "oracle_gn_256.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
