"""Batched GN-Krylov solves of many registration pairs of uneven grid sizes on
one GPU.

Worker threads each own a HIP stream (default priority) and one context per
grid size; they take pairs from a shared queue, largest first, so solves of
different pairs overlap on the GPU (a 64^3 transport step fills only a
quarter of the compute units).  Every context replays its PCG matvec from a
captured HIP graph and picks its transport tile shape with the autotuner
after its first solve; neither changes a result bit, so a batched solve
returns exactly what solving the pairs one by one returns.

The uneven batch: 16 pairs at 64^3, 16 at 96^3, 12 at 128^3 and 4 at 160^3,
in that order.  Pair p has its phantom from seed 100 + 2p (periodic Voronoi,
120 seeds, Gaussian of 2 cells, rescaled to [0, 1]) and its velocity from
seed 101 + 2p (Gaussian-filtered white noise of physical width pi/4, Leray,
max |v| drawn from U[0.05, 0.2] 2 pi by a generator seeded with 7).
"""
import math
import queue
import threading
import time

import numpy as np
import torch

from . import mireg, synth

TWO_PI = 2.0 * math.pi
UNEVEN_BATCH = [64] * 16 + [96] * 16 + [128] * 12 + [160] * 4
SOLVER = dict(nt=4, order=3, reg=mireg.H1, div=mireg.DIV_NEAR, beta_v=5e-3, beta_w=1.0)


def make_pairs(sizes, device=None):
    """[(mT, mR)] on the device for grid sizes ``sizes`` (one int per pair)."""
    amp = np.random.default_rng(7).uniform(0.05, 0.2, len(sizes)) * TWO_PI
    prep = {}
    out = []
    for p, n in enumerate(sizes):
        if n not in prep:
            prep[n] = mireg.Context((n, n, n), dtype=torch.float32, device=device, **SOLVER)
        ctx = prep[n]
        raw = torch.from_numpy(synth.voronoi_phantom((n, n, n), nseeds=120, seed=100 + 2 * p)).float().to(ctx.device)
        mT = ctx.op("rescale01", ctx.op("gauss", raw, 2.0))
        noise = torch.from_numpy(synth.white_noise((n, n, n), seed=101 + 2 * p)).float().to(ctx.device)
        sm = torch.stack([ctx.op("gauss", noise[c].contiguous(), n / 8.0) for c in range(3)]).contiguous()
        v = ctx.op("scale_maxnorm", ctx.op("leray", sm), float(amp[p]))
        ctx.set_velocity(v)
        out.append((mT, ctx.op("transport_state", mT)))
    for c in prep.values():
        c.close()
    torch.cuda.synchronize()
    return out


class BatchSolver:
    """Solve lists of (mT, mR) pairs with `workers` concurrent streams."""

    def __init__(self, workers=4, graphs=True, autotune=True, device=None, **solver):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workers, self.graphs, self.tune = int(workers), bool(graphs), bool(autotune)
        self.solver = dict(SOLVER, **solver)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.workers)]
        self.ctxs = [dict() for _ in range(self.workers)]
        self.tuned = {}

    def _context(self, w, n):
        """Worker w's context for grid n, created on worker w's stream."""
        c = self.ctxs[w].get(n)
        if c is None:
            with torch.cuda.device(self.device), torch.cuda.stream(self.streams[w]):
                c = mireg.Context(n, dtype=torch.float32, device=self.device, **self.solver)
            c.set_graphs(self.graphs)
            self.ctxs[w][n] = c
        return c

    def solve(self, pairs, **gn_opts):
        """Returns [(v, report)] in the order of `pairs` and the wall time."""
        results = [None] * len(pairs)
        order = sorted(range(len(pairs)), key=lambda i: -pairs[i][0].numel())
        todo = queue.Queue()
        for i in order:
            todo.put(i)
        errors = []
        producer = torch.cuda.current_stream(self.device)
        # Every context exists before the workers start: creating one (device
        # allocations, uploads) while another worker captures its matvec graph
        # could invalidate that capture.
        for n in sorted({tuple(p[0].shape) for p in pairs}):
            for w in range(self.workers):
                self._context(w, n)

        def work(w):
            try:
                s = self.streams[w]
                s.wait_stream(producer)
                with torch.cuda.device(self.device), torch.cuda.stream(s):
                    while True:
                        try:
                            i = todo.get_nowait()
                        except queue.Empty:
                            return
                        mT, mR = pairs[i]
                        n = tuple(mT.shape)
                        ctx = self.ctxs[w][n]
                        ctx.set_images(mT, mR)
                        v, rep = ctx.gn_solve(**gn_opts)
                        if self.tune and (w, n) not in self.tuned:
                            self.tuned[(w, n)] = ctx.autotune(reps=2)
                        results[i] = (v, rep)
            except Exception as e:  # surfaced to the caller below
                errors.append(e)

        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        threads = [threading.Thread(target=work, args=(w,)) for w in range(self.workers)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        if errors:
            raise errors[0]
        return results, wall

    def close(self):
        for d in self.ctxs:
            for c in d.values():
                c.close()
        self.ctxs = [dict() for _ in range(self.workers)]
