"""Batched GN-Krylov solves of many registration pairs of uneven grid sizes on
one GPU.

Worker threads each own a HIP stream (default priority) and one context per
grid size; they take pairs from a shared queue, largest first, so solves of
different pairs overlap on the GPU (a 64^3 transport step fills only a
quarter of the compute units).  Every context replays its PCG matvec from a
captured HIP graph and picks its transport tile shape with the autotuner
after its first solve; neither changes a result bit, so a batched solve
returns exactly what solving the pairs one by one returns.

With `lockstep={n: g}` the pairs of grid n are solved in groups of g by
the lockstep batch (`mireg.Batch`: one transport launch per step and one
Krylov pass per grid size for the whole group), each group as one job of
a worker; other sizes keep one pair per job.  Small grids gain (a 64^3
launch is latency-bound, and a group of 8 still fits the 256 MB
last-level cache step by step); large ones lose, as every lockstep kernel
then streams the fields of all members and the next kernel finds none of
them cached.  Lockstep FP32 results agree with the single-pair ones to
rounding, not bit for bit.  With `autotune` a group's first context is tuned
after the group's first solve and its shape is given to the others.

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
    """Solve lists of (mT, mR) pairs with `workers` concurrent streams;
    `lockstep` ({grid points per axis: group size}) groups pairs of those
    sizes into lockstep batches."""

    def __init__(self, workers=4, graphs=True, autotune=True, device=None, lockstep=None, **solver):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workers, self.graphs, self.tune = int(workers), bool(graphs), bool(autotune)
        self.lockstep = {int(k): int(v) for k, v in (lockstep or {}).items() if int(v) > 1}
        self.solver = dict(SOLVER, **solver)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.workers)]
        self.ctxs = [dict() for _ in range(self.workers)]
        self.groups = [dict() for _ in range(self.workers)]
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

    def _group(self, w, n, g):
        """Worker w's lockstep batch of g contexts for grid n (its stream)."""
        key = (n, g)
        b = self.groups[w].get(key)
        if b is None:
            with torch.cuda.device(self.device), torch.cuda.stream(self.streams[w]):
                cs = [mireg.Context(n, dtype=torch.float32, device=self.device, **self.solver) for _ in range(g)]
            b = (cs, mireg.Batch(cs))
            self.groups[w][key] = b
        return b

    def _jobs(self, pairs):
        """Lists of pair indices, largest work first: same-size groups for
        the lockstep sizes, single pairs otherwise."""
        by_n = {}
        for i, p in enumerate(pairs):
            by_n.setdefault(tuple(p[0].shape), []).append(i)
        jobs = []
        for n, idx in by_n.items():
            g = self.lockstep.get(n[0], 1) if n[0] == n[1] == n[2] else 1
            jobs += [idx[k:k + g] for k in range(0, len(idx), g)]
        jobs.sort(key=lambda j: -sum(pairs[i][0].numel() for i in j))
        return jobs

    def solve(self, pairs, **gn_opts):
        """Returns [(v, report)] in the order of `pairs` and the wall time."""
        results = [None] * len(pairs)
        jobs = self._jobs(pairs)
        todo = queue.Queue()
        for j in jobs:
            todo.put(j)
        errors = []
        producer = torch.cuda.current_stream(self.device)
        # Every context exists before the workers start: creating one (device
        # allocations, uploads) while another worker captures its matvec graph
        # could invalidate that capture.
        for j in jobs:
            n = tuple(pairs[j[0]][0].shape)
            for w in range(self.workers):
                if len(j) > 1:
                    self._group(w, n, len(j))
                else:
                    self._context(w, n)

        def work(w):
            try:
                s = self.streams[w]
                s.wait_stream(producer)
                with torch.cuda.device(self.device), torch.cuda.stream(s):
                    while True:
                        try:
                            j = todo.get_nowait()
                        except queue.Empty:
                            return
                        n = tuple(pairs[j[0]][0].shape)
                        if len(j) > 1:
                            cs, B = self.groups[w][(n, len(j))]
                            for c, i in zip(cs, j):
                                c.set_images(*pairs[i])
                            vs, reps = B.gn_solve(**gn_opts)
                            for i, v, rep in zip(j, vs, reps):
                                results[i] = (v, rep)
                            if self.tune and (w, n, len(j)) not in self.tuned:
                                # one tuned shape for the whole group (a lockstep
                                # batch needs the same shape in every context)
                                self.tuned[(w, n, len(j))] = cs[0].autotune(reps=2)
                                for c in cs[1:]:
                                    c.set_tuning(*cs[0].tuning())
                            continue
                        i = j[0]
                        mT, mR = pairs[i]
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
        for d in self.groups:
            for cs, B in d.values():
                B.close()
                for c in cs:
                    c.close()
        for d in self.ctxs:
            for c in d.values():
                c.close()
        self.ctxs = [dict() for _ in range(self.workers)]
        self.groups = [dict() for _ in range(self.workers)]
