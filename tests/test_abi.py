"""The C-ABI library loads and exports every function include/mireg.h and
include/mireg_net.h declare (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mireg.h")
NET_HEADER = os.path.join(ROOT, "include", "mireg_net.h")
LIB = os.path.join(ROOT, "paper_1808_04487_amd", "libmireg.so")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mireg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mireg_create", "mireg_destroy", "mireg_set_images", "mireg_set_velocity",
                     "mireg_objective", "mireg_gradient", "mireg_hessian_matvec",
                     "mireg_precond_apply", "mireg_pcg_solve", "mireg_gn_solve", "mireg_op",
                     "mireg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libmireg.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() + declared_functions(NET_HEADER) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_1808_04487_amd import mireg
    assert sorted(mireg.SIGNATURES) == declared_functions()


def test_network_binding_signatures_cover_its_header():
    from paper_1808_04487_amd import warmstart
    names = declared_functions(NET_HEADER)
    assert "mireg_net_train_step" in names and "mireg_net_forward" in names
    assert sorted(warmstart.SIGNATURES) == names


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching any device."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batch_jobs_group_lockstep_sizes():
    """The hybrid batch's job list (host logic, no GPU): pairs of a lockstep
    size come in groups of the stated size (the last one shorter), other
    sizes one pair per job, largest work first, every pair exactly once."""
    import types

    import torch

    from paper_1808_04487_amd import batch

    sizes = [64] * 11 + [96] * 3 + [128, 48, 64]
    pairs = [(torch.empty((n, n, n), dtype=torch.float32), None) for n in sizes]
    jobs = batch.BatchSolver._jobs(types.SimpleNamespace(lockstep={64: 4, 48: 2}), pairs)
    flat = sorted(i for j in jobs for i in j)
    assert flat == list(range(len(sizes)))
    for j in jobs:
        assert len({sizes[i] for i in j}) == 1
        assert len(j) == 1 or sizes[j[0]] == 64
    assert sorted(len(j) for j in jobs if sizes[j[0]] == 64) == [4, 4, 4]
    work = [sum(sizes[i] ** 3 for i in j) for j in jobs]
    assert work == sorted(work, reverse=True)
