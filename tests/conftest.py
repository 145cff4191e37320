import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def bnctx():
    """A library context on cuda:0 (GPU tests only).  Its compute calls grow the
    workspace as they need it ("workspace.auto_grow"); tests/test_gpu_workspace.py
    runs every compute entry point on contexts without it."""
    import torch
    import paper_2604_21566_amd as bn
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = bn.bn_create(0, auto_grow=True)
    yield ctx
    torch.cuda.synchronize()
    bn.bn_destroy(ctx)


@pytest.fixture(scope="session")
def c5_oracle():
    """The full 64 x 16384-limb product batch (a, b, products) from the oracle, computed
    once per session, pairs spread over host threads (the ctypes call releases the GIL)."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    from paper_2604_21566_amd import workloads as wl
    n, npairs = 16384, 64
    a, b = wl.c5()
    oracle._load()
    r = np.empty(2 * n * npairs, np.uint64)

    def one(p):
        r[p * 2 * n:(p + 1) * 2 * n] = oracle.mul(a[p * n:(p + 1) * n], b[p * n:(p + 1) * n])

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(one, range(npairs)))
    return a, b, r


def announce(*parts):
    """Name the case on stdout before a GPU step (flushed, so a crash still shows it)."""
    import sys
    sys.stdout.write("[case] " + " ".join(str(p) for p in parts) + "\n")
    sys.stdout.flush()
