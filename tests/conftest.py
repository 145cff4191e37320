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
    """A library context on cuda:0 (GPU tests only)."""
    import torch
    import paper_2604_21566_amd as bn
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = bn.bn_create(0)
    yield ctx
    torch.cuda.synchronize()
    bn.bn_destroy(ctx)


def announce(*parts):
    """Name the case on stdout before a GPU step (flushed, so a crash still shows it)."""
    import sys
    sys.stdout.write("[case] " + " ".join(str(p) for p in parts) + "\n")
    sys.stdout.flush()
