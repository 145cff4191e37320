"""The large MFMA kernel with 64 Toeplitz rows per column block (mul.mfma_rows = 1;
the default, 2, is what the other multiplication tests run) against the CPU oracle,
bit-exact: unsplit and split launches, staged rounds of several lengths,
pathological operands, and C5 (sampled pairs + residues)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_21566_amd as bn
from _bigint import to_int
from conftest import announce
from paper_2604_21566_amd import workloads as wl

pytestmark = pytest.mark.gpu
D = bn.to_device
H = bn.to_host
MAX = 2 ** 64 - 1


@pytest.fixture(scope="module")
def ctx1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bn.bn_create(0, auto_grow=True)
    bn.bn_set_param(c, "mul.mfma_rows", 1)
    yield c
    torch.cuda.synchronize()
    bn.bn_destroy(c)


def _check(ctx, a, b, na, nb, npairs):
    announce("mul mfma rows=1", f"na={na}", f"nb={nb}", f"npairs={npairs}")
    tr = torch.full((npairs * (na + nb),), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(ctx, tr, D(a), D(b), na, nb, npairs, "mfma")
    torch.cuda.synchronize()
    r = H(tr)
    rr = oracle.mul_batch(a, b, na, nb, npairs)
    bad = np.nonzero(r != rr)[0]
    assert bad.size == 0, f"na={na} nb={nb}: {bad.size} bad limbs, first at {bad[0]}"


SHAPES = [(129, 128), (300, 1), (1, 300), (257, 3), (3, 257), (256, 256), (200, 312), (511, 513), (1000, 24),
          (7, 1017), (1024, 1024), (1000, 999), (2047, 2049), (4099, 1031), (1031, 4099), (4096, 4096)]


@pytest.mark.parametrize("na,nb", SHAPES)
def test_random(ctx1, na, nb):
    g = np.random.default_rng(na * 31 + nb)
    npairs = 3
    _check(ctx1, g.integers(0, MAX, na * npairs, dtype=np.uint64, endpoint=True),
           g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True), na, nb, npairs)


@pytest.mark.parametrize("chunk", [0, 16, 50, 224, 234, 256])
@pytest.mark.parametrize("na,nb", [(1500, 1500), (3000, 700), (16384, 16384)])
def test_round_lengths(ctx1, chunk, na, nb):
    """Staged rounds of 16, 50, 224, 234 (the longest with three workgroups per CU) and
    256 steps (the last round ragged), and the by-size default (0), unsplit and split
    (one or two pairs leave too few workgroups, so the contraction is sliced)."""
    old = bn.bn_get_param(ctx1, "mul.mfma_chunk")
    bn.bn_set_param(ctx1, "mul.mfma_chunk", chunk)
    try:
        g = np.random.default_rng(chunk + na)
        npairs = 1 if na == 16384 else 2
        _check(ctx1, g.integers(0, MAX, na * npairs, dtype=np.uint64, endpoint=True),
               g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True), na, nb, npairs)
    finally:
        bn.bn_set_param(ctx1, "mul.mfma_chunk", old)


@pytest.mark.parametrize("n", [300, 480, 2048])
def test_pathological(ctx1, n):
    pa, pb = wl.pathological(n, 1, seed=n)
    _check(ctx1, pa.reshape(-1), pb.reshape(-1), n, n, pa.shape[0])


def test_c5_full(ctx1):
    """64 pairs x 16384 limbs: sampled pairs against the oracle, every pair by residues."""
    n, npairs = 16384, 64
    a, b = wl.c5()
    announce("mul mfma rows=1", "c5 full")
    tr = torch.full((npairs * 2 * n,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(ctx1, tr, D(a), D(b), n, n, npairs, "mfma")
    torch.cuda.synchronize()
    r = H(tr)
    for p in (0, 1, 2, 63):
        rr = oracle.mul(a[p * n:(p + 1) * n], b[p * n:(p + 1) * n])
        assert (r[p * 2 * n:(p + 1) * 2 * n] == rr).all(), f"pair {p}"
    for p in range(npairs):
        A, B = to_int(a[p * n:(p + 1) * n]), to_int(b[p * n:(p + 1) * n])
        R = to_int(r[p * 2 * n:(p + 1) * 2 * n])
        for q in (65537, 998244353, (1 << 61) - 1):
            assert (A % q) * (B % q) % q == R % q, f"pair {p} mod {q}"


def test_param_range(ctx1):
    for bad in (0, 3, 4):
        with pytest.raises(bn.BnError):
            bn.bn_set_param(ctx1, "mul.mfma_rows", bad)
    assert bn.bn_get_param(ctx1, "mul.mfma_rows") == 1
