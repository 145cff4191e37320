"""Seeded random shapes for the general-size paths, bit-exact against the oracle:
Karatsuba levels over odd and unequal lengths, and unequal-length add/sub batches,
with random alignment and in-place use."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_21566_amd as bn
from conftest import announce

pytestmark = pytest.mark.gpu
D = bn.to_device
H = bn.to_host
MAX = 2 ** 64 - 1


def _rand(g, n):
    x = g.integers(0, MAX, n, dtype=np.uint64, endpoint=True)
    # runs of all-ones and zeros so that carries cross limbs and tiles
    for _ in range(max(1, n // 500)):
        s = int(g.integers(0, max(1, n)))
        x[s:s + int(g.integers(1, 300))] = MAX if g.integers(0, 2) else 0
    return x


def _log_size(g, lo, hi):
    return int(np.exp(g.uniform(np.log(lo), np.log(hi + 1))))


@pytest.mark.parametrize("seed", range(24))
def test_karatsuba_random_shapes(bnctx, seed):
    g = np.random.default_rng(1000 + seed)
    hi = _log_size(g, 1, 3000)
    lo = max(1, min(hi, _log_size(g, max(1, hi // 3), hi)))
    na, nb = (hi, lo) if g.integers(0, 2) else (lo, hi)
    npairs = int(g.integers(1, max(2, 6000 // max(na, nb)) + 1))
    levels = int(g.integers(0, 4))
    form = ("mad", "mfma", "auto")[seed % 3]
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    want = oracle.mul_batch(a, b, na, nb, npairs)
    announce("random karatsuba", seed, na, nb, npairs, levels, form)
    tr = torch.full(((na + nb) * npairs,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_karatsuba_batch(bnctx, tr, D(a), na, D(b), nb, npairs, levels, form)
    torch.cuda.synchronize()
    got = H(tr)
    assert (got == want).all(), f"na={na} nb={nb} npairs={npairs} levels={levels} {form}: " \
                                f"first bad limb {np.argmax(got != want)}"


@pytest.mark.parametrize("seed", range(12))
def test_unequal_addsub_random_shapes(bnctx, seed):
    g = np.random.default_rng(2000 + seed)
    na = _log_size(g, 1, 300000)
    nb = int(g.integers(0, na + 1))
    npairs = int(g.integers(1, max(2, 400000 // na) + 1))
    op = "add" if seed % 2 == 0 else "sub"
    offset = int(g.integers(0, 2))
    in_place = bool(g.integers(0, 2))
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    bext = np.zeros((npairs, na), np.uint64)
    bext[:, :nb] = b.reshape(npairs, nb)
    want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, bext.reshape(-1), na)
    announce("random unequal", seed, op, na, nb, npairs, offset, in_place)
    ta = D(np.concatenate([np.zeros(offset, np.uint64), a]))[offset:]
    tb = D(b) if nb else torch.zeros(1, dtype=torch.int64, device="cuda")
    tr = ta if in_place else torch.full((na * npairs + offset,), -1, dtype=torch.int64, device="cuda")[offset:]
    tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
    (bn.bn_add_unequal_n_batch if op == "add" else bn.bn_sub_unequal_n_batch)(bnctx, tr, ta, na, tb, nb, npairs, tc)
    torch.cuda.synchronize()
    got = H(tr)
    assert (got == want).all(), f"{op} na={na} nb={nb} npairs={npairs}: first bad limb {np.argmax(got != want)}"
    assert (H(tc) == wc).all()


@pytest.mark.parametrize("seed", range(16))
def test_addsub_random_forms(bnctx, seed):
    """Seeded random add/sub batches over the scan's forms: pair lengths from 1 to 3e5
    limbs, 8-byte or 16-byte alignment, in place or not, the deferred form forced or
    off, spin limits from 0 up; inputs with long propagate runs."""
    g = np.random.default_rng(3000 + seed)
    n = _log_size(g, 1, 300000)
    npairs = int(g.integers(1, max(2, 1200000 // n) + 1))
    op = ("add", "sub")[seed % 2]
    offset = int(g.integers(0, 2))
    in_place = ("none", "a", "b")[int(g.integers(0, 3))]
    defer = int(g.choice([0, 1, 64]))
    spin = int(g.choice([0, 4, 2048]))
    N = n * npairs
    a, b = _rand(g, N), _rand(g, N)
    if op == "sub":  # propagate runs for subtraction are equal limbs
        m = g.random(N) < 0.3
        b[m] = a[m]
    else:
        m = g.random(N) < 0.3
        b[m] = ~a[m]
    want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)
    announce("random add/sub form", seed, op, n, npairs, offset, in_place, defer, spin)
    old = (bn.bn_get_param(bnctx, "addsub.defer_tiles"), bn.bn_get_param(bnctx, "lookback.spin_limit"))
    try:
        bn.bn_set_param(bnctx, "addsub.defer_tiles", defer)
        bn.bn_set_param(bnctx, "lookback.spin_limit", spin)
        ta = D(np.concatenate([np.zeros(offset, np.uint64), a]))[offset:]
        tb = D(np.concatenate([np.zeros(offset, np.uint64), b]))[offset:]
        tr = {"a": ta, "b": tb}.get(in_place)
        if tr is None:
            tr = torch.full((N + offset,), -1, dtype=torch.int64, device="cuda")[offset:]
        tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
        (bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch)(bnctx, tr, ta, tb, n, npairs, tc)
        torch.cuda.synchronize()
        got = H(tr)
    finally:
        bn.bn_set_param(bnctx, "addsub.defer_tiles", old[0])
        bn.bn_set_param(bnctx, "lookback.spin_limit", old[1])
    assert (got == want).all(), f"{op} n={n} npairs={npairs}: first bad limb {np.argmax(got != want)}"
    assert (H(tc) == wc).all()


@pytest.mark.parametrize("seed", range(8))
def test_square_mfma_random(bnctx, seed):
    """Square MFMA products of random sizes and batch counts: the two operand
    conversions run as one two-part launch when the first ends on a tile boundary, as
    two launches otherwise."""
    g = np.random.default_rng(4000 + seed)
    n = int(g.choice([520, 777, 1024, 2048, 3001, 4096, 6000]))
    npairs = int(g.integers(1, 6))
    a, b = _rand(g, n * npairs), _rand(g, n * npairs)
    want = oracle.mul_batch(a, b, n, n, npairs)
    announce("random square mfma", seed, n, npairs)
    tr = torch.full((2 * n * npairs,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, tr, D(a), D(b), n, n, npairs, "mfma")
    torch.cuda.synchronize()
    got = H(tr)
    assert (got == want).all(), f"n={n} npairs={npairs}: first bad limb {np.argmax(got != want)}"


@pytest.mark.parametrize("seed", range(12))
def test_auto_form_class_boundaries(bnctx, seed):
    """The automatic form around its size classes: products whose length sits on either
    side of a class boundary (64/65, 128/129, 256/257, 512/513, 1024/1025 limbs) with a
    shorter operand just below, at and above the class's crossover, random batch counts
    and operand order, against the oracle (either form is exact; this checks the dispatch
    and the workspace each class picks)."""
    g = np.random.default_rng(5000 + seed)
    P = int(g.choice([64, 65, 128, 129, 256, 257, 512, 513, 1024, 1025]))
    cross = {64: 28, 128: 28, 256: 2, 512: 2, 1024: 40}[min(c for c in (64, 128, 256, 512, 1024) if c >= P)
                                                          if P <= 1024 else 1024]
    s = max(1, min(P // 2, cross + int(g.integers(-2, 3))))
    na, nb = (P - s, s) if g.integers(0, 2) else (s, P - s)
    npairs = int(g.integers(1, 40))
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    want = oracle.mul_batch(a, b, na, nb, npairs)
    announce("auto form class boundary", seed, na, nb, npairs)
    bn.bn_reserve_for(bnctx, bn.BN_OP_MUL, na, nb, npairs, "auto", 0)
    tr = torch.full(((na + nb) * npairs,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, tr, D(a), D(b), na, nb, npairs, "auto")
    torch.cuda.synchronize()
    got = H(tr)
    assert (got == want).all(), f"{na}x{nb} npairs={npairs}: first bad limb {np.argmax(got != want)}"
