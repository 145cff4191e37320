"""Karatsuba levels above the schoolbook kernels: bit-exact against the CPU oracle's
schoolbook product (the product is unique, so the recursion must reproduce it)."""
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


def _kmul(ctx, a, b, n, npairs, levels, form):
    announce("karatsuba", form, f"n={n}", f"npairs={npairs}", f"levels={levels}")
    tr = torch.full((2 * n * npairs,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_karatsuba_n_batch(ctx, tr, D(a), D(b), n, npairs, levels, form)
    torch.cuda.synchronize()
    return H(tr)


def _check(ctx, a, b, n, npairs, levels, form):
    r = _kmul(ctx, a, b, n, npairs, levels, form)
    rr = oracle.mul_batch(a, b, n, n, npairs)
    bad = np.nonzero(r != rr)[0]
    assert bad.size == 0, f"{form} n={n} levels={levels}: {bad.size} bad limbs, first at {bad[0]}"


SHAPES = [(2, 3, 1), (8, 5, 1), (8, 3, 3), (64, 7, 2), (96, 4, 5), (256, 4, 1), (1024, 3, 2), (2048, 2, 3),
          (4096, 2, 1), (640, 9, 4)]


@pytest.mark.parametrize("form", ["auto", "mad", "mfma"])
@pytest.mark.parametrize("n,npairs,levels", SHAPES)
def test_random(bnctx, form, n, npairs, levels):
    g = np.random.default_rng(n * 31 + levels)
    a = g.integers(0, MAX, n * npairs, dtype=np.uint64, endpoint=True)
    b = g.integers(0, MAX, n * npairs, dtype=np.uint64, endpoint=True)
    _check(bnctx, a, b, n, npairs, levels, form)


def _halves(lo, hi):
    return np.concatenate([lo, hi])


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_signs_and_carries(bnctx, form, levels):
    """Every sign pattern of the differences (A_H >, =, < A_L and the same for B),
    all-ones operands (the largest carries in the combine), zeros, and the
    pathological patterns."""
    n = 64
    g = np.random.default_rng(levels)
    ones = np.full(n // 2, MAX, np.uint64)
    zero = np.zeros(n // 2, np.uint64)
    rnd = lambda: g.integers(0, MAX, n // 2, dtype=np.uint64, endpoint=True)
    x = rnd()
    y = x.copy()
    y[-1] ^= np.uint64(1)  # differs in the top limb only
    halves = [_halves(x, x), _halves(x, y), _halves(y, x), _halves(ones, ones), _halves(zero, ones),
              _halves(ones, zero), _halves(zero, zero), _halves(rnd(), rnd())]
    A = np.concatenate([h for h in halves for _ in halves])
    B = np.concatenate([h for _ in halves for h in halves])
    npairs = len(halves) ** 2
    _check(bnctx, A, B, n, npairs, levels, form)
    pa, pb = wl.pathological(n, 1, seed=levels)
    _check(bnctx, pa.reshape(-1), pb.reshape(-1), n, pa.shape[0], levels, form)


@pytest.mark.parametrize("n,min_half,levels", [(2048, 4096, 0), (4096, 2048, 1), (12000, 1000, 3)])
def test_auto_levels(bnctx, n, min_half, levels):
    """levels = BN_KARATSUBA_AUTO splits while the halves keep mul.karatsuba_limbs limbs:
    the same product as the schoolbook oracle, and the level count the rule gives."""
    assert bn.bn_karatsuba_auto_levels(n, min_half) == levels
    old = bn.bn_get_param(bnctx, "mul.karatsuba_limbs")
    bn.bn_set_param(bnctx, "mul.karatsuba_limbs", min_half)
    try:
        g = np.random.default_rng(n + levels)
        a = g.integers(0, MAX, n * 2, dtype=np.uint64, endpoint=True)
        b = g.integers(0, MAX, n * 2, dtype=np.uint64, endpoint=True)
        _check(bnctx, a, b, n, 2, bn.BN_KARATSUBA_AUTO, "mfma")
    finally:
        bn.bn_set_param(bnctx, "mul.karatsuba_limbs", old)


@pytest.mark.parametrize("n", [12288, 12000])
def test_sign_pieces(bnctx, n):
    """Halves that differ in one limb only, at the ends and the boundaries of the
    2048-limb pieces the split's sign pass works in (k = n/2 = 6144: three whole
    pieces; 6000: a ragged last piece), in both directions: the sign must come from
    the highest differing piece whatever the pieces above it hold (equal limbs)."""
    k = n // 2
    g = np.random.default_rng(n)
    positions = [0, 5, 2047, 2048, 4095, 4096, k - 1]
    A, B = [], []
    for idx, pos in enumerate(positions):
        lo = g.integers(1, MAX - 1, k, dtype=np.uint64, endpoint=True)
        hi = lo.copy()
        hi[pos] += np.uint64(1) if idx % 2 == 0 else np.uint64(0)
        hi[pos] -= np.uint64(0) if idx % 2 == 0 else np.uint64(1)
        A.append(np.concatenate([lo, hi]))
        # b: the opposite direction at another piece boundary
        lo2 = g.integers(1, MAX - 1, k, dtype=np.uint64, endpoint=True)
        hi2 = lo2.copy()
        p2 = positions[(idx + 3) % len(positions)]
        hi2[p2] += np.uint64(0) if idx % 2 == 0 else np.uint64(1)
        hi2[p2] -= np.uint64(1) if idx % 2 == 0 else np.uint64(0)
        B.append(np.concatenate([lo2, hi2]))
    a, b = np.concatenate(A), np.concatenate(B)
    for levels in (1, 2):
        _check(bnctx, a, b, n, len(positions), levels, "mfma")


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_c5_full(bnctx, c5_oracle, levels):
    """64 pairs x 16384 limbs (incl. all-ones x all-ones and zero x zero): every limb of
    every product against the oracle; residues as an extra check."""
    n, npairs = 16384, 64
    a, b, want = c5_oracle
    announce("C5 full, Karatsuba", f"levels={levels}")
    r = _kmul(bnctx, a, b, n, npairs, levels, "mfma")
    bad = np.flatnonzero(r != want)
    assert bad.size == 0, f"{bad.size} limbs differ, first at pair {bad[0] // (2 * n)} limb {bad[0] % (2 * n)}"
    for p in range(npairs):
        A = to_int(a[p * n:(p + 1) * n])
        B = to_int(b[p * n:(p + 1) * n])
        R = to_int(r[p * 2 * n:(p + 1) * 2 * n])
        for q in (65537, 998244353, (1 << 61) - 1):
            assert (A % q) * (B % q) % q == R % q, f"pair {p} mod {q}"


def test_errors(bnctx):
    ta = torch.zeros(96, dtype=torch.int64, device="cuda")
    tr = torch.zeros(192, dtype=torch.int64, device="cuda")
    with pytest.raises(bn.BnError) as e:
        bn.bn_mul_karatsuba_n_batch(bnctx, tr, ta, ta, 96, 1, 9)  # more levels than allowed
    assert e.value.status == bn.BN_EINVAL
    # empty batch and n = 0 are no-ops
    bn.bn_mul_karatsuba_n_batch(bnctx, tr, ta, ta, 96, 0, 2)
    bn.bn_mul_karatsuba_n_batch(bnctx, tr, ta, ta, 0, 3, 2)


def _kmul_general(ctx, a, na, b, nb, npairs, levels, form, in_place=False):
    announce("karatsuba general", form, f"na={na}", f"nb={nb}", f"npairs={npairs}", f"levels={levels}",
             f"in_place={in_place}")
    if in_place:   # r over a, with room for the products
        buf = torch.zeros(max(na * npairs, (na + nb) * npairs), dtype=torch.int64, device="cuda")
        buf[:na * npairs].copy_(D(a))
        bn.bn_mul_karatsuba_batch(ctx, buf[:(na + nb) * npairs], buf[:na * npairs], na, D(b), nb, npairs, levels,
                                  form)
        torch.cuda.synchronize()
        return H(buf[:(na + nb) * npairs])
    tr = torch.full(((na + nb) * npairs,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_karatsuba_batch(ctx, tr, D(a), na, D(b), nb, npairs, levels, form)
    torch.cuda.synchronize()
    return H(tr)


GENERAL = [(3, 3, 4, 1), (5, 5, 3, 2), (7, 7, 2, 2), (97, 97, 3, 2), (1001, 1001, 2, 3), (4097, 4097, 2, 2),
           (100, 60, 5, 2), (60, 100, 5, 1), (1000, 999, 3, 3), (513, 257, 4, 2), (10, 100, 3, 2),
           (2049, 2048, 2, 3), (12001, 12000, 1, 3), (333, 1, 6, 1), (1, 9, 2, 2)]


@pytest.mark.parametrize("form", ["auto", "mad", "mfma"])
@pytest.mark.parametrize("na,nb,npairs,levels", GENERAL)
def test_odd_and_unequal_sizes(bnctx, form, na, nb, npairs, levels):
    """Odd lengths (high halves zero-extended at every level) and unequal lengths (both
    operands zero-extended to the longer at the top, product of exactly na + nb limbs),
    bit-exact against the oracle's schoolbook product."""
    g = np.random.default_rng(na * 7 + nb * 13 + levels)
    a = g.integers(0, MAX, na * npairs, dtype=np.uint64, endpoint=True)
    b = g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True)
    a[:na] = MAX   # pair 0: all-ones operands (the largest carries in the combines)
    b[:nb] = MAX
    want = oracle.mul_batch(a, b, na, nb, npairs)
    r = _kmul_general(bnctx, a, na, b, nb, npairs, levels, form)
    bad = np.flatnonzero(r != want)
    assert bad.size == 0, f"{bad.size} bad limbs, first at {bad[0]}"
    if form == "mfma":
        r = _kmul_general(bnctx, a, na, b, nb, npairs, levels, form, in_place=True)
        assert (r == want).all(), "in place"


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_odd_split_signs(bnctx, levels):
    """m = 65: the high half (32 limbs) is zero-extended to 33, so it can equal, exceed or
    fall below the low half only through the low half's top limb; every pairing of those
    cases on a and b, through one to three levels."""
    n, k = 65, 33
    g = np.random.default_rng(levels)
    rnd = lambda m: g.integers(0, MAX, m, dtype=np.uint64, endpoint=True)
    ops = []
    lo = rnd(k)
    lo[k - 1] = 0
    ops.append(np.concatenate([lo, lo[:k - 1]]))                 # halves equal
    lo2 = lo.copy()
    lo2[k - 1] = 1
    ops.append(np.concatenate([lo2, lo2[:k - 1]]))               # high below low (top limb)
    hi = lo[:k - 1].copy()
    hi[-1] += np.uint64(1)
    ops.append(np.concatenate([lo, hi]))                         # high above low
    ops.append(np.full(n, MAX, np.uint64))                       # all ones
    ops.append(np.zeros(n, np.uint64))
    A = np.concatenate([x for x in ops for _ in ops])
    B = np.concatenate([y for _ in ops for y in ops])
    npairs = len(ops) ** 2
    want = oracle.mul_batch(A, B, n, n, npairs)
    for form in ("mad", "mfma"):
        r = _kmul_general(bnctx, A, n, B, n, npairs, levels, form)
        assert (r == want).all(), f"{form}: first bad limb {np.argmax(r != want)}"


def test_auto_levels_unequal(bnctx):
    """BN_KARATSUBA_AUTO: lengths within a factor of two recurse on the longer one's level
    count; lengths further apart take the schoolbook kernels (levels 0)."""
    old = bn.bn_get_param(bnctx, "mul.karatsuba_limbs")
    bn.bn_set_param(bnctx, "mul.karatsuba_limbs", 500)
    try:
        g = np.random.default_rng(9)
        for na, nb in ((3000, 2001), (3000, 1400), (1401, 3001)):
            a = g.integers(0, MAX, na * 2, dtype=np.uint64, endpoint=True)
            b = g.integers(0, MAX, nb * 2, dtype=np.uint64, endpoint=True)
            r = _kmul_general(bnctx, a, na, b, nb, 2, bn.BN_KARATSUBA_AUTO, "mfma")
            assert (r == oracle.mul_batch(a, b, na, nb, 2)).all(), (na, nb)
    finally:
        bn.bn_set_param(bnctx, "mul.karatsuba_limbs", old)


@pytest.mark.parametrize("na,nb,npairs,levels", [(4096, 4096, 2, 2), (1001, 777, 3, 1), (97, 97, 5, 3)])
def test_unaligned_output(bnctx, na, nb, npairs, levels):
    """An output 8-byte but not 16-byte aligned: the combine scan's 8-byte kernels."""
    g = np.random.default_rng(na + 3 * levels)
    a = g.integers(0, MAX, na * npairs, dtype=np.uint64, endpoint=True)
    b = g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True)
    a[:na] = MAX
    announce("karatsuba unaligned output", f"na={na}", f"nb={nb}", f"npairs={npairs}", f"levels={levels}")
    P = (na + nb) * npairs
    tr = torch.full((P + 1,), -1, dtype=torch.int64, device="cuda")[1:]
    bn.bn_mul_karatsuba_batch(bnctx, tr, D(a), na, D(b), nb, npairs, levels, "mfma")
    torch.cuda.synchronize()
    want = oracle.mul_batch(a, b, na, nb, npairs)
    got = H(tr)
    assert (got == want).all(), f"first bad limb {np.argmax(got != want)}"
