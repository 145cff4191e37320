"""Maximum sizes, checked without moving the operands to the host: add/sub over more
than 2^32 limbs (64-bit tile and limb indices, 2^20 chained tiles) by closed forms
and the (a + b) - b = a round trip, and one 2^20 x 2^20-limb product on both forms
(the MFMA form split into ~65 contraction slices) by closed forms, by residues and
by its low limbs, which depend only on the operands' low limbs."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_21566_amd as bn
from _bigint import to_int
from conftest import announce

pytestmark = pytest.mark.gpu
H = bn.to_host
GIB = 1 << 30


def _need_free(nbytes):
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / GIB:.0f} GiB of free device memory, {free / GIB:.0f} GiB free")


@pytest.fixture
def release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


N_BIG = (1 << 32) + 3


def test_add_sub_closed_forms_beyond_2p32_limbs(bnctx, release):
    """(2^(64N) - 1) + 1 = 0 with carry 1 (the carry crosses every limb), and
    2^(64(N-1)) - 1 = N-1 limbs of all-ones with borrow 0."""
    _need_free(3 * 8 * N_BIG + 8 * GIB)
    announce("max size add/sub closed forms", f"n={N_BIG}")
    a = torch.full((N_BIG,), -1, dtype=torch.int64, device="cuda")
    b = torch.zeros(N_BIG, dtype=torch.int64, device="cuda")
    b[0] = 1
    r = torch.full((N_BIG,), 7, dtype=torch.int64, device="cuda")
    c = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    bn.bn_add(bnctx, r, a, b, c)
    torch.cuda.synchronize()
    assert int(c[0]) == 1
    assert not bool(r.any())
    a.zero_()
    a[-1] = 1
    bn.bn_sub(bnctx, r, a, b, c)
    torch.cuda.synchronize()
    assert int(c[0]) == 0
    assert int(r[-1]) == 0 and bool((r[:-1] == -1).all())


def test_add_sub_round_trip_beyond_2p32_limbs(bnctx, release):
    """Random a, b of 2^32 + 3 limbs: r = a + b, then r - b (in place) = a with the
    same carry and borrow."""
    _need_free(3 * 8 * N_BIG + 12 * GIB)
    announce("max size add/sub round trip", f"n={N_BIG}")
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    a = torch.randint(-2 ** 63, 2 ** 63 - 1, (N_BIG,), dtype=torch.int64, device="cuda", generator=g)
    b = torch.randint(-2 ** 63, 2 ** 63 - 1, (N_BIG,), dtype=torch.int64, device="cuda", generator=g)
    r = torch.empty_like(a)
    c1 = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    c2 = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    bn.bn_add(bnctx, r, a, b, c1)
    bn.bn_sub(bnctx, r, r, b, c2)
    torch.cuda.synchronize()
    assert int(c1[0]) == int(c2[0]) in (0, 1)
    assert torch.equal(r, a)
    # the low limbs against the oracle (no carry enters limb 0)
    k = 4096
    rr, _ = oracle.add(H(a[:k]), H(b[:k]))
    bn.bn_add(bnctx, r, a, b, c1)
    torch.cuda.synchronize()
    assert (H(r[:k]) == rr).all()


N_MUL = 1 << 20


@pytest.mark.parametrize("form", ["mfma", "mad"])
def test_product_closed_forms_max_size(bnctx, release, form):
    """(2^(64n) - 1)^2 = X^(2n) - 2 X^n + 1 and 0 x 0 = 0 for n = 2^20 limbs."""
    _need_free(24 * GIB)
    n = N_MUL
    announce("max size product closed forms", form, f"n={n}")
    a = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    r = torch.full((2 * n,), 7, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, r, a, a.clone(), n, n, 1, form)
    torch.cuda.synchronize()
    assert int(r[0]) == 1 and not bool(r[1:n].any())
    assert int(r[n]) == -2 and bool((r[n + 1:] == -1).all())
    z = torch.zeros(n, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, r, z, z.clone(), n, n, 1, form)
    torch.cuda.synchronize()
    assert not bool(r.any())


@pytest.mark.parametrize("form", ["mfma", "mad"])
@pytest.mark.parametrize("kind", ["random", "most_negative_digits"])
def test_product_random_max_size(bnctx, release, form, kind):
    """2^20 x 2^20 limbs, random or the square of 0x7f...7f80 (every balanced digit
    -128: each digit product is +2^14, column sums up to 2^37): residues modulo three
    primes and 2^64 - 1, and the low 256 limbs against the oracle's product of the
    low 256 limbs."""
    _need_free(24 * GIB)
    n = N_MUL
    announce("max size product", kind, form, f"n={n}")
    g = np.random.default_rng(11)
    if kind == "random":
        ah = g.integers(0, 2 ** 64 - 1, n, dtype=np.uint64, endpoint=True)
        bh = g.integers(0, 2 ** 64 - 1, n, dtype=np.uint64, endpoint=True)
    else:
        ah = np.full(n, 0x7F7F7F7F7F7F7F7F, np.uint64)
        ah[0] = 0x7F7F7F7F7F7F7F80
        bh = ah.copy()
    r = torch.full((2 * n,), 7, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, r, bn.to_device(ah), bn.to_device(bh), n, n, 1, form)
    torch.cuda.synchronize()
    rh = H(r)
    k = 256
    assert (rh[:k] == oracle.mul(ah[:k], bh[:k])[:k]).all()
    A, B, R = to_int(ah), to_int(bh), to_int(rh)
    for q in (998244353, (1 << 61) - 1, (1 << 64) - 1, 1000000007):
        assert (A % q) * (B % q) % q == R % q, q
