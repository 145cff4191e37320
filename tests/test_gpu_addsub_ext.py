"""Add/sub with carry-in, unequal lengths and |a - b| against the CPU oracle,
bit-exact, through the C ABI."""
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
    return g.integers(0, MAX, n, dtype=np.uint64, endpoint=True)


def _operands(g, n, npairs):
    """Random pairs, with every third pair all-ones + zero so that a carry-in runs
    through the whole pair (and across workgroup tiles when n is large)."""
    a, b = _rand(g, n * npairs).reshape(npairs, n), _rand(g, n * npairs).reshape(npairs, n)
    a[::3] = MAX
    b[::3] = 0
    return a.reshape(-1), b.reshape(-1)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n,npairs", [(1, 1000), (4, 1088), (3, 257), (64, 4096), (129, 33), (5000, 7),
                                      (100003, 3)])
def test_carry_in_batches(bnctx, op, n, npairs):
    announce("carry-in", op, f"n={n}", f"npairs={npairs}")
    g = np.random.default_rng(n * 13 + npairs)
    a, b = _operands(g, n, npairs)
    if op == "sub":
        b, a = a, b  # borrows run through the zero operand minus all-ones
    cin = g.integers(0, 2, npairs, dtype=np.uint64)
    cin[::3] = 1
    tr = torch.full((n * npairs,), -1, dtype=torch.int64, device="cuda")
    tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
    f = bn.bn_add_nc_n_batch if op == "add" else bn.bn_sub_nc_n_batch
    f(bnctx, tr, D(a), D(b), n, npairs, D(cin), tc)
    torch.cuda.synchronize()
    rr, rc = (oracle.add_nc_batch if op == "add" else oracle.sub_nc_batch)(a, b, n, cin)
    assert (H(tr) == rr).all() and (H(tc) == rc).all()


def test_carry_in_misaligned_and_in_place(bnctx):
    """8-byte aligned operands (the unaligned kernel path) and r == a."""
    g = np.random.default_rng(5)
    n, npairs = 300, 17
    a, b = _operands(g, n, npairs)
    cin = np.ones(npairs, np.uint64)
    ta = D(np.concatenate([np.zeros(1, np.uint64), a]))[1:]
    tb = D(np.concatenate([np.zeros(1, np.uint64), b]))[1:]
    tc = torch.zeros(npairs, dtype=torch.int64, device="cuda")
    bn.bn_add_nc_n_batch(bnctx, ta, ta, tb, n, npairs, D(cin), tc)
    torch.cuda.synchronize()
    rr, rc = oracle.add_nc_batch(a, b, n, cin)
    assert (H(ta) == rr).all() and (H(tc) == rc).all()


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("na,nb", [(10, 3), (1, 0), (5, 5), (4097, 4096), (70000, 1), (300001, 17), (8, 0)])
def test_unequal_lengths(bnctx, op, na, nb):
    announce("unequal", op, f"na={na}", f"nb={nb}")
    g = np.random.default_rng(na + 7 * nb)
    a = _rand(g, na)
    b = _rand(g, nb)
    # force the carry (borrow) out of the low part to run through most of the top part
    if op == "add":
        a[nb:max(nb, na - 1)] = MAX
        if nb:
            b[:] = MAX
    else:
        a[nb:max(nb, na - 1)] = 0
        if nb:
            a[:nb] = 0
            b[0] = 1
    bext = np.concatenate([b, np.zeros(na - nb, np.uint64)])
    tr = torch.full((max(na, 1),), -1, dtype=torch.int64, device="cuda")[:na]
    tc = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    f = bn.bn_add_unequal if op == "add" else bn.bn_sub_unequal
    f(bnctx, tr, D(a) if na else tr, na, D(b) if nb else tr, nb, tc)
    torch.cuda.synchronize()
    rr, rc = (oracle.add if op == "add" else oracle.sub)(a, bext)
    assert (H(tr) == rr).all() and int(H(tc)[0]) == rc


@pytest.mark.parametrize("n,npairs", [(1, 600), (4, 1088), (64, 999), (5000, 5), (100003, 2)])
def test_sub_abs(bnctx, n, npairs):
    announce("|a-b|", f"n={n}", f"npairs={npairs}")
    g = np.random.default_rng(n + npairs)
    a = _rand(g, n * npairs).reshape(npairs, n)
    b = _rand(g, n * npairs).reshape(npairs, n)
    b[::4] = a[::4]          # equal pairs: zero, sign 0
    b[1::4, :-1] = a[1::4, :-1]  # differ only in the top limb
    a, b = a.reshape(-1), b.reshape(-1)
    r1, s1 = oracle.sub_batch(a, b, n)
    r2, _ = oracle.sub_batch(b, a, n)
    want = np.where(np.repeat(s1, n).astype(bool), r2, r1)
    for alias in ("none", "a", "b"):
        ta, tb = D(a), D(b)
        tr = {"none": torch.empty_like(ta), "a": ta, "b": tb}[alias]
        ts = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
        bn.bn_sub_abs_n_batch(bnctx, tr, ta, tb, n, npairs, ts)
        torch.cuda.synchronize()
        assert (H(tr) == want).all(), alias
        assert (H(ts) == s1).all(), alias


def test_errors(bnctx):
    t = torch.zeros(64, dtype=torch.int64, device="cuda")
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_unequal(bnctx, t[:8], t[8:12], 4, t[16:24], 8)  # na < nb
    assert e.value.status == bn.BN_EINVAL
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_nc_n_batch(bnctx, t[:16], t[16:32], t[32:48], 4, 4, None, c)  # no carry-in
    assert e.value.status == bn.BN_EINVAL
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_nc_n_batch(bnctx, t[:16], t[16:32], t[32:48], 4, 4, c, c)  # carry-out over carry-in
    assert e.value.status == bn.BN_EALIAS
    # n = 0: the carry passes through
    cin = D(np.array([1, 0, 1, 1], np.uint64))
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    bn.bn_add_nc_n_batch(bnctx, t[:0], t[:0], t[:0], 0, 4, cin, out)
    torch.cuda.synchronize()
    assert H(out).tolist() == [1, 0, 1, 1]


def _unequal_operands(g, na, nb, npairs, op):
    """Pairs of na and nb limbs; every second pair makes its carry (borrow) run from b's
    top limb through all of a's limbs above it (b all-ones or a zero there)."""
    a = _rand(g, na * npairs).reshape(npairs, na)
    b = _rand(g, nb * npairs).reshape(npairs, nb)
    for p in range(0, npairs, 2):
        if op == "add":
            a[p, nb:] = MAX
            if nb:
                b[p, :] = MAX
                a[p, :nb] = 1
        else:
            a[p, nb:] = 0
            if nb:
                a[p, :nb] = 0
                b[p, 0] = 1
    bext = np.zeros((npairs, na), np.uint64)
    bext[:, :nb] = b
    return a.reshape(-1), b.reshape(-1), bext.reshape(-1)


UNEQUAL = [(4, 1, 1088), (64, 10, 4096), (100, 100, 77), (129, 64, 33), (5000, 37, 7), (100003, 70001, 3),
           (7, 0, 100), (128, 127, 50), (1, 1, 10), (300, 1, 31), (4096, 4095, 5), (262147, 3, 2)]


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("na,nb,npairs", UNEQUAL)
def test_unequal_batches(bnctx, op, na, nb, npairs):
    """Theorem 2's zero-extension: a_p +- b_p with b_p padded to na limbs, bit-exact
    against the oracle's equal-length batch on the padded operands."""
    announce("unequal batch", op, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    g = np.random.default_rng(na * 31 + nb * 7 + npairs)
    a, b, bext = _unequal_operands(g, na, nb, npairs, op)
    rr, rc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, bext, na)
    f = bn.bn_add_unequal_n_batch if op == "add" else bn.bn_sub_unequal_n_batch
    for offset in (0, 1):   # 16-byte and 8-byte aligned operands
        ta = D(np.concatenate([np.zeros(offset, np.uint64), a]))[offset:]
        tb = D(np.concatenate([np.zeros(offset, np.uint64), b]))[offset:] if nb else \
            torch.zeros(1, dtype=torch.int64, device="cuda")
        tr = torch.full((na * npairs + offset,), -1, dtype=torch.int64, device="cuda")[offset:]
        tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
        f(bnctx, tr, ta, na, tb, nb, npairs, tc)
        torch.cuda.synchronize()
        got = H(tr)
        assert (got == rr).all(), f"offset {offset}: first bad limb {np.argmax(got != rr)}"
        assert (H(tc) == rc).all(), f"offset {offset}: first bad carry {np.argmax(H(tc) != rc)}"
        # in place over a
        f(bnctx, ta, ta, na, tb, nb, npairs, tc)
        torch.cuda.synchronize()
        assert (H(ta) == rr).all() and (H(tc) == rc).all(), f"in place, offset {offset}"


def test_unequal_batch_rejects_bad_arguments(bnctx):
    g = np.random.default_rng(1)
    a, b = D(_rand(g, 40)), D(_rand(g, 40))
    r = torch.empty(40, dtype=torch.int64, device="cuda")
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_unequal_n_batch(bnctx, r, a, 4, b, 5, 8)     # nb > na
    assert e.value.status == bn.BN_EINVAL
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_unequal_n_batch(bnctx, b, a, 5, b, 4, 8)   # r is b while the lengths differ
    assert e.value.status == bn.BN_EALIAS
