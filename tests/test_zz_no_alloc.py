"""bn_addsub_n_batch_noalloc: the add/sub entry point whose look-back state lives in the
library's fixed per-GPU array.  Through the C ABI, every case runs two calls in a row,
the second on a smaller input (it finds the first call's status words in the array),
and each result is compared limb by limb with bn_add_n_batch / bn_sub_n_batch on a
context with a reserved workspace and with the CPU oracle (Theorem 1)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2604_21566_amd as bn
from conftest import announce
from paper_2604_21566_amd import workloads as wl

pytestmark = pytest.mark.gpu
D = bn.to_device
H = bn.to_host
MAX = 2 ** 64 - 1


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    strict = bn.bn_create(0)            # no workspace, no growth: the call must not need one
    ref = bn.bn_create(0, auto_grow=True)
    yield strict, ref
    torch.cuda.synchronize()
    bn.bn_destroy(strict)
    bn.bn_destroy(ref)


def _inputs(kind, op, n, npairs, seed):
    g = np.random.default_rng(seed)
    if kind == "runs":       # one pair, random limbs with long carry (borrow) runs across tiles
        return wl.c3(op, n=n, seed=seed)
    if kind == "worst":      # one pair, the carry (borrow) crosses every limb
        return wl.c3(op, n=n, worst=True)
    a = g.integers(0, MAX, n * npairs, dtype=np.uint64, endpoint=True)
    b = g.integers(0, MAX, n * npairs, dtype=np.uint64, endpoint=True)
    if op == "add":          # every 3rd pair: all-propagate body with a generate at limb 0
        for p in range(0, npairs, 3):
            s = slice(p * n + 1, (p + 1) * n)
            b[s] = ~a[s]
            a[p * n], b[p * n] = MAX, 1
    else:
        for p in range(0, npairs, 3):
            s = slice(p * n + 1, (p + 1) * n)
            b[s] = a[s]
            a[p * n], b[p * n] = 0, 1
    return a, b


def _run_pair(ctxs, op, a, b, n, npairs, offset=0, in_place=False):
    """The new call and the existing one on the same device inputs; returns both results
    and the oracle's.  offset: limbs the operands start past a 16-byte boundary."""
    strict, ref = ctxs
    sub = 1 if op == "sub" else 0
    N = n * npairs
    want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)
    ta_buf, tb_buf = D(np.concatenate([np.zeros(offset, np.uint64), a])), \
        D(np.concatenate([np.zeros(offset, np.uint64), b]))
    ta, tb = ta_buf[offset:], tb_buf[offset:]
    tr = ta if in_place else torch.full((N,), 7, dtype=torch.int64, device="cuda")
    tc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
    bn.bn_addsub_n_batch_noalloc(strict, sub, tr, ta, tb, n, npairs, tc)
    got, gc = H(tr), H(tc)
    # the existing entry point on fresh copies of the operands
    ra_buf, rb_buf = D(np.concatenate([np.zeros(offset, np.uint64), a])), \
        D(np.concatenate([np.zeros(offset, np.uint64), b]))
    ra, rb = ra_buf[offset:], rb_buf[offset:]
    rr = ra if in_place else torch.full((N,), 7, dtype=torch.int64, device="cuda")
    rc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
    (bn.bn_sub_n_batch if sub else bn.bn_add_n_batch)(ref, rr, ra, rb, n, npairs, rc)
    return (got, gc), (H(rr), H(rc)), (want, wc)


def _assert_same(res, what):
    (got, gc), (old, oc), (want, wc) = res
    assert (got == old).all() and (gc == oc).all(), \
        f"{what}: differs from the existing entry point at limb {np.argmax(got != old)}"
    assert (got == want).all() and (gc == np.asarray(wc, np.uint64)).all(), \
        f"{what}: differs from the oracle at limb {np.argmax(got != want)}"


CASES = [
    # (kind, n1, npairs1, n2, npairs2): second call smaller
    ("runs", 1 << 22, 1, 300001, 1),        # chained single pair, carries cross tiles
    ("worst", 1 << 21, 1, 70001, 1),        # all-propagate: the look-back walks to tile 0
    ("batch", 30011, 40, 4099, 13),         # chained batch (pairs longer than a tile)
    ("batch", 100, 20000, 3, 50000),        # chained batch (pairs not dividing 128)
    ("batch", 64, 1 << 15, 4, 1088),        # independent tiles: no status words at all
]


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("kind,n1,p1,n2,p2", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}" for c in CASES])
def test_two_calls_second_smaller(ctxs, op, kind, n1, p1, n2, p2):
    for step, (n, npairs) in enumerate(((n1, p1), (n2, p2))):
        announce("noalloc", op, kind, f"call {step}", n, npairs)
        a, b = _inputs(kind, op, n, npairs, seed=17 * step + n)
        _assert_same(_run_pair(ctxs, op, a, b, n, npairs), f"{op} {kind} call {step} {n}x{npairs}")


@pytest.mark.parametrize("op", ["add", "sub"])
def test_unaligned_and_in_place(ctxs, op):
    """8-byte-aligned operands (the unaligned tile shape) and r == a, two calls each."""
    for step, n in enumerate((500009, 123457)):
        announce("noalloc unaligned", op, n)
        a, b = _inputs("runs", op, n, 1, seed=5 + step)
        _assert_same(_run_pair(ctxs, op, a, b, n, 1, offset=1), f"{op} unaligned {n}")
        announce("noalloc in place", op, n)
        _assert_same(_run_pair(ctxs, op, a, b, n, 1, in_place=True), f"{op} in place {n}")


def test_captured_replays_match_eager_calls(ctxs):
    """Recorded into a graph, the launch takes its epoch from the array's control block;
    replays interleaved with eager calls of another size stay exact."""
    strict, _ = ctxs
    n = 1 << 20
    a, b = _inputs("runs", "add", n, 1, seed=99)
    want, wc = oracle.add(a, b)
    ta, tb = D(a), D(b)
    tr = torch.empty(n, dtype=torch.int64, device="cuda")
    tc = torch.empty(1, dtype=torch.int64, device="cuda")
    a2, b2 = _inputs("worst", "sub", 77777, 1, seed=0)
    want2, wc2 = oracle.sub(a2, b2)
    ta2, tb2 = D(a2), D(b2)
    tr2 = torch.empty(77777, dtype=torch.int64, device="cuda")
    tc2 = torch.empty(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    announce("noalloc capture")
    with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
        bn.bn_addsub_n_batch_noalloc(strict, 0, tr, ta, tb, n, 1, tc)
    for rep in range(3):
        tr.fill_(7)
        tc.fill_(7)
        torch.cuda.synchronize()
        announce("noalloc replay", rep)
        graph.replay()
        torch.cuda.synchronize()
        assert (H(tr) == want).all() and int(H(tc)[0]) == wc, f"replay {rep}"
        bn.bn_addsub_n_batch_noalloc(strict, 1, tr2, ta2, tb2, 77777, 1, tc2)
        torch.cuda.synchronize()
        assert (H(tr2) == want2).all() and int(H(tc2)[0]) == wc2, f"eager call after replay {rep}"
    del graph


def test_maximum_size_then_smaller(ctxs):
    """One pair at the array's limit at the default shapes (2^28 limbs, 2 GiB per operand)
    against the existing entry point on the device, then one limb-tile more is refused
    on the host with BN_ERANGE and nothing enqueued, then a smaller call."""
    strict, ref = ctxs
    n = 1 << 28
    announce("noalloc maximum size", n)
    gen = torch.Generator(device="cuda").manual_seed(11)
    a = torch.randint(-2 ** 63, 2 ** 63 - 1, (n,), dtype=torch.int64, device="cuda", generator=gen)
    b = torch.randint(-2 ** 63, 2 ** 63 - 1, (n,), dtype=torch.int64, device="cuda", generator=gen)
    # carries that cross many tiles: an all-propagate stretch fed by a generating limb
    lo, hi = 12345, 12345 + (1 << 24)
    b[lo + 1:hi] = torch.bitwise_not(a[lo + 1:hi])
    a[lo] = -1
    b[lo] = 1
    r_new = torch.full((n,), 7, dtype=torch.int64, device="cuda")
    r_old = torch.full((n,), 5, dtype=torch.int64, device="cuda")
    c = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    bn.bn_addsub_n_batch_noalloc(strict, 0, r_new, a, b, n, 1, c[0:1])
    bn.bn_add(ref, r_old, a, b, c[1:2])
    torch.cuda.synchronize()
    assert torch.equal(r_new, r_old) and int(c[0]) == int(c[1])
    # spot checks against the oracle: the stretch's two ends and the top limbs
    ah, bh, rh = H(a), H(b), H(r_new)
    for s0, s1 in ((lo - 3, lo + 70), (hi - 70, hi + 5), (n - 64, n)):
        # carry into limb s0: limb s0-1 took carry c = (r - a - b) mod 2^64 (must be 0 or 1)
        # and passes on floor((a + b + c) / 2^64)
        x, y, z = int(ah[s0 - 1]), int(bh[s0 - 1]), int(rh[s0 - 1])
        c_prev = (z - x - y) % 2 ** 64
        assert c_prev in (0, 1)
        cin = (x + y + c_prev) >> 64
        exp, _ = oracle.add_nc_batch(ah[s0:s1].copy(), bh[s0:s1].copy(), s1 - s0, np.array([cin], np.uint64))
        assert (rh[s0:s1] == exp).all(), f"limbs {s0}..{s1}"
    del ah, bh, rh
    # one 2048-limb tile more than the array holds: refused before anything is enqueued
    m = n + 2048
    big = torch.empty(3 * m, dtype=torch.int64, device="cuda")
    before = c.clone()
    st = bn.lib().bn_addsub_n_batch_noalloc(strict, 0, big[2 * m:].data_ptr(), big[:m].data_ptr(),
                                            big[m:2 * m].data_ptr(), m, 1, c.data_ptr(),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == bn.BN_ERANGE
    torch.cuda.synchronize()
    assert torch.equal(c, before)
    del big, a, b, r_new, r_old
    torch.cuda.empty_cache()
    # and a smaller call after it
    a2, b2 = _inputs("worst", "add", 333333, 1, seed=0)
    _assert_same(_run_pair(ctxs, "add", a2, b2, 333333, 1), "after the refused call")


def test_bad_arguments_are_refused(ctxs):
    strict, _ = ctxs
    L = bn.lib()
    assert L.bn_addsub_n_batch_noalloc(None, 0, None, None, None, 0, 0, None, None) == bn.BN_EINVAL
    assert L.bn_addsub_n_batch_noalloc(strict, 2, None, None, None, 0, 0, None, None) == bn.BN_EINVAL
    # n = 0: the carries are 0
    c = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    assert L.bn_addsub_n_batch_noalloc(strict, 0, None, None, None, 0, 4, c.data_ptr(),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == bn.BN_OK
    torch.cuda.synchronize()
    assert (H(c) == 0).all()
