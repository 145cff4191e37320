"""Deferred all-propagate tiles.  In chained add/sub launches of at least
"addsub.defer_tiles" tiles, a tile whose every limb propagates stores nothing; after the
launch a scan of the status words finds its carry-in and a fill pass writes its constant
result (all ones or all zeros).  Here the threshold is 1, so every chained launch takes
that form, and each result is compared limb by limb with the oracle.  Full-size C3 runs
the deferred form by default (test_gpu_addsub.py)."""
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


@pytest.fixture
def dctx(bnctx):
    old = bn.bn_get_param(bnctx, "addsub.defer_tiles")
    bn.bn_set_param(bnctx, "addsub.defer_tiles", 1)
    try:
        yield bnctx
    finally:
        bn.bn_set_param(bnctx, "addsub.defer_tiles", old)


def _mixed(op, N, seed):
    """Random limbs with all-propagate runs of 300..40000 limbs; the limb under each run
    is random, so runs are entered with carry 0 or 1 about equally often."""
    g = np.random.default_rng(seed)
    a = g.integers(0, MAX, N, dtype=np.uint64, endpoint=True)
    b = g.integers(0, MAX, N, dtype=np.uint64, endpoint=True)
    pos = 0
    while True:
        pos += int(g.integers(1, 30000))
        ln = int(g.integers(300, 40000))
        if pos + ln > N:
            break
        if op == "add":
            a[pos:pos + ln] = g.integers(0, MAX, ln, dtype=np.uint64, endpoint=True)
            b[pos:pos + ln] = ~a[pos:pos + ln]
        else:
            b[pos:pos + ln] = a[pos:pos + ln]
        pos += ln
    return a, b


def _inputs(op, kind, N, seed=0):
    if kind in ("runs", "worst"):
        return wl.c3(op, n=N, worst=kind == "worst", seed=seed)
    if kind == "propagate0":
        a = np.full(N, MAX if op == "add" else 5, np.uint64)
        return a, (np.zeros(N, np.uint64) if op == "add" else a.copy())
    return _mixed(op, N, seed)


def _run(ctx, op, a, b, n, npairs, offset=0, fn=None):
    N = n * npairs
    ta = D(np.concatenate([np.zeros(offset, np.uint64), a]))[offset:]
    tb = D(np.concatenate([np.zeros(offset, np.uint64), b]))[offset:]
    tr = torch.full((N + offset,), 7, dtype=torch.int64, device="cuda")[offset:]
    tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
    if fn is None:
        (bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch)(ctx, tr, ta, tb, n, npairs, tc)
    else:
        fn(tr, ta, tb, tc)
    torch.cuda.synchronize()
    return H(tr), H(tc)


def _expect(op, a, b, n):
    return (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)


def _same(got, want, what):
    r, c = got
    wr, wc = want
    assert (r == wr).all(), f"{what}: first bad limb {np.argmax(r != wr)} of {r.size}"
    assert (c == wc).all(), f"{what}: carries {c} vs {wc}"


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("kind", ["runs", "worst", "propagate0", "mixed"])
@pytest.mark.parametrize("N,offset", [((1 << 18) + 77, 0), (1 << 20, 0), ((1 << 18) + 77, 1), (1 << 20, 1)])
def test_single_pair(dctx, op, kind, N, offset):
    """One pair: aligned (16-byte loads, vector fill) and shifted by one limb (8-byte
    loads, scalar fill), with a ragged top tile and without."""
    a, b = _inputs(op, kind, N, seed=N + offset)
    announce("deferred", op, kind, f"N={N}", f"offset={offset}")
    _same(_run(dctx, op, a, b, N, 1, offset), _expect(op, a, b, N), f"{op} {kind} N={N} offset={offset}")


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n,npairs", [(100003, 5), (3001, 300), (40000, 20)])
def test_batches(dctx, op, n, npairs):
    """Pairs longer than a tile: all-propagate tiles inside pairs, segment ends in
    others (their carry-outs are stored by the tiles that hold them)."""
    a, b = _mixed(op, n * npairs, seed=n)
    announce("deferred batch", op, f"n={n}", f"npairs={npairs}")
    _same(_run(dctx, op, a, b, n, npairs), _expect(op, a, b, n), f"{op} n={n} npairs={npairs}")


@pytest.mark.parametrize("op", ["add", "sub"])
def test_carry_in_batch(dctx, op):
    """Per-pair carry-in (the carry-in kernel variant): every limb propagates, so each
    pair's carry-in decides all of its limbs."""
    n, npairs = 100003, 4
    a = np.full(n * npairs, MAX if op == "add" else 9, np.uint64)
    b = np.zeros(n * npairs, np.uint64) if op == "add" else a.copy()
    cin = np.array([1, 0, 0, 1], np.uint64)
    announce("deferred carry-in", op, f"n={n}", f"npairs={npairs}")
    tci = D(cin)
    f = bn.bn_add_nc_n_batch if op == "add" else bn.bn_sub_nc_n_batch
    got = _run(dctx, op, a, b, n, npairs, fn=lambda tr, ta, tb, tc: f(dctx, tr, ta, tb, n, npairs, tci, tc))
    want = (oracle.add_nc_batch if op == "add" else oracle.sub_nc_batch)(a, b, n, cin)
    _same(got, want, f"{op} carry-in")


@pytest.mark.parametrize("op", ["add", "sub"])
def test_unequal_batch(dctx, op):
    """b shorter than a in every pair (b zero-extended): past nb the limbs of a = all
    ones (add) or 0 (sub) propagate."""
    na, nb, npairs = 120011, 30007, 3
    g = np.random.default_rng(5)
    a = np.full(na * npairs, MAX if op == "add" else 0, np.uint64)
    b = g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True)
    a.reshape(npairs, na)[:, :nb] = g.integers(0, MAX, (npairs, nb), dtype=np.uint64, endpoint=True)
    bext = np.zeros((npairs, na), np.uint64)
    bext[:, :nb] = b.reshape(npairs, nb)
    announce("deferred unequal", op, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    ta, tb = D(a), D(b)
    tr = torch.full((na * npairs,), 7, dtype=torch.int64, device="cuda")
    tc = torch.full((npairs,), -1, dtype=torch.int64, device="cuda")
    (bn.bn_add_unequal_n_batch if op == "add" else bn.bn_sub_unequal_n_batch)(dctx, tr, ta, na, tb, nb, npairs, tc)
    torch.cuda.synchronize()
    _same((H(tr), H(tc)), _expect(op, a, bext.reshape(-1), na), f"{op} unequal")


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("target", ["a", "b"])
def test_in_place_spin_zero(dctx, op, target):
    """In place at a spin limit of 0: every tile whose predecessor has not published
    leaves its repair to the fill pass, and all-propagate tiles leave their operand
    limbs untouched until the fill pass overwrites them."""
    old = bn.bn_get_param(dctx, "lookback.spin_limit")
    try:
        bn.bn_set_param(dctx, "lookback.spin_limit", 0)
        for kind in ("worst", "mixed"):
            N = (1 << 18) + 77
            a, b = _inputs(op, kind, N, seed=3)
            announce("deferred in place", op, kind, f"r={target}")
            ta, tb = D(a), D(b)
            tc = torch.full((1,), -1, dtype=torch.int64, device="cuda")
            r = ta if target == "a" else tb
            (bn.bn_add if op == "add" else bn.bn_sub)(dctx, r, ta, tb, tc)
            torch.cuda.synchronize()
            _same((H(r), H(tc)), _expect(op, a, b, N), f"{op} {kind} in place r={target}")
    finally:
        bn.bn_set_param(dctx, "lookback.spin_limit", old)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_spin_zero(dctx, op):
    """Out of place at a spin limit of 0: a tile whose nearest predecessor that does not
    propagate has not published yet never waits (deferred launches have no self-help);
    it leaves its repair to the fill pass."""
    old = bn.bn_get_param(dctx, "lookback.spin_limit")
    try:
        bn.bn_set_param(dctx, "lookback.spin_limit", 0)
        for kind in ("runs", "mixed", "worst"):
            N = (1 << 20) + 3
            a, b = _inputs(op, kind, N, seed=11)
            announce("deferred, spin limit 0", op, kind)
            _same(_run(dctx, op, a, b, N, 1), _expect(op, a, b, N), f"{op} {kind} spin 0")
    finally:
        bn.bn_set_param(dctx, "lookback.spin_limit", old)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_graph_replay(dctx, op):
    """Captured deferred launch (its epoch comes from the control block): four replays,
    each followed by the same eager call, all exact."""
    n, npairs = 50021, 6
    a, b = _mixed(op, n * npairs, seed=21)
    want = _expect(op, a, b, n)
    announce("deferred graph replay", op, f"n={n}", f"npairs={npairs}")
    ta, tb = D(a), D(b)
    tr = torch.empty_like(ta)
    tc = torch.empty(npairs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    g = bn.bn_graph_capture_batch(dctx, 0 if op == "add" else 1, tr, ta, tb, n, 0, npairs, tc, stream=s)
    try:
        for rep in range(4):
            tr.fill_(7)
            tc.fill_(7)
            torch.cuda.synchronize()
            bn.bn_graph_launch(g, s)
            s.synchronize()
            _same((H(tr), H(tc)), want, f"replay {rep}")
            tr.fill_(7)
            (bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch)(dctx, tr, ta, tb, n, npairs, tc)
            torch.cuda.synchronize()
            _same((H(tr), H(tc)), want, f"eager after replay {rep}")
    finally:
        bn.bn_graph_destroy(g)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_no_alloc_entry_point(dctx, op):
    """The fixed per-GPU array holds the fill codes after the status words: two calls
    in a row, the second smaller, both exact."""
    for N, kind in (((1 << 20) + 9, "mixed"), ((1 << 18) + 1, "worst")):
        a, b = _inputs(op, kind, N, seed=N)
        announce("deferred no-alloc", op, kind, f"N={N}")
        got = _run(dctx, op, a, b, N, 1,
                   fn=lambda tr, ta, tb, tc: bn.bn_addsub_n_batch_noalloc(dctx, 0 if op == "add" else 1, tr, ta, tb,
                                                                           N, 1, tc))
        _same(got, _expect(op, a, b, N), f"{op} {kind} no-alloc N={N}")


def test_products(dctx):
    """Products whose operand conversion and carry pass are chained scans (constant-b
    and plain variants), on both forms, with all-ones operands (every column's carries
    run far)."""
    for na, nb, npairs, form in ((4096, 4096, 3, "mfma"), (3000, 2000, 2, "mad"), (20000, 20000, 1, "mfma")):
        a = np.full(na * npairs, MAX, np.uint64)
        b = np.full(nb * npairs, MAX, np.uint64)
        a[::7] = 12345
        announce("deferred product", f"na={na}", f"nb={nb}", f"npairs={npairs}", form)
        tr = torch.full(((na + nb) * npairs,), 7, dtype=torch.int64, device="cuda")
        bn.bn_mul_n_batch(dctx, tr, D(a), D(b), na, nb, npairs, form)
        torch.cuda.synchronize()
        want = oracle.mul_batch(a, b, na, nb, npairs)
        got = H(tr)
        assert (got == want).all(), f"{na}x{nb} {form}: first bad limb {np.argmax(got != want)}"


@pytest.mark.parametrize("offset", [0, 1])
def test_karatsuba(dctx, offset):
    """Karatsuba levels: split scans and the combine scan that forms its own terms, in
    the deferred form, into a 16-byte aligned output and one shifted by a limb (the
    8-byte kernels).  Operands with long all-ones and zero stretches make the
    combine's sums propagate across many tiles."""
    g = np.random.default_rng(31 + offset)
    for na, nb, npairs, levels, form in ((4096, 4096, 3, 2, "mfma"), (3001, 2500, 2, 1, "mad"),
                                         (9000, 9000, 1, 3, "auto")):
        a = g.integers(0, MAX, na * npairs, dtype=np.uint64, endpoint=True)
        b = g.integers(0, MAX, nb * npairs, dtype=np.uint64, endpoint=True)
        a[: na // 2] = MAX
        b[nb // 3: nb // 2] = 0
        announce("deferred karatsuba", f"na={na}", f"nb={nb}", f"npairs={npairs}", f"levels={levels}", form,
                 f"offset={offset}")
        P = (na + nb) * npairs
        tr = torch.full((P + offset,), 7, dtype=torch.int64, device="cuda")[offset:]
        bn.bn_mul_karatsuba_batch(dctx, tr, D(a), na, D(b), nb, npairs, levels, form)
        torch.cuda.synchronize()
        want = oracle.mul_batch(a, b, na, nb, npairs)
        got = H(tr)
        assert (got == want).all(), f"{na}x{nb} L{levels} {form}: first bad limb {np.argmax(got != want)}"


def test_param(bnctx):
    old = bn.bn_get_param(bnctx, "addsub.defer_tiles")
    assert old == 8192
    assert "addsub.defer_tiles" in bn.bn_param_names()
    with pytest.raises(bn.BnError):
        bn.bn_set_param(bnctx, "addsub.defer_tiles", -1)
    bn.bn_set_param(bnctx, "addsub.defer_tiles", 0)
    assert bn.bn_get_param(bnctx, "addsub.defer_tiles") == 0
    bn.bn_set_param(bnctx, "addsub.defer_tiles", old)
