"""GPU add/sub parity against the CPU oracle, bit-exact, through the C ABI."""
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


def _run_batch(ctx, op, a, b, n, npairs, offset=0):
    """Run the GPU batch op; `offset` shifts the operands by that many limbs inside
    larger buffers (8-byte aligned but not 16-byte aligned when odd)."""
    N = n * npairs
    ta = D(np.concatenate([np.zeros(offset, np.uint64), a]))[offset:]
    tb = D(np.concatenate([np.zeros(offset, np.uint64), b]))[offset:]
    tr = torch.empty(N + offset, dtype=torch.int64, device="cuda")[offset:]
    tc = torch.full((max(npairs, 1),), -1, dtype=torch.int64, device="cuda")
    f = bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch
    f(ctx, tr, ta, tb, n, npairs, tc)
    torch.cuda.synchronize()
    return H(tr), H(tc)[:npairs]


def _check(ctx, op, a, b, n, npairs, offset=0):
    announce(op, f"n={n}", f"npairs={npairs}", f"offset={offset}")
    r, c = _run_batch(ctx, op, a, b, n, npairs, offset)
    ref = oracle.add_batch if op == "add" else oracle.sub_batch
    rr, rc = ref(a, b, n)
    assert (r == rr).all(), f"{op} n={n} npairs={npairs}: first bad limb {np.argmax(r != rr)}"
    assert (c == rc).all(), f"{op} n={n} npairs={npairs}: first bad carry {np.argmax(c != rc)}"


SHAPES = [(1, 1), (1, 1000), (2, 700), (3, 333), (4, 1088), (5, 211), (7, 100), (63, 77), (64, 130),
          (65, 65), (127, 9), (128, 40), (129, 33), (1000, 17), (4095, 3), (4096, 5), (4097, 4),
          (100000, 2), (262145, 1)]


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n,npairs", SHAPES)
def test_batch_random(bnctx, op, n, npairs):
    g = np.random.default_rng(n * 7 + npairs)
    a = g.integers(0, 2 ** 64 - 1, n * npairs, dtype=np.uint64, endpoint=True)
    b = g.integers(0, 2 ** 64 - 1, n * npairs, dtype=np.uint64, endpoint=True)
    _check(bnctx, op, a, b, n, npairs)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n", [1, 2, 4, 9, 64, 200, 5000])
def test_pathological(bnctx, op, n):
    pa, pb = wl.pathological(n, 4, seed=n)
    _check(bnctx, op, pa.reshape(-1), pb.reshape(-1), n, pa.shape[0])


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n,npairs", [(4, 1088), (64, 300), (129, 50), (5000, 19)])
def test_unaligned_operands(bnctx, op, n, npairs):
    g = np.random.default_rng(n)
    pa, pb = wl.pathological(n, 2, seed=3)
    a = np.concatenate([pa.reshape(-1), g.integers(0, 2 ** 63, n * (npairs - pa.shape[0]), dtype=np.uint64)])
    b = np.concatenate([pb.reshape(-1), g.integers(0, 2 ** 63, n * (npairs - pb.shape[0]), dtype=np.uint64)])
    _check(bnctx, op, a, b, n, npairs, offset=1)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_c1(bnctx, op):
    a, b = wl.c1(op)
    _check(bnctx, op, a, b, 4, 1088)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_c2_reduced(bnctx, op):
    a, b = wl.c2(op, npairs=1 << 14)
    _check(bnctx, op, a, b, 64, 1 << 14)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_c2_full(bnctx, op):
    a, b = wl.c2(op)
    _check(bnctx, op, a, b, 64, 1 << 20)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("kind", ["runs", "worst", "propagate0"])
def test_c3_full(bnctx, op, kind):
    """2^26 limbs: random with carry runs, the carry crossing every limb, and every limb
    propagating with no carry entering anywhere (every tile but the first is an
    all-propagate tile whose carry-in is 0)."""
    if kind == "propagate0":
        n = 1 << 26
        a = np.full(n, 2 ** 64 - 1 if op == "add" else 5, np.uint64)
        b = np.zeros(n, np.uint64) if op == "add" else a.copy()
    else:
        a, b = wl.c3(op, worst=kind == "worst")
    _check(bnctx, op, a, b, a.size, 1)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("kind", ["runs", "worst"])
def test_c3_full_waiting_form(bnctx, op, kind):
    """2^26 limbs in the waiting form (addsub.defer_tiles 0: every tile looks back before
    it finishes), the second form the benchmark times at this size."""
    a, b = wl.c3(op, worst=kind == "worst")
    old = bn.bn_get_param(bnctx, "addsub.defer_tiles")
    bn.bn_set_param(bnctx, "addsub.defer_tiles", 0)
    try:
        _check(bnctx, op, a, b, a.size, 1)
    finally:
        bn.bn_set_param(bnctx, "addsub.defer_tiles", old)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("waves,rows", [(w, r) for w in (1, 2, 4, 8) for r in (1, 2, 4, 8, 16) if w * r < 128])
def test_every_tile_shape(bnctx, op, waves, rows):
    keys = ("addsub.batch_waves", "addsub.batch_rows", "addsub.chain_waves", "addsub.chain_rows")
    old = {k: bn.bn_get_param(bnctx, k) for k in keys}
    try:
        for k, v in zip(keys, (waves, rows, waves, rows)):
            bn.bn_set_param(bnctx, k, v)
        a, b = wl.c3(op, n=300007)
        _check(bnctx, op, a, b, a.size, 1)
        pa, pb = wl.pathological(333, 3, seed=5)
        _check(bnctx, op, pa.reshape(-1), pb.reshape(-1), 333, pa.shape[0])
        pa, pb = wl.pathological(64, 3, seed=6)
        _check(bnctx, op, pa.reshape(-1), pb.reshape(-1), 64, pa.shape[0])
        aw, bw = wl.c3(op, n=70001, worst=True)
        _check(bnctx, op, aw, bw, aw.size, 1)
    finally:
        for k, v in old.items():
            bn.bn_set_param(bnctx, k, v)


def test_in_place_and_single_pair_api(bnctx):
    announce("in-place add/sub")
    g = np.random.default_rng(2)
    a = g.integers(0, 2 ** 64 - 1, 10007, dtype=np.uint64, endpoint=True)
    b = g.integers(0, 2 ** 64 - 1, 10007, dtype=np.uint64, endpoint=True)
    ta, tb = D(a), D(b)
    c = torch.zeros(1, dtype=torch.int64, device="cuda")
    bn.bn_add(bnctx, ta, ta, tb, c)          # r == a
    r, cc = oracle.add(a, b)
    assert (H(ta) == r).all() and int(H(c)[0]) == cc
    bn.bn_sub(bnctx, tb, ta, tb, c)          # r == b: (a + b) - b
    d, br = oracle.sub(r, b)
    assert (H(tb) == d).all() and int(H(c)[0]) == br


def test_empty_and_errors(bnctx):
    announce("empty sizes and argument errors")
    z = torch.empty(0, dtype=torch.int64, device="cuda")
    c = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    bn.bn_add_n_batch(bnctx, z, z, z, 0, 3, c)      # n = 0: carries are 0
    torch.cuda.synchronize()
    assert (H(c) == 0).all()
    bn.bn_add_n_batch(bnctx, z, z, z, 5, 0, None)   # no pairs
    t = torch.zeros(16, dtype=torch.int64, device="cuda")
    with pytest.raises(bn.BnError) as e:
        bn.bn_add_n_batch(bnctx, t[1:9], t[0:8], t[8:16], 8, 1)   # partial overlap r/a
    assert e.value.status == bn.BN_EALIAS
    L = bn.lib()
    assert L.bn_add(bnctx, t.data_ptr() + 4, t.data_ptr(), t.data_ptr(), 1, None, None) == bn.BN_EINVAL
    assert L.bn_add(bnctx, None, t.data_ptr(), t.data_ptr(), 1, None, None) == bn.BN_EINVAL
    assert L.bn_add_n_batch(bnctx, t.data_ptr(), t.data_ptr(), t.data_ptr(), 1 << 40, 1 << 40, None,
                            None) == bn.BN_ERANGE
    with pytest.raises(bn.BnError):
        bn.bn_set_param(bnctx, "addsub.chain_rows", 3)
    with pytest.raises(bn.BnError):
        bn.bn_set_param(bnctx, "mul.mfma_chunk", 2048)      # beyond the int32 accumulator bound


def test_graph_replay_matches_eager(bnctx):
    announce("graph capture + replay of a batched add")
    n, npairs = 64, 5000
    a, b = wl.c2("add", npairs=npairs)
    ta, tb = D(a), D(b)
    tr = torch.empty_like(ta)
    tc = torch.empty(npairs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    g = bn.bn_graph_capture_batch(bnctx, 0, tr, ta, tb, n, 0, npairs, tc, stream=s)
    rr, rc = oracle.add_batch(a, b, n)
    try:
        for rep in range(4):
            tr.zero_()
            tc.zero_()
            torch.cuda.synchronize()
            bn.bn_graph_launch(g, s)
            s.synchronize()
            assert (H(tr) == rr).all() and (H(tc) == rc).all(), f"replay {rep}"
            # eager work on the same context between replays
            bn.bn_sub_n_batch(bnctx, tr, ta, tb, n, npairs, tc)
            torch.cuda.synchronize()
    finally:
        bn.bn_graph_destroy(g)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_graph_replay_chained(bnctx, op):
    """A captured chained launch (tiles look back; the graph reads its epoch from the
    control block and a bump kernel moves it on) replayed four times, with eager
    chained launches (host epochs) on the same context in between.  All-propagate
    pairs: every tile but the first of a pair waits for its predecessor's carry."""
    n, npairs = 300001, 2
    announce("graph replay, chained", op, f"n={n}", f"npairs={npairs}")
    if op == "add":
        a = np.full(n * npairs, 2 ** 64 - 1, np.uint64)
        b = np.zeros(n * npairs, np.uint64)
        b[::n] = 1
        want, wc = oracle.add_batch(a, b, n)
    else:
        a = np.zeros(n * npairs, np.uint64)
        a[n - 1::n] = 1
        b = np.zeros(n * npairs, np.uint64)
        b[::n] = 1
        want, wc = oracle.sub_batch(a, b, n)
    ta, tb = D(a), D(b)
    tr = torch.empty_like(ta)
    tc = torch.empty(npairs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    g = bn.bn_graph_capture_batch(bnctx, 0 if op == "add" else 1, tr, ta, tb, n, 0, npairs, tc, stream=s)
    try:
        for rep in range(4):
            tr.fill_(7)
            tc.fill_(7)
            torch.cuda.synchronize()
            bn.bn_graph_launch(g, s)
            s.synchronize()
            assert (H(tr) == want).all() and (H(tc) == wc).all(), f"replay {rep}"
            # eager chained work on the same context between replays
            (bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch)(bnctx, tr, ta, tb, n, npairs, tc)
            torch.cuda.synchronize()
            assert (H(tr) == want).all() and (H(tc) == wc).all(), f"eager after replay {rep}"
    finally:
        bn.bn_graph_destroy(g)


def test_graph_replay_large_product(bnctx):
    """A captured large product (column workspace, fold, chained carry pass) replayed
    three times with eager products in between."""
    na, nb, npairs = 700, 600, 3
    announce("graph replay, large product", f"na={na}", f"nb={nb}", f"npairs={npairs}")
    g0 = np.random.default_rng(9)
    a = g0.integers(0, 2 ** 64 - 1, na * npairs, dtype=np.uint64, endpoint=True)
    b = g0.integers(0, 2 ** 64 - 1, nb * npairs, dtype=np.uint64, endpoint=True)
    want = oracle.mul_batch(a, b, na, nb, npairs)
    ta, tb = D(a), D(b)
    for form in ("mad", "mfma"):
        tr = torch.empty((na + nb) * npairs, dtype=torch.int64, device="cuda")
        s = torch.cuda.Stream()
        g = bn.bn_graph_capture_batch(bnctx, 2, tr, ta, tb, na, nb, npairs, None, form, stream=s)
        try:
            for rep in range(3):
                tr.fill_(7)
                torch.cuda.synchronize()
                bn.bn_graph_launch(g, s)
                s.synchronize()
                assert (H(tr) == want).all(), f"{form} replay {rep}"
                bn.bn_mul_n_batch(bnctx, tr, ta, tb, na, nb, npairs, form)
                torch.cuda.synchronize()
                assert (H(tr) == want).all(), f"{form} eager after replay {rep}"
        finally:
            bn.bn_graph_destroy(g)


def test_self_help_lookback_forced_from_host(bnctx):
    """Tile 0 never publishes (debug flag): its successor polls a few times, then
    computes tile 0's carry from the operands itself.  The kernel exits normally,
    the result is exact, and the latch reports that the self-help path ran."""
    announce("self-help look-back")
    old = bn.bn_get_param(bnctx, "lookback.spin_limit")
    try:
        bn.bn_set_param(bnctx, "lookback.spin_limit", 16)
        bn.bn_set_param(bnctx, "debug.flags", 1)
        bn.bn_check(bnctx)
        for op, worst in (("add", True), ("sub", True), ("add", False)):
            a, b = wl.c3(op, n=1 << 16, worst=worst)
            _check(bnctx, op, a, b, a.size, 1)
            assert bn.bn_check(bnctx) & 1
        assert bn.bn_check(bnctx) == 0   # the latch was cleared
    finally:
        bn.bn_set_param(bnctx, "debug.flags", 0)
        bn.bn_set_param(bnctx, "lookback.spin_limit", old)
    a, b = wl.c3("add", n=1 << 16)
    _check(bnctx, "add", a, b, a.size, 1)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_self_help_every_tile(bnctx, op):
    """spin_limit 0: every waiting tile computes its predecessors itself."""
    announce("self-help on every wait", op)
    old = bn.bn_get_param(bnctx, "lookback.spin_limit")
    try:
        bn.bn_set_param(bnctx, "lookback.spin_limit", 0)
        for worst in (False, True):
            a, b = wl.c3(op, n=(1 << 18) + 77, worst=worst)
            _check(bnctx, op, a, b, a.size, 1)
    finally:
        bn.bn_set_param(bnctx, "lookback.spin_limit", old)


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n,npairs", [((1 << 20) + 5, 1), (100003, 7)])
def test_lookback_histogram_counts_every_chained_tile(bnctx, op, n, npairs):
    """With debug flag bit 1 every tile that looks back records one distance: the
    histogram total is the number of tiles that do not start a segment (launches that
    wait: all-propagate tiles of deferred launches do not look back)."""
    announce("look-back histogram", op, f"n={n}", f"npairs={npairs}")
    old = bn.bn_get_param(bnctx, "debug.flags")
    old_defer = bn.bn_get_param(bnctx, "addsub.defer_tiles")
    waves = bn.bn_get_param(bnctx, "addsub.chain_waves")
    rows = bn.bn_get_param(bnctx, "addsub.chain_rows")
    N = n * npairs
    # the launch halves the tuned rows until it has at least 8 tiles per CU
    want = 8 * torch.cuda.get_device_properties(0).multi_processor_count
    while rows > 1 and -(-N // (waves * rows * 128)) < want:
        rows //= 2
    TL = waves * rows * 128
    ntiles = -(-N // TL)
    expect = sum(1 for t in range(1, ntiles) if (t * TL) % n != 0)
    a, b = wl.c3(op, n=N, worst=True)
    bn.bn_lookback_stats(bnctx)  # clear
    try:
        bn.bn_set_param(bnctx, "addsub.defer_tiles", 0)
        bn.bn_set_param(bnctx, "debug.flags", 2)
        _check(bnctx, op, a, b, n, npairs)
        h = bn.bn_lookback_stats(bnctx)
    finally:
        bn.bn_set_param(bnctx, "debug.flags", old)
        bn.bn_set_param(bnctx, "addsub.defer_tiles", old_defer)
    assert sum(h) == expect, (sum(h), expect, h)
    assert all(v == 0 for v in h[max(1, ntiles.bit_length()):]), h
    # not recorded with the flag off
    _check(bnctx, op, a, b, n, npairs)
    assert sum(bn.bn_lookback_stats(bnctx)) == 0


def _in_place_case(ctx, op, a, b, target):
    """r == a (target "a") or r == b (target "b") on one pair; returns (r, carry)."""
    ta, tb = D(a), D(b)
    c = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    r = ta if target == "a" else tb
    (bn.bn_add if op == "add" else bn.bn_sub)(ctx, r, ta, tb, c)
    torch.cuda.synchronize()
    return H(r), int(H(c)[0])


@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("target", ["a", "b"])
def test_in_place_waits_instead_of_self_help(bnctx, op, target):
    """In place, a waiting tile must not compute an unpublished predecessor from the
    operands (that tile may already have overwritten them with sums).  With a spin
    limit of 0 and the silent-tile-0 debug flag, which force self-help on every wait
    of an out-of-place call, in-place calls stay exact and the self-help latch stays
    clear; the same settings out of place still take self-help."""
    old_spin = bn.bn_get_param(bnctx, "lookback.spin_limit")
    old_dbg = bn.bn_get_param(bnctx, "debug.flags")
    try:
        bn.bn_set_param(bnctx, "lookback.spin_limit", 0)
        for dbg in (0, 1):
            bn.bn_set_param(bnctx, "debug.flags", dbg)
            for worst in (False, True):
                n = (1 << 18) + 77
                announce("in place, no self-help", op, f"r={target}", f"n={n}", f"debug={dbg}", f"worst={worst}")
                a, b = wl.c3(op, n=n, worst=worst)
                bn.bn_check(bnctx)
                r, c = _in_place_case(bnctx, op, a, b, target)
                want, wc = (oracle.add if op == "add" else oracle.sub)(a, b)
                assert (r == want).all(), f"first bad limb {np.argmax(r != want)}"
                assert c == wc
                assert bn.bn_check(bnctx) == 0, "in place must never take self-help"
        # out of place with the same settings: self-help runs (the latch is set)
        a, b = wl.c3(op, n=(1 << 18) + 77, worst=True)
        _check(bnctx, op, a, b, a.size, 1)
        assert bn.bn_check(bnctx) & 1
    finally:
        bn.bn_set_param(bnctx, "debug.flags", old_dbg)
        bn.bn_set_param(bnctx, "lookback.spin_limit", old_spin)


def test_in_place_extras_at_spin_limit_zero(bnctx):
    """The in-place forms of the add/sub extras (carry-in batch, unequal lengths with
    r == a, |a - b| with r == a and r == b) at a spin limit of 0."""
    old = bn.bn_get_param(bnctx, "lookback.spin_limit")
    g = np.random.default_rng(44)
    try:
        bn.bn_set_param(bnctx, "lookback.spin_limit", 0)
        n, npairs = 100003, 3
        announce("in-place extras", f"n={n}", f"npairs={npairs}")
        a = np.full(n * npairs, 2 ** 64 - 1, np.uint64)
        a[g.integers(0, n * npairs, 5)] = g.integers(0, 2 ** 63, 5, dtype=np.uint64)
        b = np.zeros(n * npairs, np.uint64)
        cin = np.array([1, 0, 1], np.uint64)
        ta, tb, tci = D(a), D(b), D(cin)
        tco = torch.empty(npairs, dtype=torch.int64, device="cuda")
        bn.bn_add_nc_n_batch(bnctx, ta, ta, tb, n, npairs, tci, tco)
        torch.cuda.synchronize()
        want, wc = oracle.add_nc_batch(a, b, n, cin)
        assert (H(ta) == want).all() and (H(tco) == wc).all()
        na, nb = 300007, 200003
        a = g.integers(0, 2 ** 64 - 1, na, dtype=np.uint64, endpoint=True)
        a[nb:] = 2 ** 64 - 1
        b = np.full(nb, 2 ** 64 - 1, np.uint64)
        ta, tb = D(a), D(b)
        tc = torch.empty(1, dtype=torch.int64, device="cuda")
        bn.bn_add_unequal(bnctx, ta, ta, na, tb, nb, tc)
        torch.cuda.synchronize()
        bext = np.concatenate([b, np.zeros(na - nb, np.uint64)])
        want, wc = oracle.add(a, bext)
        assert (H(ta) == want).all() and int(H(tc)[0]) == wc
        for target in ("a", "b"):
            a, b = wl.c3("sub", n=(1 << 18) + 77, worst=True)
            if target == "b":
                a, b = b, a   # a < b: the result is b - a
            ta, tb = D(a), D(b)
            ts = torch.empty(1, dtype=torch.int64, device="cuda")
            r = ta if target == "a" else tb
            bn.bn_sub_abs_n_batch(bnctx, r, ta, tb, a.size, 1, ts)
            torch.cuda.synchronize()
            neg = int(oracle.sub(a, b)[1])
            want = oracle.sub(b, a)[0] if neg else oracle.sub(a, b)[0]
            assert (H(r) == want).all() and int(H(ts)[0]) == neg, target
    finally:
        bn.bn_set_param(bnctx, "lookback.spin_limit", old)
