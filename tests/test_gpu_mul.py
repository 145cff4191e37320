"""GPU multiplication parity (mad and MFMA forms) against the CPU oracle, bit-exact."""
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


def _rand(g, n):
    return g.integers(0, MAX, n, dtype=np.uint64, endpoint=True)


def _mul_batch(ctx, a, b, na, nb, npairs, form):
    announce("mul", form, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    ta, tb = D(a), D(b)
    tr = torch.full((npairs * (na + nb),), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(ctx, tr, ta, tb, na, nb, npairs, form)
    torch.cuda.synchronize()
    return H(tr)


def _check(ctx, a, b, na, nb, npairs, form):
    r = _mul_batch(ctx, a, b, na, nb, npairs, form)
    rr = oracle.mul_batch(a, b, na, nb, npairs)
    bad = np.nonzero(r != rr)[0]
    assert bad.size == 0, f"{form} na={na} nb={nb}: {bad.size} bad limbs, first at {bad[0]}"


SMALL = [(1, 1), (1, 2), (2, 1), (3, 5), (4, 4), (5, 5), (8, 8), (13, 29), (31, 33), (32, 32), (63, 1),
         (64, 64), (100, 28), (37, 91), (127, 1), (1, 255), (255, 1), (128, 128), (120, 136)]


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("na,nb", SMALL)
def test_small_random(bnctx, form, na, nb):
    g = np.random.default_rng(na * 1000 + nb)
    npairs = 37
    _check(bnctx, _rand(g, na * npairs), _rand(g, nb * npairs), na, nb, npairs, form)


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("n", [1, 4, 16, 100, 128])
def test_small_pathological(bnctx, form, n):
    pa, pb = wl.pathological(n, 2, seed=n)
    _check(bnctx, pa.reshape(-1), pb.reshape(-1), n, n, pa.shape[0], form)


LARGE = [(129, 128), (300, 1), (1, 300), (257, 3), (3, 257), (256, 256), (200, 312), (500, 500), (511, 513),
         (1000, 24), (7, 1017), (512, 512), (513, 512), (1000, 999), (1024, 1024), (4099, 1031), (1031, 4099),
         (4096, 4096)]


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("na,nb", LARGE)
def test_large_random(bnctx, form, na, nb):
    g = np.random.default_rng(na * 7919 + nb)
    npairs = 3
    _check(bnctx, _rand(g, na * npairs), _rand(g, nb * npairs), na, nb, npairs, form)


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("n", [300, 480, 2048])
def test_large_pathological(bnctx, form, n):
    pa, pb = wl.pathological(n, 1, seed=n)
    _check(bnctx, pa.reshape(-1), pb.reshape(-1), n, n, pa.shape[0], form)


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("na,nb,npairs", [(1000, 24, 3), (600, 700, 2), (3000, 2000, 1), (40, 30, 9)])
def test_misaligned_operands(bnctx, form, na, nb, npairs):
    """Operands and product one limb into their buffers (8-byte but not 16-byte
    aligned): the operand conversion and carry scans take their 8-byte-load shapes;
    the limb before the product stays untouched."""
    announce("mul misaligned", form, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    g = np.random.default_rng(na + 7 * nb)
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    ta = torch.zeros(na * npairs + 1, dtype=torch.int64, device="cuda")
    tb = torch.zeros(nb * npairs + 1, dtype=torch.int64, device="cuda")
    ta[1:] = D(a)
    tb[1:] = D(b)
    tr = torch.full((npairs * (na + nb) + 1,), -1, dtype=torch.int64, device="cuda")
    bn.bn_mul_n_batch(bnctx, tr[1:], ta[1:], tb[1:], na, nb, npairs, form)
    torch.cuda.synchronize()
    r = H(tr)
    assert int(r[0]) == 2 ** 64 - 1
    assert (r[1:] == oracle.mul_batch(a, b, na, nb, npairs)).all()


@pytest.mark.parametrize("form", ["mad", "mfma"])
def test_c1(bnctx, form):
    a, b = wl.c1("mul")
    _check(bnctx, a, b, 4, 4, 1088, form)


@pytest.mark.parametrize("form", ["mad", "mfma"])
def test_c5_reduced(bnctx, form):
    a, b = wl.c5(npairs=3, n=16384)
    _check(bnctx, a, b, 16384, 16384, 3, form)


def _residues_ok(a, b, r, n, npairs):
    for p in range(npairs):
        A = to_int(a[p * n:(p + 1) * n])
        B = to_int(b[p * n:(p + 1) * n])
        R = to_int(r[p * 2 * n:(p + 1) * 2 * n])
        for q in (65537, 998244353, (1 << 61) - 1, (1 << 64) - 1):
            if (A % q) * (B % q) % q != R % q:
                return p
    return -1


@pytest.mark.parametrize("form", ["mad", "mfma"])
def test_c5_full(bnctx, c5_oracle, form):
    """64 pairs x 16384 limbs (incl. all-ones x all-ones and zero x zero): every limb of
    every product against the oracle; residues as an extra check."""
    n, npairs = 16384, 64
    a, b, want = c5_oracle
    announce("C5 full", form)
    r = _mul_batch(bnctx, a, b, n, n, npairs, form)
    bad = np.flatnonzero(r != want)
    assert bad.size == 0, f"{bad.size} limbs differ, first at pair {bad[0] // (2 * n)} limb {bad[0] % (2 * n)}"
    assert _residues_ok(a, b, r, n, npairs) == -1


def _ragged_inputs(npairs, seed=0):
    a, b, desc, rsz = wl.c4(npairs=npairs, seed=seed)
    return a, b, desc, rsz


@pytest.mark.parametrize("form", ["auto", "mad", "mfma"])
def test_ragged_c4_reduced(bnctx, form):
    a, b, desc, rsz = _ragged_inputs(3000, seed=1)
    announce("ragged mul", form, "npairs=3000")
    plan = bn.bn_plan_mul_ragged(bnctx, desc, form)
    try:
        ta, tb = D(a), D(b)
        tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
        bn.bn_mul_ragged(bnctx, plan, tr, ta, tb)
        torch.cuda.synchronize()
        rr = oracle.mul_ragged(a, b, desc, rsz)
        assert (H(tr) == rr).all()
    finally:
        bn.bn_plan_destroy(plan)


def test_ragged_unsorted_sparse_and_large_items(bnctx):
    """Pairs in arbitrary pool positions, including ones beyond the one-wave limit."""
    announce("ragged mul: mixed sizes")
    g = np.random.default_rng(4)
    sizes = [(1, 1), (300, 20), (4, 4), (128, 128), (1, 255), (700, 900), (33, 2), (2, 33), (256, 1)]
    a_off = b_off = r_off = 0
    desc, A, B = [], [], []
    for na, nb in sizes:
        gap = int(g.integers(0, 3))
        a_off += gap
        b_off += gap
        r_off += gap
        desc.append((a_off, b_off, r_off, na, nb))
        a_off += na
        b_off += nb
        r_off += na + nb
    a = _rand(g, a_off)
    b = _rand(g, b_off)
    desc = np.array(desc, np.uint64)
    for form in ("mad", "mfma", "auto"):
        plan = bn.bn_plan_mul_ragged(bnctx, desc, form)
        try:
            tr = torch.zeros(r_off, dtype=torch.int64, device="cuda")
            bn.bn_mul_ragged(bnctx, plan, tr, D(a), D(b))
            torch.cuda.synchronize()
            rr = oracle.mul_ragged(a, b, desc, r_off)
            assert (H(tr) == rr).all(), form
        finally:
            bn.bn_plan_destroy(plan)


def test_ragged_c4_full_graph_replay(bnctx):
    """2^16 ragged pairs in one persistent launch captured in a HIP graph (one form, or
    both forms in one launch for auto), replayed with eager work in between; every
    replay equals the oracle."""
    a, b, desc, rsz = _ragged_inputs(1 << 16)
    rr = oracle.mul_ragged(a, b, desc, rsz)
    ta, tb = D(a), D(b)
    tr = torch.zeros(rsz, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    for form in ("mad", "mfma", "auto"):
        announce("ragged mul graph", form)
        plan = bn.bn_plan_mul_ragged(bnctx, desc, form)
        g = bn.bn_graph_capture_mul_ragged(bnctx, plan, tr, ta, tb, s)
        try:
            for rep in range(3):
                tr.fill_(-1)
                torch.cuda.synchronize()
                bn.bn_graph_launch(g, s)
                s.synchronize()
                assert (H(tr) == rr).all(), f"{form} replay {rep}"
                bn.bn_mul_ragged(bnctx, plan, tr, ta, tb)   # eager, same plan
                torch.cuda.synchronize()
                assert (H(tr) == rr).all(), f"{form} eager {rep}"
        finally:
            bn.bn_graph_destroy(g)
            bn.bn_plan_destroy(plan)


def _check_pool(got, want, desc, what):
    """Item limbs equal the oracle's; limbs between items keep the -1 fill (nothing is
    written outside a product)."""
    inside = np.zeros(got.size, bool)
    for _, _, ro, na, nb in desc:
        inside[int(ro):int(ro) + int(na) + int(nb)] = True
    bad = np.flatnonzero(inside & (got != want))
    assert bad.size == 0, f"{what}: {bad.size} limbs differ, first at {bad[0]}"
    assert (got[~inside] == np.uint64(MAX)).all(), f"{what}: a limb outside every product was written"


def _tiny_ragged(g, shapes):
    """Pool layout for the given (na, nb) shapes, gaps between them; every 5th item all-ones."""
    desc, a_off, b_off, r_off = [], 0, 0, 0
    for na, nb in shapes:
        gap = int(g.integers(0, 2))
        a_off, b_off, r_off = a_off + gap, b_off + gap, r_off + gap
        desc.append((a_off, b_off, r_off, na, nb))
        a_off, b_off, r_off = a_off + na, b_off + nb, r_off + na + nb
    a, b = _rand(g, a_off), _rand(g, b_off)
    for i in range(0, len(desc), 5):
        ao, bo, _, na, nb = desc[i]
        a[ao:ao + na] = MAX
        b[bo:bo + nb] = MAX
    return a, b, np.array(desc, np.uint64), r_off


@pytest.mark.parametrize("pair", [1, 0])
@pytest.mark.parametrize("form", ["auto", "mad"])
def test_ragged_small_mad_pairs(bnctx, form, pair):
    """Mad items of at most 32 product limbs run two to a wave when their shorter operands
    have equal length (ragged.pair_small 1, the default): couples at every shorter length
    1..16, products of exactly 32 limbs, items of 33 limbs beside them (never paired),
    items left without a partner, the larger operand first or second, all-ones items (the
    longest carries); every limb against the oracle, and the same with pairing off."""
    g = np.random.default_rng(21 + pair)
    shapes = []
    for s in range(1, 17):
        for _ in range(int(g.integers(1, 6))):  # odd counts leave an item without a partner
            l = int(g.integers(s, 33 - s + 1))  # longer operand: product of at most 32 limbs
            shapes.append((s, l) if g.integers(0, 2) else (l, s))
    shapes += [(16, 16), (16, 16), (1, 31), (31, 1), (17, 16), (16, 17), (1, 32), (32, 1), (20, 13)]
    shapes += [(int(x), int(y)) for x, y in g.integers(1, 30, (300, 2))]
    order = g.permutation(len(shapes))
    a, b, desc, rsz = _tiny_ragged(g, [shapes[i] for i in order])
    announce("ragged mul: small mad pairs", form, f"pair={pair}", f"items={len(desc)}")
    old = bn.bn_get_param(bnctx, "ragged.pair_small")
    bn.bn_set_param(bnctx, "ragged.pair_small", pair)
    try:
        plan = bn.bn_plan_mul_ragged(bnctx, desc, form)
    finally:
        bn.bn_set_param(bnctx, "ragged.pair_small", old)
    try:
        tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
        bn.bn_mul_ragged(bnctx, plan, tr, D(a), D(b))
        torch.cuda.synchronize()
        _check_pool(H(tr), oracle.mul_ragged(a, b, desc, rsz), desc, f"{form} pair={pair}")
    finally:
        bn.bn_plan_destroy(plan)


def test_ragged_pairs_and_mfma_items(bnctx):
    """Couples of small mad items beside MFMA items and no single mad item (the mixed
    kernel runs the couples, then a list of MFMA items only)."""
    g = np.random.default_rng(24)
    shapes = [(5, 9), (9, 5), (11, 21), (21, 11)] * 30 + [(28, 100), (40, 40), (64, 64), (128, 100), (30, 226)] * 12
    order = g.permutation(len(shapes))
    a, b, desc, rsz = _tiny_ragged(g, [shapes[i] for i in order])
    announce("ragged mul: couples and MFMA items", f"items={len(desc)}")
    plan = bn.bn_plan_mul_ragged(bnctx, desc, "auto")
    try:
        tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
        bn.bn_mul_ragged(bnctx, plan, tr, D(a), D(b))
        torch.cuda.synchronize()
        _check_pool(H(tr), oracle.mul_ragged(a, b, desc, rsz), desc, "couples + MFMA")
    finally:
        bn.bn_plan_destroy(plan)


def test_ragged_only_pairs(bnctx):
    """A batch of nothing but pairable items (one kernel path: couples, no single items),
    captured in a graph and replayed."""
    g = np.random.default_rng(23)
    shapes = [(7, 9), (9, 7), (7, 25), (3, 3), (3, 29), (12, 20), (20, 12)] * 40
    a, b, desc, rsz = _tiny_ragged(g, shapes)
    announce("ragged mul: pairs only", f"items={len(desc)}")
    rr = oracle.mul_ragged(a, b, desc, rsz)
    ta, tb = D(a), D(b)
    tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    plan = bn.bn_plan_mul_ragged(bnctx, desc, "mad")
    g_ = bn.bn_graph_capture_mul_ragged(bnctx, plan, tr, ta, tb, s)
    try:
        for rep in range(2):
            tr.fill_(-1)
            torch.cuda.synchronize()
            bn.bn_graph_launch(g_, s)
            s.synchronize()
            _check_pool(H(tr), rr, desc, f"replay {rep}")
    finally:
        bn.bn_graph_destroy(g_)
        bn.bn_plan_destroy(plan)


def test_ragged_add(bnctx):
    announce("ragged add")
    g = np.random.default_rng(8)
    ns = [1, 5, 128, 129, 1000, 3, 64, 0, 77]
    desc, off = [], 0
    for n in ns:
        desc.append((off, off, off, n, n))
        off += n
    a, b = _rand(g, off), _rand(g, off)
    pa, pb = wl.pathological(129, 1, seed=2)
    a[5 + 1:5 + 1 + 129] = pa[0]
    b[5 + 1:5 + 1 + 129] = pb[0]
    desc = np.array(desc, np.uint64)
    plan = bn.bn_plan_add_ragged(bnctx, desc)
    try:
        tr = torch.zeros(off, dtype=torch.int64, device="cuda")
        tc = torch.full((len(ns),), -1, dtype=torch.int64, device="cuda")
        bn.bn_add_ragged(bnctx, plan, tr, D(a), D(b), tc)
        torch.cuda.synchronize()
        r, c = H(tr), H(tc)
        o = 0
        for i, n in enumerate(ns):
            rr, cc = oracle.add(a[o:o + n], b[o:o + n])
            assert (r[o:o + n] == rr).all() and int(c[i]) == cc, i
            o += n
    finally:
        bn.bn_plan_destroy(plan)


def test_ragged_plan_offset_range(bnctx):
    """Descriptors whose offset plus length would pass 2^60 limbs are refused at plan time."""
    announce("ragged plan offset range")
    top = (1 << 60) - 8
    for bad in ((top, 0, 0, 9, 4), (0, top, 0, 4, 9), (0, 0, top, 4, 5), ((1 << 64) - 1, 0, 0, 1, 1)):
        desc = np.array([(0, 0, 0, 4, 4), bad], np.uint64)
        with pytest.raises(bn.BnError) as e:
            bn.bn_plan_mul_ragged(bnctx, desc)
        assert e.value.status == bn.BN_ERANGE, bad
        add = desc.copy()   # one length n for a, b and r
        add[1, 3] = add[1, 4] = 9 if top in bad else 1
        with pytest.raises(bn.BnError) as e:
            bn.bn_plan_add_ragged(bnctx, add)
        assert e.value.status == bn.BN_ERANGE, bad
    # the largest offsets that still fit are accepted (nothing is launched)
    ok = np.array([(top, top, top - 8, 8, 8)], np.uint64)
    for plan in (bn.bn_plan_mul_ragged(bnctx, ok), bn.bn_plan_add_ragged(bnctx, ok)):
        bn.bn_plan_destroy(plan)


def test_mul_errors(bnctx):
    announce("mul argument errors")
    t = torch.zeros(64, dtype=torch.int64, device="cuda")
    # tensors smaller than the extents a call touches are refused by the binding
    # before anything reaches the device
    with pytest.raises(ValueError):
        bn.bn_mul_n_batch(bnctx, t[:15], t[16:24], t[24:32], 4, 4, 2)   # r needs 16 limbs
    with pytest.raises(ValueError):
        bn.bn_mul_n_batch(bnctx, t[:16], t[16:23], t[24:32], 4, 4, 2)   # a needs 8
    with pytest.raises(ValueError):
        bn.bn_add_n_batch(bnctx, t[:8], t[8:16], t[16:24], 4, 2, t[24:25])  # 2 carries
    with pytest.raises(ValueError):
        bn.bn_mul_karatsuba_n_batch(bnctx, t[:15], t[32:40], t[40:48], 4, 2, 1)  # r needs 16
    with pytest.raises(bn.BnError) as e:
        bn.bn_mul(bnctx, t[16:24], t[0:4], t[8:12], form=7)
    assert e.value.status == bn.BN_EINVAL
    z = torch.empty(0, dtype=torch.int64, device="cuda")
    r = torch.full((5,), 3, dtype=torch.int64, device="cuda")
    bn.bn_mul(bnctx, r, z, t[0:5])                     # 0 limbs x 5 limbs = 0 (5 limbs)
    torch.cuda.synchronize()
    assert (H(r) == 0).all()


def most_negative_digits(n):
    """The n-limb operand whose balanced digits are all -128 (top digit 1):
    2^(64 n) - 0x80...80 = 0x7f...7f80.  Squared, every digit product is +2^14 and a
    middle column reaches 2^14 (8 n) -- past int32 from n = 16384 limbs."""
    x = np.full(n, 0x7F7F7F7F7F7F7F7F, np.uint64)
    x[0] = 0x7F7F7F7F7F7F7F80
    return x


@pytest.mark.parametrize("form", ["mfma", "mad"])
def test_beyond_single_range_bound(bnctx, form):
    """min(na, nb) > 16448 limbs: a column can hold more than 131586 digit products, so
    the MFMA form must cut the contraction into slices of at most 2046 steps.  Includes
    the most-negative-digit square (every signed digit product is +2^14), zero and
    all-ones."""
    n = 16500
    g = np.random.default_rng(77)
    w = most_negative_digits(n)
    a = np.concatenate([w, np.zeros(n, np.uint64), np.full(n, 2 ** 64 - 1, np.uint64), _rand(g, n)])
    b = np.concatenate([w, np.zeros(n, np.uint64), np.full(n, 2 ** 64 - 1, np.uint64), _rand(g, n)])
    _check(bnctx, a, b, n, n, 4, form)


@pytest.mark.parametrize("n", [16384, 16448])
def test_int32_wrap_decode(bnctx, n):
    """Unsplit MFMA launches up to 16448 limbs: the most-negative-digit square drives a
    column to 2^14 (8 n) >= 2^31, which the int32 register holds wrapped and the
    epilogue recovers (16448: the largest n with at most 131586 digit pairs a column).
    64 pairs give about four workgroups per CU, so the contraction is not split (the
    workspace holds no slice sums, checked below; split slices are exact and never
    wrap).  Pairs 0 and 1 (worst x worst, worst x random) against the oracle, every
    pair by residues."""
    npairs = 64
    ws = bn.bn_workspace_size(bnctx, bn.BN_OP_MUL, n, n, npairs, bn.BN_MUL_MFMA)
    # converted operands, their top digits, lo and shifted hi; a split would add at
    # least two slices of int32 column sums (2 * npairs * 8 * 2n * 4 bytes)
    assert ws < 8 * npairs * (n + n + 2 + 2 * 2 * n) + (1 << 20), ws
    g = np.random.default_rng(n)
    w = most_negative_digits(n)
    a = np.concatenate([w, w] + [_rand(g, n) for _ in range(npairs - 2)])
    b = np.concatenate([w, _rand(g, n)] + [_rand(g, n) for _ in range(npairs - 2)])
    r = _mul_batch(bnctx, a, b, n, n, npairs, "mfma")
    for p in (0, 1):
        rr = oracle.mul(a[p * n:(p + 1) * n], b[p * n:(p + 1) * n])
        bad = np.nonzero(r[p * 2 * n:(p + 1) * 2 * n] != rr)[0]
        assert bad.size == 0, f"pair {p}: {bad.size} bad limbs, first at {bad[0]}"
    assert _residues_ok(a, b, r, n, npairs) == -1


@pytest.mark.parametrize("form", ["mfma", "mad"])
@pytest.mark.parametrize("na,nb", [(16384, 16384), (8192, 8192), (20000, 1000)])
def test_single_large_pair(bnctx, form, na, nb):
    """One pair: the launch has few column groups, so the contraction is split across
    workgroups (MFMA) or into small slices (mad)."""
    g = np.random.default_rng(na + nb)
    _check(bnctx, _rand(g, na), _rand(g, nb), na, nb, 1, form)


@pytest.mark.parametrize("form", ["mad", "mfma"])
def test_many_large_pairs(bnctx, form):
    """More pairs than one grid dimension holds (65535) on the column-workspace path."""
    na, nb, npairs = 150, 131, 70000
    g = np.random.default_rng(7)
    _check(bnctx, _rand(g, na * npairs), _rand(g, nb * npairs), na, nb, npairs, form)


@pytest.mark.parametrize("form", ["mfma", "mad"])
def test_graph_survives_workspace_growth(form):
    """A captured product keeps its buffers when later eager calls outgrow them: on a
    fresh context, capture a product on the workspace path (plus one computed in place,
    which goes through the staging buffer), grow the workspace, the status array and
    the staging buffer twice with much larger eager products, and replay after each."""
    na, nb, npairs = 700, 600, 3
    announce("graph after workspace growth", form, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    fcode = bn.BN_MUL_MFMA if form == "mfma" else bn.BN_MUL_MAD
    g0 = np.random.default_rng(12)
    a, b = _rand(g0, na * npairs), _rand(g0, nb * npairs)
    want = oracle.mul_batch(a, b, na, nb, npairs)
    R = (na + nb) * npairs
    ctx = bn.bn_create(0)
    try:
        assert bn.bn_workspace_size(ctx, bn.BN_OP_MUL, 8192, 8192, 4, fcode) > 2 * bn.bn_workspace_size(ctx, bn.BN_OP_MUL, na, nb, npairs, fcode)
        s = torch.cuda.Stream()
        ta, tb = D(a), D(b)
        tr = torch.empty(R, dtype=torch.int64, device="cuda")
        buf = torch.zeros(R + nb * npairs, dtype=torch.int64, device="cuda")   # r over a, b behind
        ri, ai, bi = buf[:R], buf[:na * npairs], buf[R:]
        g = bn.bn_graph_capture_batch(ctx, 2, tr, ta, tb, na, nb, npairs, None, form, stream=s)
        gi = bn.bn_graph_capture_batch(ctx, 2, ri, ai, bi, na, nb, npairs, None, form, stream=s)
        try:
            for big in (8192, 16384):
                # grow the workspace, the status array and the staging buffer
                bn.bn_reserve_for(ctx, bn.BN_OP_MUL | bn.BN_OP_IN_PLACE, big, big, 4, fcode)
                x = D(_rand(g0, big * 4))
                xr = torch.empty(2 * big * 4, dtype=torch.int64, device="cuda")
                bn.bn_mul_n_batch(ctx, xr, x, x, big, big, 4, form)
                xs = torch.zeros(2 * big * 4, dtype=torch.int64, device="cuda")
                xs[:big * 4].copy_(x)
                bn.bn_mul_n_batch(ctx, xs, xs[:big * 4], x, big, big, 4, form)            # in place
                torch.cuda.synchronize()
                tr.fill_(7)
                buf.zero_()
                ai.copy_(ta)
                bi.copy_(tb)
                torch.cuda.synchronize()
                bn.bn_graph_launch(g, s)
                bn.bn_graph_launch(gi, s)
                s.synchronize()
                assert (H(tr) == want).all(), f"replay after growth to {big}"
                assert (H(ri) == want).all(), f"in-place replay after growth to {big}"
                del x, xr, xs
        finally:
            bn.bn_graph_destroy(g)
            bn.bn_graph_destroy(gi)
    finally:
        torch.cuda.synchronize()
        bn.bn_destroy(ctx)


@pytest.mark.parametrize("p256,p512,p1024", [(1, 1, 1), (1 << 30, 1 << 30, 1 << 30), (1, 1 << 30, 1),
                                              (2, 2, 40), (-1, -1, -1)])
def test_crossover_classes_256_512_1024(bnctx, p256, p512, p1024):
    """The automatic form's crossovers for products of 129-256, 257-512 and 513-1024
    limbs at either extreme, the defaults and the small crossover (-1): skewed and square
    uniform batches of each class, and ragged items of 257-1024 limbs (batched path per
    item), against the oracle."""
    announce("crossover classes 256/512/1024", p256, p512, p1024)
    keys = ("mul.crossover_limbs_p256", "mul.crossover_limbs_p512", "mul.crossover_limbs_p1024")
    old = tuple(bn.bn_get_param(bnctx, k) for k in keys)
    try:
        for k, v in zip(keys, (p256, p512, p1024)):
            bn.bn_set_param(bnctx, k, v)
        g = np.random.default_rng(abs(p256) * 7 + abs(p512) + abs(p1024) * 3)
        for na, nb, npairs in ((150, 8, 20), (4, 250, 9), (128, 128, 5), (200, 30, 7),
                               (300, 4, 11), (12, 480, 5), (256, 256, 3), (400, 100, 3),
                               (700, 40, 3), (28, 990, 2), (600, 16, 3), (512, 512, 2)):
            _check(bnctx, _rand(g, na * npairs), _rand(g, nb * npairs), na, nb, npairs, "auto")
        a, b, desc, rsz = _tiny_ragged(g, [(300, 4), (4, 300), (256, 200), (500, 12), (20, 20), (130, 9),
                                           (700, 40), (30, 900)])
        plan = bn.bn_plan_mul_ragged(bnctx, desc, "auto")
        try:
            tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
            bn.bn_mul_ragged(bnctx, plan, tr, D(a), D(b))
            torch.cuda.synchronize()
            _check_pool(H(tr), oracle.mul_ragged(a, b, desc, rsz), desc, "ragged 257-1024")
        finally:
            bn.bn_plan_destroy(plan)
    finally:
        for k, v in zip(keys, old):
            bn.bn_set_param(bnctx, k, v)


@pytest.mark.parametrize("p64,p128", [(1, 1), (1, 1 << 30), (1 << 30, 1), (12, 20)])
def test_crossover_classes(bnctx, p64, p128):
    """The automatic form's crossovers for one-wave products of at most 64 and of 65-128
    limbs, pushed to either extreme (every product of the class on MFMA with its one
    column block, or on mad): the full 2^16-pair ragged batch and uniform batches of
    each class stay exact."""
    announce("crossover classes", p64, p128)
    old = (bn.bn_get_param(bnctx, "mul.crossover_limbs_p64"), bn.bn_get_param(bnctx, "mul.crossover_limbs_p128"))
    try:
        bn.bn_set_param(bnctx, "mul.crossover_limbs_p64", p64)
        bn.bn_set_param(bnctx, "mul.crossover_limbs_p128", p128)
        a, b, desc, rsz = _ragged_inputs(1 << 16, seed=4)
        plan = bn.bn_plan_mul_ragged(bnctx, desc, "auto")
        try:
            tr = torch.full((rsz,), -1, dtype=torch.int64, device="cuda")
            bn.bn_mul_ragged(bnctx, plan, tr, D(a), D(b))
            torch.cuda.synchronize()
            assert (H(tr) == oracle.mul_ragged(a, b, desc, rsz)).all()
        finally:
            bn.bn_plan_destroy(plan)
        g = np.random.default_rng(p64 + p128)
        for na, nb, npairs in ((3, 61, 70), (32, 32, 50), (40, 88, 33), (64, 64, 20), (100, 28, 9)):
            _check(bnctx, _rand(g, na * npairs), _rand(g, nb * npairs), na, nb, npairs, "auto")
    finally:
        bn.bn_set_param(bnctx, "mul.crossover_limbs_p64", old[0])
        bn.bn_set_param(bnctx, "mul.crossover_limbs_p128", old[1])
