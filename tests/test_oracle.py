"""Pins of the CPU oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something it does not share code with:
CPython's arbitrary-precision int, closed forms, algebraic identities, residues
computed limb-by-limb, emulations of the paper's DoT phases (Sec. 3.1 add,
Sec. 3.2 vertical-and-crosswise mul), and brute force of the Appendix B
carry lemmas.  A dropped carry, a wrong borrow, an off-by-one column or a
transposed operand in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

from _bigint import MASK64, from_int, to_int

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SPECIALS = [0, 1, 2, (1 << 63) - 1, 1 << 63, MASK64 - 1, MASK64, 0x0123456789ABCDEF]


def _rand(g, n):
    return g.integers(0, MASK64, size=n, dtype=np.uint64, endpoint=True)


# ----------------------------------------------------------------------------------------
# against CPython int
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2])
def test_add_sub_specials_exhaustive(oracle_mod, n):
    import itertools
    mod = 1 << (64 * n)
    vals = SPECIALS if n == 1 else [0, 1, MASK64, 1 << 63]
    for la in itertools.product(vals, repeat=n):
        for lb in itertools.product(vals, repeat=n):
            a = np.array(la, np.uint64)
            b = np.array(lb, np.uint64)
            A, B = to_int(a), to_int(b)
            r, c = oracle_mod.add(a, b)
            assert to_int(r) == (A + B) % mod and c == (A + B) // mod
            r, c = oracle_mod.sub(a, b)
            assert to_int(r) == (A - B) % mod and c == int(A < B)


def test_mul_1x1_specials(oracle_mod):
    for x in SPECIALS:
        for y in SPECIALS:
            r = oracle_mod.mul(np.array([x], np.uint64), np.array([y], np.uint64))
            assert to_int(r) == x * y


@pytest.mark.parametrize("n", list(range(0, 40)) + [63, 64, 65, 127, 128, 129, 300, 1000])
def test_add_sub_random_vs_int(oracle_mod, n):
    g = np.random.default_rng(1000 + n)
    mod = 1 << (64 * n)
    for _ in range(4):
        a, b = _rand(g, n), _rand(g, n)
        A, B = to_int(a), to_int(b)
        r, c = oracle_mod.add(a, b)
        assert to_int(r) == (A + B) % mod and c == (A + B) // mod
        r, c = oracle_mod.sub(a, b)
        assert to_int(r) == (A - B) % mod and c == int(A < B)


@pytest.mark.parametrize("n", [1, 2, 5, 33])
def test_carry_in_variants_vs_int(oracle_mod, n):
    """Carry (borrow) into limb 0: r = a + b + c, c_out = floor(.../X^n); r = a - b - c
    with a borrow out when it is negative.  Includes the all-ones / zero operands
    where the carry-in alone crosses every limb."""
    g = np.random.default_rng(77 + n)
    mod = 1 << (64 * n)
    ones, zero = np.full(n, MASK64, np.uint64), np.zeros(n, np.uint64)
    cases = [(_rand(g, n), _rand(g, n)) for _ in range(5)] + [(ones, zero), (zero, zero), (zero, ones),
                                                                (ones, ones)]
    a = np.concatenate([x for x, _ in cases] * 2)
    b = np.concatenate([y for _, y in cases] * 2)
    cin = np.array([0] * len(cases) + [1] * len(cases), np.uint64)
    r, c = oracle_mod.add_nc_batch(a, b, n, cin)
    r2, c2 = oracle_mod.sub_nc_batch(a, b, n, cin)
    for p in range(2 * len(cases)):
        A, B, C = to_int(a[p * n:(p + 1) * n]), to_int(b[p * n:(p + 1) * n]), int(cin[p])
        assert to_int(r[p * n:(p + 1) * n]) == (A + B + C) % mod and int(c[p]) == (A + B + C) // mod
        assert to_int(r2[p * n:(p + 1) * n]) == (A - B - C) % mod and int(c2[p]) == int(A - B - C < 0)


@pytest.mark.parametrize("na,nb", [(0, 3), (3, 0), (1, 1), (1, 7), (7, 1), (4, 4), (5, 5), (13, 29),
                                   (64, 64), (100, 37), (128, 128), (257, 129)])
def test_mul_random_vs_int(oracle_mod, na, nb):
    g = np.random.default_rng(7 * na + nb)
    for _ in range(3):
        a, b = _rand(g, na), _rand(g, nb)
        r = oracle_mod.mul(a, b)
        assert r.size == na + nb
        assert to_int(r) == to_int(a) * to_int(b)


def test_batch_and_ragged_vs_int(oracle_mod):
    g = np.random.default_rng(5)
    n, npairs = 9, 17
    a, b = _rand(g, n * npairs), _rand(g, n * npairs)
    ra, ca = oracle_mod.add_batch(a, b, n)
    rs, cs = oracle_mod.sub_batch(a, b, n)
    for p in range(npairs):
        A, B = to_int(a[p * n:(p + 1) * n]), to_int(b[p * n:(p + 1) * n])
        assert to_int(ra[p * n:(p + 1) * n]) + (int(ca[p]) << (64 * n)) == A + B
        assert to_int(rs[p * n:(p + 1) * n]) - (int(cs[p]) << (64 * n)) == A - B
    rm = oracle_mod.mul_batch(a, b, n, n, npairs)
    for p in range(npairs):
        A, B = to_int(a[p * n:(p + 1) * n]), to_int(b[p * n:(p + 1) * n])
        assert to_int(rm[p * 2 * n:(p + 1) * 2 * n]) == A * B
    # ragged: sizes differ per pair, pools packed
    sizes = [(1, 5), (4, 4), (17, 3), (2, 30)]
    a_off = b_off = r_off = 0
    desc, A, B = [], [], []
    for na, nb in sizes:
        desc.append((a_off, b_off, r_off, na, nb))
        A.append(_rand(g, na))
        B.append(_rand(g, nb))
        a_off += na
        b_off += nb
        r_off += na + nb
    r = oracle_mod.mul_ragged(np.concatenate(A), np.concatenate(B), np.array(desc, np.uint64), r_off)
    for (ao, bo, ro, na, nb), x, y in zip(desc, A, B):
        assert to_int(r[ro:ro + na + nb]) == to_int(x) * to_int(y)


# ----------------------------------------------------------------------------------------
# closed forms (all-ones carry-chain worst cases)
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 64, 257])
def test_closed_forms(oracle_mod, n):
    ones = np.full(n, MASK64, np.uint64)
    one = np.zeros(n, np.uint64)
    one[0] = 1
    # (2^(64n)-1) + 1 = 2^(64n): all limbs 0, carry 1
    r, c = oracle_mod.add(ones, one)
    assert not r.any() and c == 1
    # (2^(64n)-1) + (2^(64n)-1) = 2^(64n+1) - 2: limb0 = 0xFF..FE, others 0xFF..FF, carry 1
    r, c = oracle_mod.add(ones, ones)
    assert int(r[0]) == MASK64 - 1 and (r[1:] == np.uint64(MASK64)).all() and c == 1
    # 2^(64k) - 1 on k+1 limbs: k limbs of 0xFF..FF then 0, borrow 0 (full borrow chain)
    pw = np.zeros(n + 1, np.uint64)
    pw[n] = 1
    one1 = np.zeros(n + 1, np.uint64)
    one1[0] = 1
    r, c = oracle_mod.sub(pw, one1)
    assert (r[:n] == np.uint64(MASK64)).all() and int(r[n]) == 0 and c == 0
    # 0 - 1 wraps to all-ones with borrow 1
    r, c = oracle_mod.sub(np.zeros(n, np.uint64), one)
    assert (r == np.uint64(MASK64)).all() and c == 1
    # (2^(64n)-1)^2 = X^(2n) - 2 X^n + 1: r0 = 1, r1..r_{n-1} = 0, r_n = 0xFF..FE, rest 0xFF..FF
    r = oracle_mod.mul(ones, ones)
    assert int(r[0]) == 1 and not r[1:n].any()
    assert int(r[n]) == MASK64 - 1 and (r[n + 1:] == np.uint64(MASK64)).all()


@pytest.mark.parametrize("N,M", [(64, 64), (100, 37), (128, 1), (1000, 999), (4096, 64 * 33)])
def test_closed_form_mersenne_product(oracle_mod, N, M):
    # (2^N - 1)(2^M - 1) = 2^(N+M) - 2^N - 2^M + 1
    na, nb = (N + 63) // 64, (M + 63) // 64
    a = from_int((1 << N) - 1, na)
    b = from_int((1 << M) - 1, nb)
    r = oracle_mod.mul(a, b)
    assert to_int(r) == (1 << (N + M)) - (1 << N) - (1 << M) + 1


# ----------------------------------------------------------------------------------------
# algebraic identities
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 16, 65])
def test_identities(oracle_mod, n):
    g = np.random.default_rng(31 + n)
    for _ in range(5):
        a, b, c = _rand(g, n), _rand(g, n), _rand(g, n)
        # a + b = b + a
        r1, c1 = oracle_mod.add(a, b)
        r2, c2 = oracle_mod.add(b, a)
        assert (r1 == r2).all() and c1 == c2
        # (a + b) - b = a, on n+1 limbs
        s = np.append(r1, np.uint64(c1))
        d, br = oracle_mod.sub(s, np.append(b, np.uint64(0)))
        assert (d[:n] == a).all() and int(d[n]) == 0 and br == 0
        # (a - b) + b = a mod 2^(64n), and borrow-out equals carry-out of the re-add
        d, br = oracle_mod.sub(a, b)
        e, ce = oracle_mod.add(d, b)
        assert (e == a).all() and ce == br
        # a*b = b*a
        assert (oracle_mod.mul(a, b) == oracle_mod.mul(b, a)).all()
        # a*(b + c) = a*b + a*c, with b + c on n+1 limbs
        bc, cc = oracle_mod.add(b, c)
        lhs = oracle_mod.mul(a, np.append(bc, np.uint64(cc)))
        ab, ac = oracle_mod.mul(a, b), oracle_mod.mul(a, c)
        rhs, co = oracle_mod.add(np.append(ab, np.uint64(0)), np.append(ac, np.uint64(0)))
        assert co == 0 and (lhs == rhs).all()


# ----------------------------------------------------------------------------------------
# residues, computed limb by limb (Horner) without building big integers
# ----------------------------------------------------------------------------------------
PRIMES = [3, 5, 7, 641, 65537, 998244353, 10 ** 9 + 7, (1 << 61) - 1]


def _res(x, p):
    h = 0
    base = (1 << 64) % p
    for limb in reversed([int(v) for v in x]):
        h = (h * base + limb) % p
    return h


@pytest.mark.parametrize("n", [7, 64, 200])
def test_residues(oracle_mod, n):
    g = np.random.default_rng(77 + n)
    a, b = _rand(g, n), _rand(g, n)
    ra, ca = oracle_mod.add(a, b)
    rs, cs = oracle_mod.sub(a, b)
    rm = oracle_mod.mul(a, b)
    for p in PRIMES:
        top = pow(2, 64 * n, p)
        A, B = _res(a, p), _res(b, p)
        assert (_res(ra, p) + ca * top) % p == (A + B) % p
        assert (_res(rs, p) - cs * top) % p == (A - B) % p
        assert _res(rm, p) == (A * B) % p
    # mod 2^64 - 1: sum of limbs with end-around carry
    m = MASK64

    def r64(x):
        s = 0
        for v in x:
            s += int(v)
            s = (s & m) + (s >> 64)
        return s % m

    assert r64(rm) == (r64(a) * r64(b)) % m


# ----------------------------------------------------------------------------------------
# emulations of the paper's phases (restated, not the oracle's code path)
# ----------------------------------------------------------------------------------------
def _dot_add_chunked(A, B, k, w):
    """Sec. 3.1: limbs in chunks of w.  Phase 1 sums limbs without carries, Phase 2
    marks the limbs that overflowed and shifts the marks up one position (the top
    mark is the chunk's carry-out, the chunk's carry-in enters at the bottom),
    Phase 3 adds the aligned marks, Phase 4 (only when Phase 3 overflowed somewhere)
    resolves cascades through maxed-out limbs with one integer addition over the
    w-bit masks, Kogge-Stone style.  Returns (limbs, carry-out, #chunks with Phase 4)."""
    X = 1 << k
    full = (1 << w) - 1
    out = []
    carry = 0
    fired = 0
    for base in range(0, len(A), w):
        a = A[base:base + w]
        b = B[base:base + w]
        ww = len(a)
        mask_w = (1 << ww) - 1
        s = [(x + y) % X for x, y in zip(a, b)]                       # Phase 1
        gen = sum(1 << i for i in range(ww) if s[i] < a[i])           # Phase 2 (Lemma 1)
        cout = (gen >> (ww - 1)) & 1
        aligned = ((gen << 1) | carry) & mask_w
        s2 = [(s[i] + ((aligned >> i) & 1)) % X for i in range(ww)]   # Phase 3
        over = sum(1 << i for i in range(ww) if s2[i] < s[i])
        if over:                                                      # Phase 4
            fired += 1
            maxed = sum(1 << i for i in range(ww) if s2[i] == X - 1)
            t = (over << 1) + maxed
            cout |= (t >> ww) & 1
            fix = (t ^ maxed) & mask_w
            s2 = [(s2[i] + ((fix >> i) & 1)) % X for i in range(ww)]
        out.extend(s2)
        carry = cout
    del full
    return out, carry, fired


def test_dot_add_phases_match_oracle_k64(oracle_mod):
    from paper_2604_21566_amd import workloads as wl
    g = np.random.default_rng(3)
    cases = [(_rand(g, n), _rand(g, n)) for n in (1, 5, 8, 9, 16, 37)]
    pa, pb = wl.pathological(16, 2)
    cases += list(zip(pa, pb))
    fired_any = False
    for a, b in cases:
        limbs, c, fired = _dot_add_chunked([int(x) for x in a], [int(x) for x in b], 64, 8)
        fired_any |= fired > 0
        r, co = oracle_mod.add(a, b)
        assert limbs == [int(x) for x in r] and c == co
    assert fired_any  # the pathological set exercises Phase 4


def test_dot_add_phases_small_k_bruteforce():
    """With k = 2..4 bits per limb every cascade shape occurs; the phase emulation must
    equal integer addition exactly (Theorem 1)."""
    g = np.random.default_rng(11)
    for k in (2, 3, 4):
        X = 1 << k
        for _ in range(3000):
            m = int(g.integers(1, 20))
            A = [int(v) for v in g.integers(0, X, m)]
            B = [int(v) for v in g.integers(0, X, m)]
            limbs, c, _ = _dot_add_chunked(A, B, k, 8)
            va = sum(v << (k * i) for i, v in enumerate(A))
            vb = sum(v << (k * i) for i, v in enumerate(B))
            assert sum(v << (k * i) for i, v in enumerate(limbs)) + (c << (k * m)) == va + vb


def _vnc_mul(A, B, k):
    """Sec. 3.2 vertical-and-crosswise: gather every (i, j) by output column c = i + j,
    form all lo/hi halves independently, deposit lo into column c and hi into c + 1,
    then one sequential carry pass over the columns."""
    m_a, m_b = len(A), len(B)
    X = 1 << k
    ncol = m_a + m_b
    pairs = [(i, c - i) for c in range(ncol - 1) for i in range(m_a) if 0 <= c - i < m_b]
    prods = [(i + j, (A[i] * B[j]) % X, (A[i] * B[j]) // X) for i, j in pairs]
    col = [0] * ncol
    for c, lo, hi in prods:
        col[c] += lo
        col[c + 1] += hi
    out, carry = [], 0
    for c in range(ncol):
        v = col[c] + carry
        out.append(v % X)
        carry = v // X
    return out, carry, pairs


def test_vnc_mul_matches_oracle(oracle_mod):
    g = np.random.default_rng(9)
    for na, nb in [(1, 1), (4, 4), (5, 5), (3, 8), (16, 16)]:
        for _ in range(3):
            a, b = _rand(g, na), _rand(g, nb)
            limbs, carry, _ = _vnc_mul([int(x) for x in a], [int(x) for x in b], 64)
            assert carry == 0  # the product of na and nb limbs fits na + nb limbs
            assert limbs == [int(x) for x in oracle_mod.mul(a, b)]
    ones = np.full(6, MASK64, np.uint64)
    limbs, carry, _ = _vnc_mul([MASK64] * 6, [MASK64] * 6, 64)
    assert carry == 0 and limbs == [int(x) for x in oracle_mod.mul(ones, ones)]


def test_vnc_structure_golden():
    with open(os.path.join(GOLDEN, "vnc_m5_structure.json")) as f:
        gold = json.load(f)
    m = gold["m"]
    limbs, carry, pairs = _vnc_mul([1] * m, [1] * m, 52)
    counts = [sum(1 for i, j in pairs if i + j == c) for c in range(2 * m - 1)]
    assert counts == gold["pairs_per_column"]
    assert len(counts) == gold["columns"] and len(pairs) == gold["total_pairs"]
    col4 = sorted([i, j] for i, j in pairs if i + j == 4)
    assert col4 == gold["column_4_pairs"]
    lo_col, hi_col = 2 + 3, 2 + 3 + 1
    assert (lo_col, hi_col) == (gold["pair_2_3_lo_column"], gold["pair_2_3_hi_column"])
    assert len(limbs) == gold["product_limbs"]


def test_carry_lemmas_k8_golden():
    """Appendix B lemmas at k = 8 by brute force, plus Lemma 1 (carry iff the wrapped
    sum is below an operand)."""
    with open(os.path.join(GOLDEN, "carry_lemmas_k8.json")) as f:
        gold = json.load(f)
    k = gold["k"]
    X = 1 << k
    a = np.arange(X)[:, None]
    b = np.arange(X)[None, :]
    s = a + b
    carry = s >= X
    assert int(carry.sum()) == gold["carry_pairs"]
    assert int((s == X - 1).sum()) == gold["max_sum_pairs"]
    assert carry.size == gold["total_pairs"]
    wrapped = s % X
    assert ((wrapped < a) == carry).all() and ((wrapped < b) == carry).all()


# ----------------------------------------------------------------------------------------
# ragged addition against CPython int (Theorem 1 per pair; descriptor layout read as stated)
# ----------------------------------------------------------------------------------------
def test_add_ragged_vs_int(oracle_mod):
    """Pairs of uneven length in pooled arrays with gaps between them, offsets not in
    pair order, n = 0 items, all-ones + 1 pairs (carry out of the top limb) and a
    zero - one style borrow chain.  The descriptor's nb field is ignored for addition:
    it is set to a different value here so that reading n from the wrong field fails."""
    g = np.random.default_rng(2604)
    lens = [5, 0, 1, 33, 2, 0, 17, 64, 3, 9]
    ones_pairs = {2, 6}          # a = all ones, b = 1: every limb propagates, carry 1
    npairs = len(lens)
    # pools with gaps and a permuted placement of the pairs
    order = g.permutation(npairs)
    a_pool = _rand(g, 600)
    b_pool = _rand(g, 600)
    desc, A, B = [None] * npairs, [None] * npairs, [None] * npairs
    a_off, b_off, r_off = 3, 11, 7
    for p in order:
        n = lens[p]
        if p in ones_pairs:
            a_pool[a_off:a_off + n] = MASK64
            b_pool[b_off:b_off + n] = 0
            if n:
                b_pool[b_off] = 1
        A[p] = a_pool[a_off:a_off + n].copy()
        B[p] = b_pool[b_off:b_off + n].copy()
        desc[p] = (a_off, b_off, r_off, n, n // 2)   # nb field: ignored; differs from n when n > 0
        a_off += n + 4
        b_off += n + 1
        r_off += n + 2
    r_size = r_off + 5
    r, c = oracle_mod.add_ragged(a_pool, b_pool, np.array(desc, np.uint64), r_size)
    assert c.size == npairs
    written = np.zeros(r_size, bool)
    for p in range(npairs):
        n = lens[p]
        ro = desc[p][2]
        S = to_int(A[p]) + to_int(B[p])
        assert to_int(r[ro:ro + n]) == S % (1 << (64 * n)), p
        assert int(c[p]) == S >> (64 * n), p
        written[ro:ro + n] = True
        if p in ones_pairs and n:
            assert int(c[p]) == 1 and not r[ro:ro + n].any()
    # limbs outside every pair's result range are untouched (the oracle zero-fills r)
    assert not r[~written].any()


# ----------------------------------------------------------------------------------------
# planted mistakes: each mutant of the oracle source must fail at least one pin
# ----------------------------------------------------------------------------------------
MUTANTS = {
    "dropped carry": ("c = (uint64_t)(t >> 64);       /* floor((A_i + B_i + c_i)/X) */", "c = 0;"),
    "wrong borrow": ("br = ((u128)a[i] < need) ? 1u : 0u;\n    }\n    return br;\n}\n\n/*\n * Multiplication",
                     "br = ((u128)a[i] < (u128)b[i]) ? 1u : 0u;\n    }\n    return br;\n}\n\n/*\n * Multiplication"),
    "dropped top carry": ("        r[i + nb] = c;\n", "        (void)c;\n"),
    "stray term": ("u128 t = (u128)a[i] * (u128)b[j] + (u128)r[i + j] + (u128)c;",
                   "u128 t = (u128)a[i] * (u128)b[j] + (u128)r[i + j] + (u128)c + (u128)(i == 1 && j == 2);"),
    "ragged add: n from the nb field": (
        "uint64_t c = bnref_add_n(r_pool + d[2], a_pool + d[0], b_pool + d[1], (size_t)d[3]);",
        "uint64_t c = bnref_add_n(r_pool + d[2], a_pool + d[0], b_pool + d[1], (size_t)d[4]);"),
    "ragged add: b and r offsets swapped": (
        "uint64_t c = bnref_add_n(r_pool + d[2], a_pool + d[0], b_pool + d[1], (size_t)d[3]);",
        "uint64_t c = bnref_add_n(r_pool + d[1], a_pool + d[0], b_pool + d[2], (size_t)d[3]);"),
    "ragged mul: lengths swapped": (
        "bnref_mul(r_pool + d[2], a_pool + d[0], (size_t)d[3], b_pool + d[1], (size_t)d[4]);",
        "bnref_mul(r_pool + d[2], a_pool + d[0], (size_t)d[4], b_pool + d[1], (size_t)d[3]);"),
    "carry-in ignored": ("uint64_t c = cin;", "uint64_t c = 0;"),
}


def _pins(mod):
    """The pins a mutant is run against (the same functions as above)."""
    checks = [
        lambda: test_add_sub_specials_exhaustive(mod, 1),
        lambda: test_add_sub_random_vs_int(mod, 33),
        lambda: test_carry_in_variants_vs_int(mod, 5),
        lambda: test_mul_random_vs_int(mod, 13, 29),
        lambda: test_batch_and_ragged_vs_int(mod),
        lambda: test_closed_forms(mod, 5),
        lambda: test_add_ragged_vs_int(mod),
    ]
    failed = 0
    for chk in checks:
        try:
            chk()
        except AssertionError:
            failed += 1
    return failed


_CHILD = """
import sys
sys.path[:0] = {paths!r}
import oracle
import test_oracle as T
oracle._LIB, oracle._SRC, oracle._lib = {so!r}, {src!r}, None
oracle._load()
sys.exit(3 if T._pins(oracle) >= 1 else 0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(oracle_mod, tmp_path, name):
    """The mutant runs in a child process (a mistake that writes past a buffer must
    not corrupt this one); exit status 3 means at least one pin failed on it."""
    import subprocess
    import sys
    src = open(oracle_mod._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site of {name!r} not found once"
    mut = tmp_path / "bn_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", str(mut), "-o", str(so)])
    here = os.path.dirname(os.path.abspath(__file__))
    code = _CHILD.format(paths=[os.path.dirname(here), here], so=str(so), src=str(mut))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert res.returncode == 3, f"planted mistake {name!r}: exit {res.returncode}\n{res.stderr[-2000:]}"


def test_unmutated_oracle_passes_the_mutation_pins(oracle_mod):
    assert _pins(oracle_mod) == 0
