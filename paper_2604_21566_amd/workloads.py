"""Seeded synthetic operands for the five benchmark/parity workloads.

This module only *generates inputs*; it holds none of the add/sub/mul
arithmetic.  The test-suite feeds the same arrays to the GPU library and to the
CPU oracle.

Operands are little-endian arrays of 64-bit limbs (numpy ``uint64``).  Limbs are
drawn from numpy's PCG64 bit generator (raw 64-bit outputs), seeded per
workload.  The paper draws its operands with a seeded Mersenne Twister (Sec. 4,
test-case description); PCG64 is used here only because it is ~10x faster for
the multi-GiB operands, and the limb distribution (uniform on [0, 2^64)) is the
same.  Besides uniform operands the paper uses "pathological" inputs: full
carry/borrow propagation, maxed-out and zero limbs, frequent carries/borrows
(Sec. 4); the patterns below make those concrete.

Workloads (sizes are the defaults; tests shrink them):
  c1  1024 uniform pairs of 4 limbs + 64 pathological pairs (8 patterns x 8)
  c2  2^20 pairs x 64 limbs, every 10th pair adversarial (long propagate run
      behind a forced generate/borrow limb)
  c3  one pair of 2^26 limbs with 16 embedded propagate runs of 2^10..2^20
      limbs, plus an "all-propagate" worst case
  c4  2^16 ragged pairs, bit lengths log-uniform on [256, 8192] (a and b
      independent), top limb masked to the bit length with its top bit set
  c5  64 pairs x 16384 limbs, pair 0 all-ones x all-ones, pair 1 zero x zero
"""
from __future__ import annotations

import numpy as np

MAX64 = np.uint64(0xFFFFFFFFFFFFFFFF)
SEED_BASE = 0x2604215660


def rng(tag: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + int(tag), int(stream)]))


def limbs(g: np.random.Generator, size) -> np.ndarray:
    """Uniform 64-bit limbs."""
    n = int(np.prod(size)) if not np.isscalar(size) else int(size)
    return g.bit_generator.random_raw(n).astype(np.uint64, copy=False).reshape(size)


def _below(g: np.random.Generator, hi: np.ndarray) -> np.ndarray:
    """Uniform-ish integers in [0, hi) for uint64 hi >= 1 (modulo draw; bias is irrelevant here)."""
    return limbs(g, hi.shape) % hi


def _lt(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Row-wise a < b for [npairs, n] limb arrays (compare from the top limb)."""
    neq = a != b
    n = a.shape[1]
    # index of the most significant differing limb, or -1
    rev = neq[:, ::-1]
    has = rev.any(axis=1)
    top = n - 1 - np.argmax(rev, axis=1)
    rows = np.arange(a.shape[0])
    return has & (a[rows, top] < b[rows, top])


def order_ge(a: np.ndarray, b: np.ndarray):
    """Swap rows so that a >= b row-wise (for 'a >= b ordered' subtraction)."""
    a = a.copy()
    b = b.copy()
    sw = _lt(a, b)
    t = a[sw].copy()
    a[sw] = b[sw]
    b[sw] = t
    return a, b


# --------------------------------------------------------------------------------------
# pathological patterns for small pairs (used by c1 and by edge-case tests)
# --------------------------------------------------------------------------------------
PATTERNS = (
    "ones_plus_one",      # (2^(64n)-1, 1): carry crosses every limb
    "ones_plus_ones",     # (2^(64n)-1, 2^(64n)-1)
    "pow_minus_one",      # (2^(64k), 1), k = 1..n-1: borrow crosses k limbs
    "one_off",            # all-ones with one random limb, plus 1
    "complement",         # b = ~a (every limb propagates) with a forced generate at limb 0
    "equal",              # a == b: subtraction gives 0, every limb propagates a borrow
    "zeros",              # (0, 0)
    "ones_random",        # (2^(64n)-1, uniform)
)


def pattern_pair(name: str, n: int, g: np.random.Generator, k: int = 0):
    a = np.zeros(n, np.uint64)
    b = np.zeros(n, np.uint64)
    if n == 0:
        return a, b
    if name == "ones_plus_one":
        a[:] = MAX64
        b[0] = 1
    elif name == "ones_plus_ones":
        a[:] = MAX64
        b[:] = MAX64
    elif name == "pow_minus_one":
        kk = 1 + (k % max(1, n - 1)) if n > 1 else 0
        a[kk] = 1
        b[0] = 1
    elif name == "one_off":
        a[:] = MAX64
        j = int(limbs(g, 1)[0] % np.uint64(n))
        a[j] = limbs(g, 1)[0]
        b[0] = 1
    elif name == "complement":
        a[:] = limbs(g, n)
        a[0] |= np.uint64(1)
        b[:] = ~a
        # forced generate at limb 0: b0 in [2^64 - a0, 2^64 - 1]
        b[0] = (MAX64 - a[0] + np.uint64(1)) + (limbs(g, 1)[0] % a[0])
    elif name == "equal":
        a[:] = limbs(g, n)
        b[:] = a
    elif name == "zeros":
        pass
    elif name == "ones_random":
        a[:] = MAX64
        b[:] = limbs(g, n)
    else:
        raise ValueError(name)
    return a, b


def pathological(n: int, per_pattern: int, seed: int = 0):
    """[len(PATTERNS)*per_pattern, n] arrays a, b cycling through PATTERNS."""
    g = rng(100 + seed)
    A, B = [], []
    for name in PATTERNS:
        for k in range(per_pattern):
            a, b = pattern_pair(name, n, g, k)
            A.append(a)
            B.append(b)
    return np.stack(A), np.stack(B)


# --------------------------------------------------------------------------------------
# c1: 1024 uniform + 64 pathological pairs of 4 limbs
# --------------------------------------------------------------------------------------
def c1(op: str = "add", n: int = 4, nuniform: int = 1024, per_pattern: int = 8):
    """Returns flat a, b (pairs contiguous, n limbs each).  Sub pairs are ordered a >= b."""
    g = rng(1)
    a = limbs(g, (nuniform, n))
    b = limbs(g, (nuniform, n))
    pa, pb = pathological(n, per_pattern, seed=1)
    a = np.concatenate([a, pa])
    b = np.concatenate([b, pb])
    if op == "sub":
        a, b = order_ge(a, b)
    return a.reshape(-1), b.reshape(-1)


# --------------------------------------------------------------------------------------
# c2: batched 64-limb pairs, every 10th adversarial
# --------------------------------------------------------------------------------------
def c2(op: str = "add", npairs: int = 1 << 20, n: int = 64, seed: int = 0):
    """Flat a, b of npairs*n limbs.  Pairs with p % 10 == 9 carry a propagate run
    [s+1, s+l] (l >= min(16, ...)) behind a forced generate (add) / borrow (sub) limb s.
    Sub pairs are ordered a >= b."""
    g = rng(2, seed)
    a = limbs(g, (npairs, n))
    b = limbs(g, (npairs, n))
    adv = np.arange(npairs) % 10 == 9
    na = int(adv.sum())
    if na and n >= 2:
        top = n - 1 if op == "add" else n - 2      # sub keeps the top limb free to order a >= b
        top = max(top, 1)
        lmin_all = min(16, top)                                                 # runs of >= 16 limbs when n allows
        s = (limbs(g, na) % np.uint64(max(1, top - lmin_all + 1))).astype(np.int64)  # s in [0, top-lmin]
        room = top - s                                                          # run may reach limb `top`
        lmin = np.minimum(lmin_all, room)
        lrange = np.maximum(room - lmin + 1, 1).astype(np.uint64)
        ln = lmin + (limbs(g, na) % lrange).astype(np.int64)
        idx = np.arange(n)[None, :]
        run = (idx > s[:, None]) & (idx <= (s + ln)[:, None])
        at = a[adv]
        bt = b[adv]
        rows = np.arange(na)
        if op == "add":
            at[run] = MAX64
            bt[run] = 0
            a_s = at[rows, s] | np.uint64(1)
            at[rows, s] = a_s
            bt[rows, s] = (MAX64 - a_s + np.uint64(1)) + _below(g, a_s)
        else:
            bt[run] = at[run]
            a_s = at[rows, s] & ~np.uint64(1 << 63)      # leave room so that a_s < b_s is possible
            at[rows, s] = a_s
            bt[rows, s] = a_s + np.uint64(1) + _below(g, MAX64 - a_s)
            # top limb decides a >= b
            at[:, n - 1] |= np.uint64(1 << 63)
            bt[:, n - 1] &= ~np.uint64(1 << 63)
        a[adv] = at
        b[adv] = bt
    if op == "sub":
        a, b = order_ge(a, b)
    return a.reshape(-1), b.reshape(-1)


# --------------------------------------------------------------------------------------
# c3: one huge pair with embedded propagate runs
# --------------------------------------------------------------------------------------
def c3_runs(n: int, g: np.random.Generator, nruns: int = 16, lo_log: int = 10, hi_log: int = 20):
    """Run (start, length) list: one run of each length 2^lo..2^hi, the rest log-uniform,
    one run starting at limb 0 and one ending at the top limb, all non-overlapping."""
    lens = [1 << k for k in range(lo_log, hi_log + 1)]
    while len(lens) < nruns:
        lens.append(int(2 ** (lo_log + (hi_log - lo_log) * (int(limbs(g, 1)[0] >> np.uint64(11)) / 2.0 ** 53))))
    lens = lens[:nruns]
    perm = np.argsort(limbs(g, len(lens)))
    lens = [lens[i] for i in perm]
    slot = n // nruns
    runs = []
    for i, ln in enumerate(lens):
        ln = min(ln, slot - 2)
        if i == 0:
            st = 0
        elif i == nruns - 1:
            st = n - ln
        else:
            st = i * slot + 1 + int(limbs(g, 1)[0] % np.uint64(max(1, slot - ln - 2)))
        runs.append((st, ln))
    return runs


def c3(op: str = "add", n: int = 1 << 26, worst: bool = False, seed: int = 0):
    """Single pair a, b of n limbs.  worst=True gives the input whose carry (borrow)
    crosses every limb: add (2^(64n)-1) + 1, sub 2^(64(n-1)) - 1."""
    if worst:
        a = np.zeros(n, np.uint64)
        b = np.zeros(n, np.uint64)
        if op == "add":
            a[:] = MAX64
        else:
            a[n - 1] = 1
        b[0] = 1
        return a, b
    g = rng(3, seed)
    a = limbs(g, n)
    b = limbs(g, n)
    for st, ln in c3_runs(n, g):
        if op == "add":
            a[st:st + ln] = MAX64
            b[st:st + ln] = 0
            if st > 0:
                a_s = a[st - 1] | np.uint64(1)
                a[st - 1] = a_s
                b[st - 1] = (MAX64 - a_s + np.uint64(1)) + (limbs(g, 1)[0] % a_s)
        else:
            b[st:st + ln] = a[st:st + ln]
            if st > 0:
                a_s = a[st - 1] & ~np.uint64(1 << 63)
                a[st - 1] = a_s
                b[st - 1] = a_s + np.uint64(1) + (limbs(g, 1)[0] % (MAX64 - a_s))
    return a, b


# --------------------------------------------------------------------------------------
# c4: ragged pairs
# --------------------------------------------------------------------------------------
def c4_sizes(npairs: int, lo_bits: int = 256, hi_bits: int = 8192, seed: int = 0):
    g = rng(4, seed)
    u = (limbs(g, (2, npairs)) >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    bits = np.floor(np.exp(np.log(lo_bits) + u * (np.log(hi_bits) - np.log(lo_bits)))).astype(np.int64)
    bits = np.clip(bits, lo_bits, hi_bits)
    return bits[0], bits[1]


def _masked_operand(g, bits: int) -> np.ndarray:
    n = (bits + 63) // 64
    x = limbs(g, n)
    tb = bits - 64 * (n - 1)                      # bits in the top limb, 1..64
    if tb < 64:
        x[-1] &= np.uint64((1 << tb) - 1)
    x[-1] |= np.uint64(1 << (tb - 1))
    return x


def c4(npairs: int = 1 << 16, lo_bits: int = 256, hi_bits: int = 8192, seed: int = 0):
    """Returns (a_pool, b_pool, desc[npairs,5] = (a_off, b_off, r_off, na, nb), r_size)."""
    ba, bb = c4_sizes(npairs, lo_bits, hi_bits, seed)
    g = rng(40, seed)
    na = (ba + 63) // 64
    nb = (bb + 63) // 64
    a_off = np.concatenate([[0], np.cumsum(na)[:-1]]).astype(np.int64)
    b_off = np.concatenate([[0], np.cumsum(nb)[:-1]]).astype(np.int64)
    r_off = np.concatenate([[0], np.cumsum(na + nb)[:-1]]).astype(np.int64)
    a_pool = limbs(g, int(na.sum()))
    b_pool = limbs(g, int(nb.sum()))
    # top limb of each operand masked to its bit length with the top bit set
    ta = a_off + na - 1
    tb = b_off + nb - 1
    for pool, top, bits, cnt in ((a_pool, ta, ba, na), (b_pool, tb, bb, nb)):
        tbits = bits - 64 * (cnt - 1)
        mask = np.where(tbits >= 64, MAX64, (np.uint64(1) << tbits.astype(np.uint64)) - np.uint64(1))
        pool[top] &= mask
        pool[top] |= np.uint64(1) << (tbits - 1).astype(np.uint64)
    desc = np.stack([a_off, b_off, r_off, na, nb], axis=1).astype(np.uint64)
    r_size = int((na + nb).sum())
    return a_pool, b_pool, desc, r_size


# --------------------------------------------------------------------------------------
# c5: large uniform products
# --------------------------------------------------------------------------------------
def c5(npairs: int = 64, n: int = 16384, seed: int = 0):
    """Flat a, b of npairs*n limbs; pair 0 = all-ones x all-ones, pair 1 = 0 x 0."""
    g = rng(5, seed)
    a = limbs(g, (npairs, n))
    b = limbs(g, (npairs, n))
    if npairs >= 1:
        a[0] = MAX64
        b[0] = MAX64
    if npairs >= 2:
        a[1] = 0
        b[1] = 0
    return a.reshape(-1), b.reshape(-1)
