"""The seeded generators produce the intended operand structure (CPU only)."""
import numpy as np

from paper_2604_21566_amd import workloads as wl

MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def test_deterministic():
    a1, b1 = wl.c2("add", npairs=100)
    a2, b2 = wl.c2("add", npairs=100)
    assert (a1 == a2).all() and (b1 == b2).all()


def test_c1_shape_and_sub_order():
    a, b = wl.c1("sub")
    assert a.size == 1088 * 4
    A = a.reshape(-1, 4)
    B = b.reshape(-1, 4)
    assert not wl._lt(A, B).any()
    a, b = wl.c1("add")
    # the first pathological pair is all-ones + 1
    assert (a.reshape(-1, 4)[1024] == MAX).all() and b.reshape(-1, 4)[1024][0] == 1


def _add_flags(a, b):
    s = a + b
    g = s < a
    p = s == MAX
    return g, p


def test_c2_adversarial_pairs_have_long_propagate_runs():
    n = 64
    a, b = wl.c2("add", npairs=2000, n=n)
    A, B = a.reshape(-1, n), b.reshape(-1, n)
    g, p = _add_flags(A, B)
    assert not (g & p).any()
    for i in range(9, 2000, 10):
        runs = np.diff(np.concatenate([[0], p[i].astype(np.int8), [0]]))
        st, en = np.where(runs == 1)[0], np.where(runs == -1)[0]
        longest = int((en - st).max())
        assert longest >= 16
        s0 = st[np.argmax(en - st)]
        assert g[i, s0 - 1]                       # a forced generate sits right below the run
    # uniform pairs: generate fraction ~ 1/2 (Appendix B: 1/2 - 2^-65), propagate ~ 0
    uni = np.arange(2000) % 10 != 9
    frac = g[uni].mean()
    assert abs(frac - 0.5) < 5 * np.sqrt(0.25 / g[uni].size)
    assert p[uni].sum() == 0


def test_c2_sub_pairs_ordered_and_adversarial():
    n = 64
    a, b = wl.c2("sub", npairs=500, n=n)
    A, B = a.reshape(-1, n), b.reshape(-1, n)
    assert not wl._lt(A, B).any()
    eq = A == B
    assert eq[9::10].sum(axis=1).min() >= 16


def test_c3_runs():
    n = 1 << 16
    a, b = wl.c3("add", n=n)
    g, p = _add_flags(a, b)
    assert p[:64].all()                            # a run starts at limb 0
    assert p[-64:].all()                           # a run ends at the top limb
    assert not (g & p).any()
    aw, bw = wl.c3("add", n=1024, worst=True)
    gw, pw = _add_flags(aw, bw)
    assert gw[0] and pw[1:].all()


def test_c4_sizes_and_top_bits():
    a, b, desc, rsz = wl.c4(npairs=3000)
    na, nb = desc[:, 3].astype(np.int64), desc[:, 4].astype(np.int64)
    assert na.min() >= 4 and na.max() <= 128 and nb.min() >= 4 and nb.max() <= 128
    assert (na != nb).mean() > 0.5
    assert rsz == int((na + nb).sum())
    tops = a[desc[:, 0].astype(np.int64) + na - 1]
    assert (tops != 0).all()
    # log-uniform bit lengths: median near sqrt(256 * 8192) = 1448 bits
    ba, _ = wl.c4_sizes(20000)
    assert 1200 < np.median(ba) < 1700


def test_c5_special_pairs():
    a, b = wl.c5(npairs=4, n=64)
    A = a.reshape(4, 64)
    assert (A[0] == MAX).all() and (A[1] == 0).all()
