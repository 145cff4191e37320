"""Host-CPU DoT add/sub (Sec. 3.1, Algorithm 1 with AVX-512 / AVX2, and the scalar
carry chain) against the CPU oracle, bit-exact, on every ISA this CPU runs (CPU only)."""
import os

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAX = 2 ** 64 - 1
U = np.uint64


@pytest.fixture(scope="module")
def H():
    from paper_2604_21566_amd import host
    if not os.path.exists(host.LIB_PATH):
        from paper_2604_21566_amd import build as b
        b.build_host(verbose=False)
    return host


def _isas():
    from paper_2604_21566_amd import host
    if not os.path.exists(host.LIB_PATH):
        from paper_2604_21566_amd import build as b
        b.build_host(verbose=False)
    return list(range(host.bnh_isa_best() + 1))


ISAS = _isas()


def _rand(g, n):
    return g.integers(0, MAX, n, dtype=U, endpoint=True)


def _edge(g, n):
    """Limbs from {0, 1, 2^64 - 2, 2^64 - 1}: carries, propagates and cascades everywhere."""
    return np.array([0, 1, MAX - 1, MAX], dtype=U)[g.integers(0, 4, n)]


def _batch(H, op, a, b, n, npairs, isa, threads=1):
    r = np.zeros(n * npairs, U)
    c = np.full(npairs, 7, U)
    (H.bnh_add_n_batch if op == "add" else H.bnh_sub_n_batch)(r, a, b, n, npairs, c, isa, threads)
    return r, c


@pytest.mark.parametrize("isa", ISAS)
@pytest.mark.parametrize("op", ["add", "sub"])
def test_edge_values_every_length(H, isa, op):
    """Every length 1..40 (several steps and every ragged last step), limbs drawn from
    the four values that make carries, propagates and cascades."""
    g = np.random.default_rng(isa * 10 + (op == "sub"))
    for n in range(1, 41):
        npairs = 3000
        a, b = _edge(g, n * npairs), _edge(g, n * npairs)
        r, c = _batch(H, op, a, b, n, npairs, isa)
        rr, rc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)
        assert (r == rr).all() and (c == rc).all(), f"n={n}"


@pytest.mark.parametrize("isa", ISAS)
@pytest.mark.parametrize("op", ["add", "sub"])
@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 63, 64, 65, 1000, 4097, 100003])
def test_random_with_carry_in(H, isa, op, n):
    g = np.random.default_rng(n + isa)
    a, b = _rand(g, n), _rand(g, n)
    for cin in (0, 1):
        r = np.zeros(n, U)
        c = (H.bnh_add_n if op == "add" else H.bnh_sub_n)(r, a, b, cin, isa)
        if n == 0:  # the carry passes through
            rr, rc = r, [cin]
        else:
            rr, rc = (oracle.add_nc_batch if op == "add" else oracle.sub_nc_batch)(a, b, n, np.array([cin], U))
        assert (r == rr).all() and c == rc[0], f"cin={cin}"


@pytest.mark.parametrize("isa", ISAS)
def test_full_cascades(H, isa):
    """(2^(64n) - 1) + 1 and 2^(64(n-1)) - 1: the carry (borrow) crosses every limb and
    every step; runs that end exactly at a step's top lane; a run that starts mid-step."""
    for n in (1, 3, 4, 5, 8, 9, 16, 17, 100):
        a = np.full(n, MAX, U)
        b = np.zeros(n, U)
        b[0] = 1
        r = np.zeros(n, U)
        assert H.bnh_add_n(r, a, b, 0, isa) == 1 and not r.any(), n
        a = np.zeros(n, U)
        a[-1] = 1
        assert H.bnh_sub_n(r, a, b, 0, isa) == 0, n
        want = np.full(n, MAX, U)
        want[-1] = 0
        assert (r == want).all(), n
    # generate at limb s, propagate run up to limb e (inclusive), inside and across steps
    n = 32
    for s in range(0, 20):
        for e in range(s + 1, n):
            a = np.zeros(n, U)
            b = np.zeros(n, U)
            a[s], b[s] = MAX, 2          # generates
            a[s + 1:e + 1] = MAX         # propagates
            r = np.zeros(n, U)
            c = H.bnh_add_n(r, a, b, 0, isa)
            rr, rc = oracle.add(a, b)
            assert (r == rr).all() and c == rc, (s, e)
            c = H.bnh_sub_n(r, b, a, 0, isa)
            rr, rc = oracle.sub(b, a)
            assert (r == rr).all() and c == rc, (s, e)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_batch_threads_and_in_place(H, threads):
    g = np.random.default_rng(threads)
    n, npairs = 13, 1001
    a, b = _rand(g, n * npairs), _edge(g, n * npairs)
    r, c = _batch(H, "add", a, b, n, npairs, None, threads)
    rr, rc = oracle.add_batch(a, b, n)
    assert (r == rr).all() and (c == rc).all()
    x = a.copy()
    H.bnh_sub_n_batch(x, x, b, n, npairs, None, None, threads)  # r == a, no carry array
    assert (x == oracle.sub_batch(a, b, n)[0]).all()


def test_errors(H):
    z = np.zeros(4, U)
    with pytest.raises(H.BnhError) as e:
        H.bnh_add_n(z, z, z, 0, 7)
    assert e.value.status == H.BNH_EINVAL
    with pytest.raises(H.BnhError) as e:
        H.bnh_add_n(z, z, z, 2, 0)  # carry-in must be 0 or 1
    assert e.value.status == H.BNH_EINVAL
    with pytest.raises(H.BnhError) as e:
        H.bnh_add_n_batch(z, z, z, 2, 2, None, 0, 0)  # threads < 1
    assert e.value.status == H.BNH_EINVAL
    if H.bnh_isa_best() < H.BNH_ISA_AVX512:
        with pytest.raises(H.BnhError) as e:
            H.bnh_add_n(z, z, z, 0, H.BNH_ISA_AVX512)
        assert e.value.status == H.BNH_EUNSUPPORTED
    # n = 0 passes the carry through
    assert H.bnh_add_n(z[:0], z[:0], z[:0], 1, 0) == 1
    assert H.lib().bnh_add_n(None, None, None, 0, 0, None, 0) == H.BNH_OK
