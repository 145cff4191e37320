"""Multiplication in place (the output overlapping an operand, in whole or in part)
against the CPU oracle, bit-exact, through the C ABI: every form, small and large
products, batches, Karatsuba levels and a captured graph."""
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


def _layout(na, nb, npairs, where):
    """Offsets (limbs) of a, b and r in one buffer for an overlap kind."""
    A, B, R = na * npairs, nb * npairs, (na + nb) * npairs
    if where == "r_is_a":     # r starts at a (a is the prefix of r), b elsewhere
        return 0, R + 3, 0, R + B + 3
    if where == "r_is_b":
        return R + 3, 0, 0, R + A + 3
    if where == "r_inside":   # r starts inside a and runs over b
        return 0, A, A // 2 + 1, A // 2 + 1 + R + 1
    if where == "r_below":    # r ends inside a
        return R - 1, R - 1 + A, 0, R - 1 + A + B
    raise ValueError(where)


def _run(ctx, na, nb, npairs, form, where, seed, call):
    announce("mul in place", form, where, f"na={na}", f"nb={nb}", f"npairs={npairs}")
    g = np.random.default_rng(seed)
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    oa, ob, orr, size = _layout(na, nb, npairs, where)
    host = _rand(g, size)
    host[oa:oa + a.size] = a
    host[ob:ob + b.size] = b
    buf = D(host)
    R = (na + nb) * npairs
    call(buf[orr:orr + R], buf[oa:oa + a.size], buf[ob:ob + b.size])
    torch.cuda.synchronize()
    want = host.copy()
    want[orr:orr + R] = oracle.mul_batch(a, b, na, nb, npairs)
    got = H(buf)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} bad limbs, first at {bad[0]} (r at {orr})"


CASES = [(4, 4, 1), (4, 4, 1088), (13, 29, 77), (128, 128, 9), (300, 212, 3), (700, 700, 2), (1500, 900, 1),
         (4096, 4096, 2)]


@pytest.mark.parametrize("form", ["auto", "mad", "mfma"])
@pytest.mark.parametrize("na,nb,npairs", CASES)
@pytest.mark.parametrize("where", ["r_is_a", "r_is_b", "r_inside", "r_below"])
def test_batch_in_place(bnctx, form, na, nb, npairs, where):
    _run(bnctx, na, nb, npairs, form, where, na * 7 + nb + npairs,
         lambda r, a, b: bn.bn_mul_n_batch(bnctx, r, a, b, na, nb, npairs, form))


@pytest.mark.parametrize("form", ["mad", "mfma"])
def test_single_in_place(bnctx, form):
    _run(bnctx, 333, 64, 1, form, "r_is_a", 11, lambda r, a, b: bn.bn_mul(bnctx, r, a, b, form))


@pytest.mark.parametrize("form", ["mad", "mfma"])
@pytest.mark.parametrize("n,npairs,levels", [(64, 5, 1), (256, 3, 2), (2048, 2, 3)])
@pytest.mark.parametrize("where", ["r_is_a", "r_inside"])
def test_karatsuba_in_place(bnctx, form, n, npairs, levels, where):
    _run(bnctx, n, n, npairs, form, where, n + levels,
         lambda r, a, b: bn.bn_mul_karatsuba_n_batch(bnctx, r, a, b, n, npairs, levels, form))


def test_graph_in_place(bnctx):
    """A captured in-place batch replays exactly (operands re-staged between replays)."""
    na, nb, npairs = 40, 24, 300
    announce("mul in place graph", f"na={na}", f"nb={nb}", f"npairs={npairs}")
    g = np.random.default_rng(3)
    a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
    R = (na + nb) * npairs
    buf = torch.zeros(R + nb * npairs, dtype=torch.int64, device="cuda")
    r, ta, tb = buf[:R], buf[:na * npairs], buf[R:]
    s = torch.cuda.Stream()
    graph = bn.bn_graph_capture_batch(bnctx, 2, r, ta, tb, na, nb, npairs, None, bn.BN_MUL_AUTO, stream=s)
    want = oracle.mul_batch(a, b, na, nb, npairs)
    try:
        for rep in range(3):
            buf.zero_()
            ta.copy_(D(a))
            tb.copy_(D(b))
            torch.cuda.synchronize()
            bn.bn_graph_launch(graph, s)
            s.synchronize()
            assert (H(r) == want).all(), f"replay {rep}"
            bn.bn_mul_n_batch(bnctx, torch.empty_like(r), tb, tb, nb, nb, npairs)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        bn.bn_graph_destroy(graph)
