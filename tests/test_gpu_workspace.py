"""Compute calls never allocate: on contexts without "workspace.auto_grow", every
compute entry point whose shape needs workspace fails with BN_ENOSPACE and enqueues
nothing, and after one bn_reserve_for of that shape it runs inside a stream capture
(no allocation, no host synchronisation is possible there); the graph is replayed
three times, with eager calls of the same shape on the context between replays, and
every replay is checked against the oracle."""
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


def _rand(g, n):
    return g.integers(0, MAX, n, dtype=np.uint64, endpoint=True)


def _cases():
    """(name, reserve args, make) -- make() returns (run(ctx), outputs, expected)."""
    g = np.random.default_rng(808)
    cases = []

    def addsub(op, n, npairs, single):
        a, b = wl.c3(op, n=n * npairs, worst=True)
        want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full((n * npairs,), 7, dtype=torch.int64, device="cuda")
            tc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
            if single:
                f = bn.bn_add if op == "add" else bn.bn_sub
                run = lambda ctx: f(ctx, tr, ta, tb, tc)
            else:
                f = bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch
                run = lambda ctx: f(ctx, tr, ta, tb, n, npairs, tc)
            return run, (tr, tc), (want, wc)
        return make

    for op in ("add", "sub"):
        cases.append((f"bn_{op}", (bn.BN_OP_ADDSUB, 100003, 0, 1), addsub(op, 100003, 1, True)))
        cases.append((f"bn_{op}_n_batch", (bn.BN_OP_ADDSUB, 30011, 0, 5), addsub(op, 30011, 5, False)))

    def addsub_nc(op):
        n, npairs = 40009, 3
        a, b = wl.c3(op, n=n * npairs, worst=True)
        cin = np.array([1, 0, 1], np.uint64)
        want, wc = (oracle.add_nc_batch if op == "add" else oracle.sub_nc_batch)(a, b, n, cin)

        def make():
            ta, tb, tci = D(a), D(b), D(cin)
            tr = torch.full((n * npairs,), 7, dtype=torch.int64, device="cuda")
            tc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
            f = bn.bn_add_nc_n_batch if op == "add" else bn.bn_sub_nc_n_batch
            return (lambda ctx: f(ctx, tr, ta, tb, n, npairs, tci, tc)), (tr, tc), (want, wc)
        return make

    for op in ("add", "sub"):
        cases.append((f"bn_{op}_nc_n_batch", (bn.BN_OP_ADDSUB_NC, 40009, 0, 3), addsub_nc(op)))

    def unequal(op):
        na, nb = 70001, 50021
        a = _rand(g, na)
        a[nb:] = MAX if op == "add" else 0
        b = np.full(nb, MAX, np.uint64)
        bext = np.concatenate([b, np.zeros(na - nb, np.uint64)])
        want, wc = (oracle.add if op == "add" else oracle.sub)(a, bext)

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full((na,), 7, dtype=torch.int64, device="cuda")
            tc = torch.full((1,), 7, dtype=torch.int64, device="cuda")
            f = bn.bn_add_unequal if op == "add" else bn.bn_sub_unequal
            return (lambda ctx: f(ctx, tr, ta, na, tb, nb, tc)), (tr, tc), (want, np.array([wc], np.uint64))
        return make

    for op in ("add", "sub"):
        cases.append((f"bn_{op}_unequal", (bn.BN_OP_ADDSUB_UNEQUAL, 70001, 50021, 1), unequal(op)))

    def unequal_batch(op):
        na, nb, npairs = 30011, 20011, 4
        a = _rand(g, na * npairs)
        b = _rand(g, nb * npairs)
        bext = np.zeros((npairs, na), np.uint64)
        bext[:, :nb] = b.reshape(npairs, nb)
        want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, bext.reshape(-1), na)

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full((na * npairs,), 7, dtype=torch.int64, device="cuda")
            tc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
            f = bn.bn_add_unequal_n_batch if op == "add" else bn.bn_sub_unequal_n_batch
            return (lambda ctx: f(ctx, tr, ta, na, tb, nb, npairs, tc)), (tr, tc), (want, wc)
        return make

    for op in ("add", "sub"):
        cases.append((f"bn_{op}_unequal_n_batch", (bn.BN_OP_ADDSUB_UNEQUAL, 30011, 20011, 4), unequal_batch(op)))

    def sub_abs():
        n, npairs = 3001, 4
        a, b = _rand(g, n * npairs), _rand(g, n * npairs)
        pa = [a[p * n:(p + 1) * n] for p in range(npairs)]
        pb = [b[p * n:(p + 1) * n] for p in range(npairs)]
        sign = np.array([oracle.sub(x, y)[1] for x, y in zip(pa, pb)], np.uint64)
        want = np.concatenate([oracle.sub(y, x)[0] if sg else oracle.sub(x, y)[0]
                               for x, y, sg in zip(pa, pb, sign)])

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full((n * npairs,), 7, dtype=torch.int64, device="cuda")
            ts = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
            return (lambda ctx: bn.bn_sub_abs_n_batch(ctx, tr, ta, tb, n, npairs, ts)), (tr, ts), (want, sign)
        return make

    cases.append(("bn_sub_abs_n_batch", (bn.BN_OP_SUB_ABS, 3001, 0, 4), sub_abs()))

    def mul(form, na, nb, npairs, single, in_place=False):
        a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
        want = oracle.mul_batch(a, b, na, nb, npairs)

        def make():
            tb = D(b)
            if in_place:   # r over a, room for the product
                buf = torch.zeros((na + nb) * npairs, dtype=torch.int64, device="cuda")
                ta = buf[:na * npairs]
                tr = buf
                src = D(a)
                ta.copy_(src)   # run() reloads a first: a refused call then leaves buf as it was

                def run(ctx):
                    ta.copy_(src)
                    bn.bn_mul_n_batch(ctx, tr, ta, tb, na, nb, npairs, form)
                return run, (tr,), (want,)
            ta = D(a)
            tr = torch.full(((na + nb) * npairs,), 7, dtype=torch.int64, device="cuda")
            if single:
                return (lambda ctx: bn.bn_mul(ctx, tr, ta, tb, form)), (tr,), (want,)
            return (lambda ctx: bn.bn_mul_n_batch(ctx, tr, ta, tb, na, nb, npairs, form)), (tr,), (want,)
        return make

    for form in ("mad", "mfma"):
        op = bn.BN_OP_MUL
        cases.append((f"bn_mul {form}", (op, 3000, 1700, 1, form), mul(form, 3000, 1700, 1, True)))
        cases.append((f"bn_mul_n_batch {form}", (op, 900, 700, 6, form), mul(form, 900, 700, 6, False)))
        cases.append((f"bn_mul_n_batch {form} in place", (op | bn.BN_OP_IN_PLACE, 900, 700, 6, form),
                      mul(form, 900, 700, 6, False, in_place=True)))

    def karatsuba(levels):
        n, npairs = 2048, 3
        a, b = _rand(g, n * npairs), _rand(g, n * npairs)
        want = oracle.mul_batch(a, b, n, n, npairs)

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full((2 * n * npairs,), 7, dtype=torch.int64, device="cuda")
            return (lambda ctx: bn.bn_mul_karatsuba_n_batch(ctx, tr, ta, tb, n, npairs, levels, "mfma")), (tr,), \
                (want,)
        return make

    for levels in (1, 2):
        cases.append((f"bn_mul_karatsuba_n_batch levels={levels}",
                      (bn.BN_OP_MUL_KARATSUBA, 2048, 2048, 3, "mfma", levels), karatsuba(levels)))

    def karatsuba_unequal():
        na, nb, npairs = 1501, 1100, 3
        a, b = _rand(g, na * npairs), _rand(g, nb * npairs)
        want = oracle.mul_batch(a, b, na, nb, npairs)

        def make():
            ta, tb = D(a), D(b)
            tr = torch.full(((na + nb) * npairs,), 7, dtype=torch.int64, device="cuda")
            return (lambda ctx: bn.bn_mul_karatsuba_batch(ctx, tr, ta, na, tb, nb, npairs, 2, "mfma")), (tr,), \
                (want,)
        return make

    cases.append(("bn_mul_karatsuba_batch 1501x1100 levels=2",
                  (bn.BN_OP_MUL_KARATSUBA, 1501, 1100, 3, "mfma", 2), karatsuba_unequal()))
    return cases


CASES = _cases()


def _capture(run, ctx, s):
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
        run(ctx)
    return graph


def _check(outs, wants, what):
    torch.cuda.synchronize()
    for o, w in zip(outs, wants):
        got = H(o)
        assert (got == np.asarray(w, np.uint64)).all(), f"{what}: first bad at {np.argmax(got != w)}"


@pytest.mark.parametrize("name,reserve,make", CASES, ids=[c[0] for c in CASES])
def test_strict_context_enospace_then_captured(name, reserve, make):
    announce("strict workspace", name)
    run, outs, wants = make()
    ctx = bn.bn_create(0)
    try:
        before = [o.clone() for o in outs]
        with pytest.raises(bn.BnError) as e:
            run(ctx)
        assert e.value.status == bn.BN_ENOSPACE, name
        torch.cuda.synchronize()
        for o, b in zip(outs, before):       # nothing was enqueued
            assert torch.equal(o, b), f"{name}: output changed by a refused call"
        assert bn.bn_workspace_size(ctx, *reserve) > 0
        bn.bn_reserve_for(ctx, *reserve)
        s = torch.cuda.Stream()
        graph = _capture(run, ctx, s)
        for rep in range(3):
            for o in outs:
                o.fill_(7)
            torch.cuda.synchronize()
            graph.replay()
            _check(outs, wants, f"{name} replay {rep}")
            run(ctx)                           # eager call of the same shape between replays
            _check(outs, wants, f"{name} eager after replay {rep}")
        del graph
    finally:
        torch.cuda.synchronize()
        bn.bn_destroy(ctx)


def test_ragged_plan_reserves_its_large_items():
    """A ragged plan with products above one wave's size reserves the workspace when it
    is built: bn_mul_ragged then runs inside a capture on a strict context."""
    announce("strict workspace, ragged plan with large items")
    g = np.random.default_rng(3)
    sizes = [(5, 9), (300, 200), (40, 33), (700, 650), (128, 128)]
    desc, A, B = [], [], []
    ao = bo = ro = 0
    for na, nb in sizes:
        desc.append((ao, bo, ro, na, nb))
        A.append(_rand(g, na))
        B.append(_rand(g, nb))
        ao, bo, ro = ao + na, bo + nb, ro + na + nb
    a, b = np.concatenate(A), np.concatenate(B)
    want = oracle.mul_ragged(a, b, np.array(desc, np.uint64), ro)
    ctx = bn.bn_create(0)
    try:
        ta, tb = D(a), D(b)
        tr = torch.zeros(ro, dtype=torch.int64, device="cuda")
        for form in ("mad", "mfma", "auto"):
            plan = bn.bn_plan_mul_ragged(ctx, desc, form)
            try:
                s = torch.cuda.Stream()
                graph = _capture(lambda c: bn.bn_mul_ragged(c, plan, tr, ta, tb), ctx, s)
                for rep in range(3):
                    tr.zero_()
                    torch.cuda.synchronize()
                    graph.replay()
                    _check((tr,), (want,), f"ragged {form} replay {rep}")
                del graph
            finally:
                bn.bn_plan_destroy(plan)
    finally:
        torch.cuda.synchronize()
        bn.bn_destroy(ctx)


def test_auto_grow_refuses_growth_during_capture():
    """With auto_grow the call grows the workspace eagerly, but never inside a capture:
    there it returns BN_ECAPTURE."""
    announce("auto_grow and capture")
    ctx = bn.bn_create(0, auto_grow=True)
    try:
        a, b = wl.c3("add", n=100003)
        ta, tb = D(a), D(b)
        tr = torch.empty(a.size, dtype=torch.int64, device="cuda")
        s = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with pytest.raises(bn.BnError) as e:
            with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
                bn.bn_add(ctx, tr, ta, tb)
        assert e.value.status == bn.BN_ECAPTURE
        del graph
        torch.cuda.synchronize()
        bn.bn_add(ctx, tr, ta, tb)   # eager: grows, then exact
        _check((tr,), (oracle.add(a, b)[0],), "eager add after growth")
    finally:
        torch.cuda.synchronize()
        bn.bn_destroy(ctx)


@pytest.mark.parametrize("n,npairs", [(4, 1088), (64, 1 << 12), (1, 5000), (128, 33)])
def test_independent_tile_batches_need_no_workspace(n, npairs):
    """Batches whose pair length divides the 128-limb tile run as independent tiles:
    they publish no status words, so a fresh strict context runs them unreserved."""
    announce("unreserved independent-tile batch", n, npairs)
    g = np.random.default_rng(n * 7919 + npairs)
    a, b = _rand(g, n * npairs), _rand(g, n * npairs)
    ctx = bn.bn_create(0)
    try:
        assert bn.bn_workspace_size(ctx, bn.BN_OP_ADDSUB, n, n, npairs) == 0
        assert bn.bn_workspace_size(ctx, bn.BN_OP_ADDSUB, 3, 3, npairs) > 0   # 3 does not divide 128: chained
        for op in ("add", "sub"):
            ta, tb = D(a), D(b)
            tr = torch.full((n * npairs,), 7, dtype=torch.int64, device="cuda")
            tc = torch.full((npairs,), 7, dtype=torch.int64, device="cuda")
            (bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch)(ctx, tr, ta, tb, n, npairs, tc)
            want, wc = (oracle.add_batch if op == "add" else oracle.sub_batch)(a, b, n)
            _check((tr, tc), (want, wc), f"unreserved {op} {n}x{npairs}")
    finally:
        torch.cuda.synchronize()
        bn.bn_destroy(ctx)
