"""The in-library autotuner runs on the device, writes a table that a fresh context
loads back, and results stay exact with the tuned parameters."""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2604_21566_amd as bn
from conftest import announce
from paper_2604_21566_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("addsub.batch_waves", "addsub.batch_rows", "addsub.chain_waves", "addsub.chain_rows",
        "mul.crossover_limbs", "mul.small_crossover_limbs", "mul.mad_xchunk", "mul.mfma_chunk", "mul.mfma_rows")


def test_autotune_roundtrip(tmp_path):
    announce("autotune")
    path = str(tmp_path / "tune.json")
    ctx = bn.bn_create(0)
    try:
        bn.bn_autotune(ctx, path)
        tuned = {k: bn.bn_get_param(ctx, k) for k in KEYS}
    finally:
        bn.bn_destroy(ctx)
    table = json.load(open(path))
    for k in KEYS:
        assert table[k] == tuned[k]
    ctx = bn.bn_create(0, tuning=path)   # the table loaded at creation
    try:
        assert {k: bn.bn_get_param(ctx, k) for k in KEYS} == tuned
        # exact results with the tuned table: batched add, one long add, AUTO multiply
        # (a context without auto_grow: every call's workspace reserved first)
        bn.bn_reserve_for(ctx, bn.BN_OP_ADDSUB, 64, 0, 3000)
        bn.bn_reserve_for(ctx, bn.BN_OP_ADDSUB, 1 << 17, 0, 1)
        for n in (16, 300, 2000):
            bn.bn_reserve_for(ctx, bn.BN_OP_MUL, n, n, 2, "auto")
        a, b = wl.c2("add", npairs=3000)
        ta, tb = bn.to_device(a), bn.to_device(b)
        tr = torch.empty_like(ta)
        tc = torch.empty(3000, dtype=torch.int64, device="cuda")
        bn.bn_add_n_batch(ctx, tr, ta, tb, 64, 3000, tc)
        a3, b3 = wl.c3("add", n=1 << 17)
        t3 = torch.empty(a3.size, dtype=torch.int64, device="cuda")
        bn.bn_add(ctx, t3, bn.to_device(a3), bn.to_device(b3))
        g = np.random.default_rng(1)
        for n in (16, 300, 2000):
            x = g.integers(0, 2 ** 64 - 1, n * 2, dtype=np.uint64, endpoint=True)
            y = g.integers(0, 2 ** 64 - 1, n * 2, dtype=np.uint64, endpoint=True)
            r = torch.empty(4 * n, dtype=torch.int64, device="cuda")
            bn.bn_mul_n_batch(ctx, r, bn.to_device(x), bn.to_device(y), n, n, 2, "auto")
            torch.cuda.synchronize()
            assert (bn.to_host(r) == oracle.mul_batch(x, y, n, n, 2)).all(), n
        torch.cuda.synchronize()
        rr, rc = oracle.add_batch(a, b, 64)
        assert (bn.to_host(tr) == rr).all() and (bn.to_host(tc) == rc).all()
        r3, _ = oracle.add(a3, b3)
        assert (bn.to_host(t3) == r3).all()
    finally:
        bn.bn_destroy(ctx)


def test_probe_rates_are_plausible(bnctx):
    """The measured ceilings sit between a tenth of and just above the published
    figures (VALU: 256 CUs x 64 lanes x 2.4 GHz per full-rate op; int8 MFMA 5.0 POPS)."""
    mac, mfma, copy = bn.bn_probe_rates(bnctx)
    assert 1e12 < mac < 4.0e13, mac
    assert 5e14 < mfma < 5.5e15, mfma
    assert 1e12 < copy < 8.0e12, copy  # HBM3E: 8 TB/s published


def test_load_tuning_all_or_nothing(tmp_path):
    """A table with a rejected value changes nothing, also the entries before it;
    a good table applies every entry.  bn_create refuses a bad table."""
    announce("load tuning: all or nothing")
    ctx = bn.bn_create(0)
    try:
        before = {k: bn.bn_get_param(ctx, k) for k in KEYS}
        bad = tmp_path / "bad.json"
        bad.write_text(json.dumps({"device": "gfx950", "mul.crossover_limbs": before["mul.crossover_limbs"] + 1,
                                   "mul.mfma_rows": 3}))   # 1 or 2 only
        with pytest.raises(bn.BnError) as e:
            bn.bn_load_tuning(ctx, str(bad))
        assert e.value.status == bn.BN_EINVAL
        assert {k: bn.bn_get_param(ctx, k) for k in KEYS} == before
        with pytest.raises(bn.BnError):
            bn.bn_load_tuning(ctx, str(tmp_path / "missing.json"))
        good = tmp_path / "good.json"
        good.write_text(json.dumps({"device": "gfx950", "mul.crossover_limbs": before["mul.crossover_limbs"] + 1,
                                    "mul.mfma_rows": 1}))
        bn.bn_load_tuning(ctx, str(good))
        assert bn.bn_get_param(ctx, "mul.crossover_limbs") == before["mul.crossover_limbs"] + 1
        assert bn.bn_get_param(ctx, "mul.mfma_rows") == 1
    finally:
        bn.bn_destroy(ctx)
    for path in (bad, tmp_path / "missing.json"):
        with pytest.raises(bn.BnError) as e:
            bn.bn_create(0, tuning=str(path))
        assert e.value.status == bn.BN_EINVAL
