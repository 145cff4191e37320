"""C-ABI library: it loads, it exports every entry point include/bn.h declares, and
host-side argument checks that need no GPU behave (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bn.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bn_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def bn():
    import paper_2604_21566_amd as bn
    if not os.path.exists(bn.LIB_PATH):
        from paper_2604_21566_amd import build as b
        b.build(verbose=False)
    return bn


def test_header_declares_the_core_calls():
    names = _declared()
    for core in ("bn_add", "bn_sub", "bn_mul", "bn_add_n_batch", "bn_sub_n_batch", "bn_mul_n_batch",
                 "bn_plan_mul_ragged", "bn_mul_ragged", "bn_graph_capture_mul_ragged", "bn_autotune"):
        assert core in names


def test_library_exports_every_declared_symbol(bn):
    L = bn.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared calls
    assert sorted(bn.EXPORTED) == _declared()


def test_host_library_exports_every_declared_symbol():
    """libbn_host.so (DoT on the host CPU) against include/bn_host.h."""
    from paper_2604_21566_amd import host
    if not os.path.exists(host.LIB_PATH):
        from paper_2604_21566_amd import build as b
        b.build_host(verbose=False)
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "bn_host.h")).read(), flags=re.S)
    declared = sorted(set(re.findall(r"\b(bnh_[a-z0-9_]+)\s*\(", src)))
    L = host.lib()
    assert declared and not [n for n in declared if not hasattr(L, n)]
    assert host.EXPORTED == declared


def test_strerror_and_version(bn):
    assert bn.bn_strerror(bn.BN_OK) == "ok"
    assert "overlap" in bn.bn_strerror(bn.BN_EALIAS)
    assert bn.bn_strerror(123) == "unknown status"
    assert "gfx950" in bn.bn_version()
    assert "mul.crossover_limbs" in bn.bn_param_names()


def test_null_context_is_rejected_without_touching_a_device(bn):
    L = bn.lib()
    assert L.bn_add(None, None, None, None, 0, None, None) == bn.BN_EINVAL
    assert L.bn_mul(None, None, None, 0, None, 0, 0, None) == bn.BN_EINVAL
    assert L.bn_set_param(None, b"mul.crossover_limbs", 5) == bn.BN_EINVAL
    assert L.bn_lookback_stats(None, None, None, 0) == bn.BN_EINVAL
    assert L.bn_probe_rates(None, None, None, None) == bn.BN_EINVAL
    assert L.bn_create(None, 0, None) == bn.BN_EINVAL
    assert L.bn_reserve_for(None, bn.BN_OP_MUL, 4, 4, 1, 0, 0) == bn.BN_EINVAL
    assert L.bn_workspace_size(None, bn.BN_OP_MUL, 4, 4, 1, 0, 0) == 0
    assert L.bn_plan_destroy(None) == bn.BN_OK
    assert L.bn_graph_destroy(None) == bn.BN_OK
    assert L.bn_destroy(None) == bn.BN_OK


def test_create_without_gfx950_reports_unsupported(bn):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert bn.lib().bn_create(ctypes.byref(ctx), 0, None) in (bn.BN_EUNSUPPORTED, bn.BN_EINVAL)


def test_product_path_fails_loudly_when_library_missing(tmp_path, monkeypatch):
    import paper_2604_21566_amd as bn
    monkeypatch.setattr(bn, "_lib", None)
    monkeypatch.setattr(bn, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(bn.BnLibraryMissing):
        bn.lib()


def test_karatsuba_auto_levels(bn):
    """BN_KARATSUBA_AUTO's level rule: split (halves of ceil(m/2) limbs) while the operand
    has at least 2 limbs and the halves keep min_half_limbs limbs, at most
    BN_KARATSUBA_MAX_LEVELS levels."""
    f = bn.bn_karatsuba_auto_levels
    assert f(16384, 4096) == 2          # C5: 8192, 4096
    assert f(16384, 4097) == 1
    assert f(8191, 4096) == 1           # 4096 (odd: the high half is zero-extended)
    assert f(8191, 4097) == 0
    assert f(12000, 1000) == 3          # 6000, 3000, 1500 (750 < 1000)
    assert f(12001, 1000) == 3          # 6001, 3001, 1501 (751 < 1000)
    assert f(12000, 1) == bn.BN_KARATSUBA_MAX_LEVELS   # 6000 ... 47
    assert f(3, 2) == 1 and f(3, 3) == 0  # 2, then 1 < 2
    assert f(1 << 20, 1) == bn.BN_KARATSUBA_MAX_LEVELS
    assert f(0, 4096) == 0 and f(1, 0) == 0 and f(2, 0) == 1
