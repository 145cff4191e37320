"""MI355X (gfx950) large-number add / sub / mul -- Python binding of libbn.so.

A thin ctypes layer over the C ABI declared in ``include/bn.h``: every function
has the C name, converts its arguments (torch device tensors -> device pointers,
torch streams -> hipStream_t) and calls the library.  All arithmetic runs in the
library's HIP kernels; there is no fallback path.  If ``libbn.so`` has not been
built, every call raises ``BnLibraryMissing``.

Operands are contiguous torch tensors of dtype int64 or uint64 on a ROCm device,
holding little-endian 64-bit limbs (limb 0 least significant).  PyTorch is used
for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbn.so")

BN_OK = 0
BN_EINVAL = -1
BN_EALIAS = -2
BN_ERANGE = -3
BN_ENOMEM = -4
BN_EHIP = -5
BN_EUNSUPPORTED = -6
BN_ECAPTURE = -7
BN_ENOSPACE = -8

BN_OP_ADDSUB = 0
BN_OP_ADDSUB_NC = 1
BN_OP_ADDSUB_UNEQUAL = 2
BN_OP_SUB_ABS = 3
BN_OP_MUL = 4
BN_OP_MUL_KARATSUBA = 5
BN_OP_IN_PLACE = 0x100

BN_MUL_AUTO = 0
BN_MUL_MAD = 1
BN_MUL_MFMA = 2
BN_KARATSUBA_AUTO = -1
BN_KARATSUBA_MAX_LEVELS = 8

FORMS = {"auto": BN_MUL_AUTO, "mad": BN_MUL_MAD, "mfma": BN_MUL_MFMA}


class BnLibraryMissing(RuntimeError):
    pass


class BnError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {bn_strerror(status)} ({status})")


class bn_pair(ctypes.Structure):
    _fields_ = [("a_off", ctypes.c_uint64), ("b_off", ctypes.c_uint64), ("r_off", ctypes.c_uint64),
                ("na", ctypes.c_uint32), ("nb", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i = ctypes.c_int
_PROTOS = {
    "bn_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.c_char_p]),
    "bn_destroy": (_i, [_vp]),
    "bn_strerror": (ctypes.c_char_p, [_i]),
    "bn_version": (ctypes.c_char_p, []),
    "bn_reserve": (_i, [_vp, _sz]),
    "bn_reserve_for": (_i, [_vp, _i, _sz, _sz, _sz, _i, _i]),
    "bn_workspace_size": (_sz, [_vp, _i, _sz, _sz, _sz, _i, _i]),
    "bn_check": (_i, [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)]),
    "bn_lookback_stats": (_i, [_vp, _vp, ctypes.POINTER(ctypes.c_uint64), _sz]),
    "bn_probe_rates": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double)]),
    "bn_add": (_i, [_vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "bn_sub": (_i, [_vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "bn_add_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _vp, _vp]),
    "bn_sub_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _vp, _vp]),
    "bn_addsub_n_batch_noalloc": (_i, [_vp, _i, _vp, _vp, _vp, _sz, _sz, _vp, _vp]),
    "bn_add_nc_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _vp, _vp, _vp]),
    "bn_sub_nc_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _vp, _vp, _vp]),
    "bn_add_unequal": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _vp, _vp]),
    "bn_sub_unequal": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _vp, _vp]),
    "bn_add_unequal_n_batch": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _sz, _vp, _vp]),
    "bn_sub_unequal_n_batch": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _sz, _vp, _vp]),
    "bn_sub_abs_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _vp, _vp]),
    "bn_mul": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _i, _vp]),
    "bn_mul_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _sz, _i, _vp]),
    "bn_mul_karatsuba_n_batch": (_i, [_vp, _vp, _vp, _vp, _sz, _sz, _i, _i, _vp]),
    "bn_mul_karatsuba_batch": (_i, [_vp, _vp, _vp, _sz, _vp, _sz, _sz, _i, _i, _vp]),
    "bn_karatsuba_auto_levels": (_i, [_sz, _sz]),
    "bn_plan_mul_ragged": (_i, [_vp, ctypes.POINTER(bn_pair), _sz, _i, ctypes.POINTER(_vp)]),
    "bn_plan_add_ragged": (_i, [_vp, ctypes.POINTER(bn_pair), _sz, ctypes.POINTER(_vp)]),
    "bn_plan_destroy": (_i, [_vp]),
    "bn_mul_ragged": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "bn_add_ragged": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bn_graph_capture_mul_ragged": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "bn_graph_capture_batch": (_i, [_vp, _i, _vp, _vp, _vp, _sz, _sz, _sz, _vp, _i, _vp, ctypes.POINTER(_vp)]),
    "bn_graph_launch": (_i, [_vp, _vp]),
    "bn_graph_destroy": (_i, [_vp]),
    "bn_set_param": (_i, [_vp, ctypes.c_char_p, ctypes.c_int64]),
    "bn_get_param": (_i, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]),
    "bn_param_names": (ctypes.c_char_p, []),
    "bn_autotune": (_i, [_vp, ctypes.c_char_p]),
    "bn_load_tuning": (_i, [_vp, ctypes.c_char_p]),
}
EXPORTED = tuple(_PROTOS)

_lib = None


def lib():
    """The loaded libbn.so (raises BnLibraryMissing if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BnLibraryMissing(f"{LIB_PATH} not built; run __graft_entry__.build() or "
                                   "python paper_2604_21566_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ck(st: int, what: str):
    if st != BN_OK:
        raise BnError(st, what)


def bn_strerror(st: int) -> str:
    try:
        return lib().bn_strerror(st).decode()
    except BnLibraryMissing:
        return f"status {st}"


def bn_version() -> str:
    return lib().bn_version().decode()


# ------------------------------------------------------------------ marshalling ----
_torch = None      # the torch module, imported on first use
_LIMB_DTYPES = ()  # int64, uint64


def _tm():
    global _torch, _LIMB_DTYPES
    if _torch is None:
        import torch
        _LIMB_DTYPES = (torch.int64, torch.uint64)
        _torch = torch
    return _torch


def _ptr(t, what: str, need: int | None = None):
    """Device pointer of a contiguous int64/uint64 torch tensor (None -> NULL).  `need`:
    the limbs the call will touch through this pointer; a smaller tensor is refused
    here, because a device pointer carries no extent that the library could check."""
    if t is None:
        return None
    torch = _tm()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must live on the GPU")
    if t.dtype not in _LIMB_DTYPES:
        raise TypeError(f"{what}: limbs must be int64/uint64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    n = t.numel()
    if need is not None and n < need:
        raise ValueError(f"{what}: tensor holds {n} limbs, the call touches {need}")
    return t.data_ptr() if n else None


def _stream(stream):
    """The hipStream_t of `stream` (a torch stream or a raw handle); None: torch's current
    stream on the current device (read through torch's raw-stream query, a tenth of the
    host cost of building a torch.cuda.Stream object, when this torch has it)."""
    if stream is None:
        torch = _tm()
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        dev = getattr(torch._C, "_cuda_getDevice", None)
        if raw is not None and dev is not None:
            return raw(dev())
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ context ----
def bn_create(device: int = 0, tuning: str | None = None, auto_grow: bool = False):
    """A context on `device`; `tuning`: a file written by bn_autotune, or None.
    auto_grow=True sets "workspace.auto_grow": compute calls then grow a short
    workspace themselves (allocation + device sync) instead of failing with
    BN_ENOSPACE."""
    ctx = _vp()
    _ck(lib().bn_create(ctypes.byref(ctx), device, tuning.encode() if tuning else None), "bn_create")
    if auto_grow:
        bn_set_param(ctx, "workspace.auto_grow", 1)
    return ctx


def bn_destroy(ctx):
    _ck(lib().bn_destroy(ctx), "bn_destroy")


def bn_reserve(ctx, nbytes: int):
    _ck(lib().bn_reserve(ctx, nbytes), "bn_reserve")


def bn_reserve_for(ctx, op: int, na: int, nb: int = 0, npairs: int = 1, form=BN_MUL_AUTO, levels: int = 0):
    """Size every workspace buffer for one call shape (host-synchronous)."""
    _ck(lib().bn_reserve_for(ctx, op, na, nb, npairs, _form(form), levels), "bn_reserve_for")


def bn_workspace_size(ctx, op: int, na: int, nb: int = 0, npairs: int = 1, form=BN_MUL_AUTO,
                      levels: int = 0) -> int:
    return lib().bn_workspace_size(ctx, op, na, nb, npairs, _form(form), levels)


def bn_check(ctx, stream=None) -> int:
    """Synchronise the stream, read and clear the device latch; returns its flags
    (bit 0: a look-back computed an unpublished predecessor's carry itself)."""
    flags = ctypes.c_uint32(0)
    _ck(lib().bn_check(ctx, _stream(stream), ctypes.byref(flags)), "bn_check")
    return flags.value


BN_LOOKBACK_BINS = 32


def bn_lookback_stats(ctx, stream=None):
    """Look-back distance histogram since the last call (recorded while debug.flags
    bit 1 is set): entry k counts tiles decided 2^k..2^(k+1)-1 tiles back."""
    h = (ctypes.c_uint64 * BN_LOOKBACK_BINS)()
    _ck(lib().bn_lookback_stats(ctx, _stream(stream), h, BN_LOOKBACK_BINS), "bn_lookback_stats")
    return [int(x) for x in h]


def bn_probe_rates(ctx):
    """Measured (mac96 per s, int8 MFMA ops per s, streaming copy bytes per s) of the
    context's device."""
    m, f, c = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _ck(lib().bn_probe_rates(ctx, ctypes.byref(m), ctypes.byref(f), ctypes.byref(c)), "bn_probe_rates")
    return m.value, f.value, c.value


def bn_set_param(ctx, key: str, value: int):
    _ck(lib().bn_set_param(ctx, key.encode(), int(value)), f"bn_set_param({key})")


def bn_get_param(ctx, key: str) -> int:
    v = ctypes.c_int64(0)
    _ck(lib().bn_get_param(ctx, key.encode(), ctypes.byref(v)), f"bn_get_param({key})")
    return v.value


def bn_param_names():
    return lib().bn_param_names().decode().split(",")


def bn_autotune(ctx, out_json: str | None = None):
    _ck(lib().bn_autotune(ctx, out_json.encode() if out_json else None), "bn_autotune")


def bn_load_tuning(ctx, path: str):
    _ck(lib().bn_load_tuning(ctx, path.encode()), "bn_load_tuning")


# ------------------------------------------------------------------ add / sub ----
def bn_add(ctx, r, a, b, carry_out=None, stream=None):
    """r = a + b (one pair, n = a.numel() limbs); carry_out: 1-limb tensor or None."""
    n = a.numel()
    _ck(lib().bn_add(ctx, _ptr(r, "r", n), _ptr(a, "a"), _ptr(b, "b", n), n, _ptr(carry_out, "carry", 1),
                     _stream(stream)), "bn_add")


def bn_sub(ctx, r, a, b, borrow_out=None, stream=None):
    n = a.numel()
    _ck(lib().bn_sub(ctx, _ptr(r, "r", n), _ptr(a, "a"), _ptr(b, "b", n), n, _ptr(borrow_out, "borrow", 1),
                     _stream(stream)), "bn_sub")


def bn_add_n_batch(ctx, r, a, b, n: int, npairs: int, carry_out=None, stream=None):
    N = n * npairs
    _ck(lib().bn_add_n_batch(ctx, _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n, npairs,
                             _ptr(carry_out, "carry", npairs),
                             _stream(stream)), "bn_add_n_batch")


def bn_sub_n_batch(ctx, r, a, b, n: int, npairs: int, borrow_out=None, stream=None):
    N = n * npairs
    _ck(lib().bn_sub_n_batch(ctx, _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n, npairs,
                             _ptr(borrow_out, "borrow", npairs),
                             _stream(stream)), "bn_sub_n_batch")


BN_SCRATCH_MAX_TILES = 1 << 17


def bn_addsub_n_batch_noalloc(ctx, sub: int, r, a, b, n: int, npairs: int, carry_out=None, stream=None):
    """bn_add_n_batch (sub=0) / bn_sub_n_batch (sub=1) with the look-back state in the
    library's fixed per-GPU array: no allocation, no workspace."""
    N = n * npairs
    _ck(lib().bn_addsub_n_batch_noalloc(ctx, int(sub), _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n,
                                        npairs, _ptr(carry_out, "carry", npairs), _stream(stream)),
        "bn_addsub_n_batch_noalloc")


# ------------------------------------------------------------------ multiply ----
def _form(form):
    return FORMS[form] if isinstance(form, str) else int(form)


def bn_mul(ctx, r, a, b, form=BN_MUL_AUTO, stream=None):
    _ck(lib().bn_mul(ctx, _ptr(r, "r", a.numel() + b.numel()), _ptr(a, "a"), a.numel(), _ptr(b, "b"), b.numel(),
                     _form(form),
                     _stream(stream)), "bn_mul")


def bn_mul_n_batch(ctx, r, a, b, na: int, nb: int, npairs: int, form=BN_MUL_AUTO, stream=None):
    _ck(lib().bn_mul_n_batch(ctx, _ptr(r, "r", (na + nb) * npairs), _ptr(a, "a", na * npairs),
                             _ptr(b, "b", nb * npairs), na, nb, npairs, _form(form),
                             _stream(stream)), "bn_mul_n_batch")


def bn_add_nc_n_batch(ctx, r, a, b, n: int, npairs: int, carry_in, carry_out=None, stream=None):
    N = n * npairs
    _ck(lib().bn_add_nc_n_batch(ctx, _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n, npairs,
                                _ptr(carry_in, "carry_in", npairs), _ptr(carry_out, "carry_out", npairs),
                                _stream(stream)), "bn_add_nc_n_batch")


def bn_sub_nc_n_batch(ctx, r, a, b, n: int, npairs: int, borrow_in, borrow_out=None, stream=None):
    N = n * npairs
    _ck(lib().bn_sub_nc_n_batch(ctx, _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n, npairs,
                                _ptr(borrow_in, "borrow_in", npairs), _ptr(borrow_out, "borrow_out", npairs),
                                _stream(stream)),
        "bn_sub_nc_n_batch")


def bn_add_unequal(ctx, r, a, na: int, b, nb: int, carry_out=None, stream=None):
    _ck(lib().bn_add_unequal(ctx, _ptr(r, "r", na), _ptr(a, "a", na), na, _ptr(b, "b", nb), nb,
                             _ptr(carry_out, "carry_out", 1),
                             _stream(stream)), "bn_add_unequal")


def bn_sub_unequal(ctx, r, a, na: int, b, nb: int, borrow_out=None, stream=None):
    _ck(lib().bn_sub_unequal(ctx, _ptr(r, "r", na), _ptr(a, "a", na), na, _ptr(b, "b", nb), nb,
                             _ptr(borrow_out, "borrow_out", 1),
                             _stream(stream)), "bn_sub_unequal")


def bn_add_unequal_n_batch(ctx, r, a, na: int, b, nb: int, npairs: int, carry_out=None, stream=None):
    """Pair p: a[p na:(p+1) na] + b[p nb:(p+1) nb] (zero-extended) -> r[p na:(p+1) na]."""
    _ck(lib().bn_add_unequal_n_batch(ctx, _ptr(r, "r", na * npairs), _ptr(a, "a", na * npairs), na,
                                     _ptr(b, "b", nb * npairs), nb, npairs, _ptr(carry_out, "carry_out", npairs),
                                     _stream(stream)), "bn_add_unequal_n_batch")


def bn_sub_unequal_n_batch(ctx, r, a, na: int, b, nb: int, npairs: int, borrow_out=None, stream=None):
    _ck(lib().bn_sub_unequal_n_batch(ctx, _ptr(r, "r", na * npairs), _ptr(a, "a", na * npairs), na,
                                     _ptr(b, "b", nb * npairs), nb, npairs, _ptr(borrow_out, "borrow_out", npairs),
                                     _stream(stream)), "bn_sub_unequal_n_batch")


def bn_sub_abs_n_batch(ctx, r, a, b, n: int, npairs: int, sign=None, stream=None):
    N = n * npairs
    _ck(lib().bn_sub_abs_n_batch(ctx, _ptr(r, "r", N), _ptr(a, "a", N), _ptr(b, "b", N), n, npairs,
                                 _ptr(sign, "sign", npairs),
                                 _stream(stream)), "bn_sub_abs_n_batch")


def bn_mul_karatsuba_n_batch(ctx, r, a, b, n: int, npairs: int, levels: int, form=BN_MUL_AUTO, stream=None):
    _ck(lib().bn_mul_karatsuba_n_batch(ctx, _ptr(r, "r", 2 * n * npairs), _ptr(a, "a", n * npairs),
                                       _ptr(b, "b", n * npairs), n, npairs, int(levels),
                                       _form(form), _stream(stream)), "bn_mul_karatsuba_n_batch")


def bn_mul_karatsuba_batch(ctx, r, a, na: int, b, nb: int, npairs: int, levels: int, form=BN_MUL_AUTO,
                           stream=None):
    """Pair p: a[p na:(p+1) na] x b[p nb:(p+1) nb] -> r[p (na+nb):(p+1) (na+nb)]."""
    _ck(lib().bn_mul_karatsuba_batch(ctx, _ptr(r, "r", (na + nb) * npairs), _ptr(a, "a", na * npairs), na,
                                     _ptr(b, "b", nb * npairs), nb, npairs, int(levels), _form(form),
                                     _stream(stream)), "bn_mul_karatsuba_batch")


def bn_karatsuba_auto_levels(n: int, min_half_limbs: int) -> int:
    """Levels BN_KARATSUBA_AUTO uses for n-limb operands (host only)."""
    return lib().bn_karatsuba_auto_levels(n, min_half_limbs)


# ------------------------------------------------------------------ ragged ----
def _pairs(desc):
    """desc: array-like [npairs, 5] of (a_off, b_off, r_off, na, nb)."""
    d = np.asarray(desc, dtype=np.uint64).reshape(-1, 5)
    arr = (bn_pair * len(d))()
    for i, (ao, bo, ro, na, nb) in enumerate(d.tolist()):
        arr[i] = bn_pair(ao, bo, ro, na, nb)
    return arr, len(d)


# pool extents (limbs) each live plan's calls touch: (a, b, r, pairs)
_PLAN_EXTENTS: dict = {}


def _extents(desc, mul: bool):
    d = np.asarray(desc, dtype=np.int64).reshape(-1, 5)
    if len(d) == 0:
        return (0, 0, 0, 0)
    a_off, b_off, r_off, na, nb = d.T
    r_len = na + nb if mul else na
    return (int((a_off + na).max()), int((b_off + nb).max()), int((r_off + r_len).max()), len(d))


def bn_plan_mul_ragged(ctx, desc, form=BN_MUL_AUTO):
    arr, n = _pairs(desc)
    plan = _vp()
    _ck(lib().bn_plan_mul_ragged(ctx, arr, n, _form(form), ctypes.byref(plan)), "bn_plan_mul_ragged")
    _PLAN_EXTENTS[plan.value] = _extents(desc, True)
    return plan


def bn_plan_add_ragged(ctx, desc):
    arr, n = _pairs(desc)
    plan = _vp()
    _ck(lib().bn_plan_add_ragged(ctx, arr, n, ctypes.byref(plan)), "bn_plan_add_ragged")
    _PLAN_EXTENTS[plan.value] = _extents(desc, False)
    return plan


def bn_plan_destroy(plan):
    _PLAN_EXTENTS.pop(getattr(plan, "value", None), None)
    _ck(lib().bn_plan_destroy(plan), "bn_plan_destroy")


def _pools(plan, r_pool, a_pool, b_pool):
    ea, eb, er, _ = _PLAN_EXTENTS.get(getattr(plan, "value", None), (None, None, None, None))
    return _ptr(r_pool, "r", er), _ptr(a_pool, "a", ea), _ptr(b_pool, "b", eb)


def bn_mul_ragged(ctx, plan, r_pool, a_pool, b_pool, stream=None):
    _ck(lib().bn_mul_ragged(ctx, plan, *_pools(plan, r_pool, a_pool, b_pool), _stream(stream)), "bn_mul_ragged")


def bn_add_ragged(ctx, plan, r_pool, a_pool, b_pool, carry_out=None, stream=None):
    npairs = _PLAN_EXTENTS.get(getattr(plan, "value", None), (0, 0, 0, None))[3]
    _ck(lib().bn_add_ragged(ctx, plan, *_pools(plan, r_pool, a_pool, b_pool), _ptr(carry_out, "carry", npairs),
                            _stream(stream)), "bn_add_ragged")


# ------------------------------------------------------------------ graphs ----
def bn_graph_capture_mul_ragged(ctx, plan, r_pool, a_pool, b_pool, stream):
    g = _vp()
    _ck(lib().bn_graph_capture_mul_ragged(ctx, plan, *_pools(plan, r_pool, a_pool, b_pool), _stream(stream),
                                          ctypes.byref(g)), "bn_graph_capture_mul_ragged")
    return g


def bn_graph_capture_batch(ctx, op: int, r, a, b, na: int, nb: int, npairs: int, carry_out=None,
                           form=BN_MUL_AUTO, stream=None):
    g = _vp()
    rn = (na + nb) * npairs if op == 2 else na * npairs
    _ck(lib().bn_graph_capture_batch(ctx, op, _ptr(r, "r", rn), _ptr(a, "a", na * npairs),
                                     _ptr(b, "b", (nb if op == 2 else na) * npairs), na, nb, npairs,
                                     _ptr(carry_out, "carry", npairs), _form(form), _stream(stream),
                                     ctypes.byref(g)),
        "bn_graph_capture_batch")
    return g


def bn_graph_launch(graph, stream=None):
    _ck(lib().bn_graph_launch(graph, _stream(stream)), "bn_graph_launch")


def bn_graph_destroy(graph):
    _ck(lib().bn_graph_destroy(graph), "bn_graph_destroy")


# ------------------------------------------------------------------ helpers ----
def to_device(x: np.ndarray, device="cuda"):
    """numpy uint64 limbs -> torch int64 device tensor (same bits)."""
    import torch
    x = np.ascontiguousarray(x, dtype=np.uint64)
    return torch.from_numpy(x.view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    """torch int64/uint64 device tensor -> numpy uint64 limbs."""
    import torch
    if t.dtype == torch.uint64:
        t = t.view(torch.int64)
    return t.detach().cpu().numpy().view(np.uint64)
