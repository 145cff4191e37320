"""Binding of libbn_host.so: DoT addition and subtraction on the host CPU (Sec. 3.1,
Algorithm 1, with AVX-512 or AVX2), a comparison point beside the GPU library.

Same names as include/bn_host.h; arguments are C-contiguous numpy uint64 arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbn_host.so")

BNH_OK = 0
BNH_EINVAL = -1
BNH_EUNSUPPORTED = -6
BNH_ISA_SCALAR = 0
BNH_ISA_AVX2 = 1
BNH_ISA_AVX512 = 2
ISA_NAMES = {BNH_ISA_SCALAR: "scalar", BNH_ISA_AVX2: "avx2", BNH_ISA_AVX512: "avx512"}

_u64p = ctypes.POINTER(ctypes.c_uint64)
_sz = ctypes.c_size_t
_PROTOS = {
    "bnh_isa_best": (ctypes.c_int, []),
    "bnh_add_n": (ctypes.c_int, [_u64p, _u64p, _u64p, _sz, ctypes.c_uint64, _u64p, ctypes.c_int]),
    "bnh_sub_n": (ctypes.c_int, [_u64p, _u64p, _u64p, _sz, ctypes.c_uint64, _u64p, ctypes.c_int]),
    "bnh_add_n_batch": (ctypes.c_int, [_u64p, _u64p, _u64p, _sz, _sz, _u64p, ctypes.c_int, ctypes.c_int]),
    "bnh_sub_n_batch": (ctypes.c_int, [_u64p, _u64p, _u64p, _sz, _sz, _u64p, ctypes.c_int, ctypes.c_int]),
}
EXPORTED = sorted(_PROTOS)


class BnhError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: status {status}")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _p(x):
    if x is None:
        return None
    if x.dtype != np.uint64 or not x.flags.c_contiguous:
        raise TypeError("expected a C-contiguous uint64 array")
    return x.ctypes.data_as(_u64p)


def _ck(st, what):
    if st != BNH_OK:
        raise BnhError(st, what)


def bnh_isa_best() -> int:
    return lib().bnh_isa_best()


def _one(fn, r, a, b, c_in, isa):
    out = ctypes.c_uint64(0)
    _ck(getattr(lib(), fn)(_p(r), _p(a), _p(b), a.size, c_in, ctypes.byref(out), isa), fn)
    return out.value


def bnh_add_n(r, a, b, carry_in=0, isa=None):
    """r = a + b + carry_in over a.size limbs; returns the carry out."""
    return _one("bnh_add_n", r, a, b, carry_in, bnh_isa_best() if isa is None else isa)


def bnh_sub_n(r, a, b, borrow_in=0, isa=None):
    """r = a - b - borrow_in (mod 2^(64 n)); returns the borrow out."""
    return _one("bnh_sub_n", r, a, b, borrow_in, bnh_isa_best() if isa is None else isa)


def _batch(fn, r, a, b, n, npairs, carry, isa, threads):
    _ck(getattr(lib(), fn)(_p(r), _p(a), _p(b), n, npairs, _p(carry), bnh_isa_best() if isa is None else isa,
                           threads), fn)


def bnh_add_n_batch(r, a, b, n, npairs, carry_out=None, isa=None, threads=1):
    _batch("bnh_add_n_batch", r, a, b, n, npairs, carry_out, isa, threads)


def bnh_sub_n_batch(r, a, b, n, npairs, carry_out=None, isa=None, threads=1):
    _batch("bnh_sub_n_batch", r, a, b, n, npairs, carry_out, isa, threads)
