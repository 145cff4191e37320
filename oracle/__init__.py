"""CPU oracle for large-number add / sub / mul (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``bn_oracle.c`` (plain C, 128-bit
intermediates) through ctypes and shares nothing with the GPU library.

Every function takes and returns numpy ``uint64`` arrays of little-endian limbs
(limb 0 least significant, radix 2^64), the number format of the paper's
Sec. 2.1 and Theorem 1.

Parity status: every function is pinned by ``tests/test_oracle.py`` against
CPython's arbitrary-precision ``int`` (an independent library routine), closed
forms, algebraic identities, residues and emulations of the paper's
Algorithms 1 and 2; the ragged forms against per-pair ``int`` sums and products
over pooled arrays with gaps, unsorted offsets and empty pairs.  Planted mistakes
(dropped carry, wrong borrow, dropped top carry, stray term, ignored carry-in,
misread ragged descriptors) are compiled into mutant copies of the C source and
each fails a pin.  No function is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_sz = ctypes.c_size_t


def build() -> str:
    """Compile the oracle with plain gcc (no vectorisation flags)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.bnref_add_n.restype = ctypes.c_uint64
    lib.bnref_add_n.argtypes = [_u64p, _u64p, _u64p, _sz]
    lib.bnref_sub_n.restype = ctypes.c_uint64
    lib.bnref_sub_n.argtypes = [_u64p, _u64p, _u64p, _sz]
    lib.bnref_mul.restype = None
    lib.bnref_mul.argtypes = [_u64p, _u64p, _sz, _u64p, _sz]
    for f in (lib.bnref_add_n_batch, lib.bnref_sub_n_batch):
        f.restype = None
        f.argtypes = [_u64p, _u64p, _u64p, _sz, _sz, _u64p]
    for f in (lib.bnref_add_nc_batch, lib.bnref_sub_nc_batch):
        f.restype = None
        f.argtypes = [_u64p, _u64p, _u64p, _sz, _sz, _u64p, _u64p]
    lib.bnref_mul_n_batch.restype = None
    lib.bnref_mul_n_batch.argtypes = [_u64p, _u64p, _u64p, _sz, _sz, _sz]
    lib.bnref_mul_ragged.restype = None
    lib.bnref_mul_ragged.argtypes = [_u64p, _u64p, _u64p, _u64p, _sz]
    lib.bnref_add_ragged.restype = None
    lib.bnref_add_ragged.argtypes = [_u64p, _u64p, _u64p, _u64p, _sz, _u64p]
    _lib = lib
    return lib


def _c(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype != np.uint64:
        raise TypeError(f"oracle expects uint64 limbs, got {x.dtype}")
    return x


def _p(x: np.ndarray):
    return x.ctypes.data_as(_u64p)


def add(a: np.ndarray, b: np.ndarray):
    """(a + b) mod 2^(64n) and the carry-out, n = len(a) = len(b)."""
    a, b = _c(a), _c(b)
    if a.shape != b.shape:
        raise ValueError("add needs equal limb counts")
    r = np.empty_like(a)
    c = _load().bnref_add_n(_p(r), _p(a), _p(b), a.size)
    return r, int(c)


def sub(a: np.ndarray, b: np.ndarray):
    """(a - b) mod 2^(64n) and the borrow-out [a < b]."""
    a, b = _c(a), _c(b)
    if a.shape != b.shape:
        raise ValueError("sub needs equal limb counts")
    r = np.empty_like(a)
    c = _load().bnref_sub_n(_p(r), _p(a), _p(b), a.size)
    return r, int(c)


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a * b as exactly len(a) + len(b) limbs."""
    a, b = _c(a), _c(b)
    r = np.empty(a.size + b.size, dtype=np.uint64)
    _load().bnref_mul(_p(r), _p(a), a.size, _p(b), b.size)
    return r


def add_batch(a: np.ndarray, b: np.ndarray, n: int):
    """Uniform batch: pair p is limbs [p*n, (p+1)*n).  Returns (r, carry[npairs])."""
    a, b = _c(a), _c(b)
    if a.size != b.size or (n and a.size % n):
        raise ValueError("bad batch shape")
    npairs = a.size // n if n else 0
    r = np.empty_like(a)
    c = np.empty(npairs, dtype=np.uint64)
    _load().bnref_add_n_batch(_p(r), _p(a), _p(b), n, npairs, _p(c))
    return r, c


def sub_batch(a: np.ndarray, b: np.ndarray, n: int):
    a, b = _c(a), _c(b)
    if a.size != b.size or (n and a.size % n):
        raise ValueError("bad batch shape")
    npairs = a.size // n if n else 0
    r = np.empty_like(a)
    c = np.empty(npairs, dtype=np.uint64)
    _load().bnref_sub_n_batch(_p(r), _p(a), _p(b), n, npairs, _p(c))
    return r, c


def add_nc_batch(a: np.ndarray, b: np.ndarray, n: int, cin: np.ndarray):
    """Uniform batch with a carry into limb 0 of pair p (cin[p] in {0, 1})."""
    a, b, cin = _c(a), _c(b), _c(cin)
    if a.size != b.size or (n and a.size % n):
        raise ValueError("bad batch shape")
    npairs = a.size // n if n else 0
    if cin.size != npairs:
        raise ValueError("one carry-in per pair")
    r = np.empty_like(a)
    c = np.empty(npairs, dtype=np.uint64)
    _load().bnref_add_nc_batch(_p(r), _p(a), _p(b), n, npairs, _p(cin), _p(c))
    return r, c


def sub_nc_batch(a: np.ndarray, b: np.ndarray, n: int, bin_: np.ndarray):
    """Uniform batch with a borrow into limb 0 of pair p (bin_[p] in {0, 1})."""
    a, b, bin_ = _c(a), _c(b), _c(bin_)
    if a.size != b.size or (n and a.size % n):
        raise ValueError("bad batch shape")
    npairs = a.size // n if n else 0
    if bin_.size != npairs:
        raise ValueError("one borrow-in per pair")
    r = np.empty_like(a)
    c = np.empty(npairs, dtype=np.uint64)
    _load().bnref_sub_nc_batch(_p(r), _p(a), _p(b), n, npairs, _p(bin_), _p(c))
    return r, c


def mul_batch(a: np.ndarray, b: np.ndarray, na: int, nb: int, npairs: int) -> np.ndarray:
    a, b = _c(a), _c(b)
    if a.size != na * npairs or b.size != nb * npairs:
        raise ValueError("bad batch shape")
    r = np.empty((na + nb) * npairs, dtype=np.uint64)
    _load().bnref_mul_n_batch(_p(r), _p(a), _p(b), na, nb, npairs)
    return r


def mul_ragged(a_pool, b_pool, desc, r_size: int) -> np.ndarray:
    """desc: uint64 array [npairs, 5] = (a_off, b_off, r_off, na, nb)."""
    a_pool, b_pool = _c(a_pool), _c(b_pool)
    desc = _c(np.asarray(desc, dtype=np.uint64).reshape(-1, 5))
    r = np.zeros(r_size, dtype=np.uint64)
    _load().bnref_mul_ragged(_p(r), _p(a_pool), _p(b_pool), _p(desc), desc.shape[0])
    return r


def add_ragged(a_pool, b_pool, desc, r_size: int):
    a_pool, b_pool = _c(a_pool), _c(b_pool)
    desc = _c(np.asarray(desc, dtype=np.uint64).reshape(-1, 5))
    r = np.zeros(r_size, dtype=np.uint64)
    c = np.empty(desc.shape[0], dtype=np.uint64)
    _load().bnref_add_ragged(_p(r), _p(a_pool), _p(b_pool), _p(desc), desc.shape[0], _p(c))
    return r, c
