"""Conversions between limb arrays and CPython ints (used by the tests only).

CPython's arbitrary-precision int is an arithmetic library independent of the
oracle; the tests pin the oracle against it.
"""
import numpy as np

MASK64 = (1 << 64) - 1


def to_int(x) -> int:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    return int.from_bytes(x.astype("<u8").tobytes(), "little")


def from_int(v: int, n: int) -> np.ndarray:
    v &= (1 << (64 * n)) - 1
    return np.frombuffer(v.to_bytes(8 * n, "little"), dtype="<u8").astype(np.uint64) if n else np.zeros(0, np.uint64)
