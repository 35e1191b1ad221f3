"""Seeded synthetic inputs for group-by workloads (shared test/bench infrastructure).

The C source `datagen.c` holds the generator; this module compiles it (gcc,
OpenMP) on first use if `libdatagen.so` is missing, and wraps it for numpy.
It holds none of the aggregation method's arithmetic: it only produces input
bytes.  Workload recipes (sizes, distributions, value ranges, budgets) live in
`datagen.workloads`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "datagen.c")
_LIB_PATH = os.path.join(_HERE, "libdatagen.so")

UNIFORM, ZIPF, HEAVY = 0, 1, 2

R16 = np.dtype([("key", "<u8"), ("v", "<i8")])
R24 = np.dtype([("k1", "<u4"), ("k2", "<u4"), ("v1", "<i8"), ("v2", "<i4"), ("v3", "<i4")])

_lib = None


def build(force: bool = False) -> str:
    """Compile libdatagen.so next to its source."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i64, f64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        lib.dg_keys.argtypes = [u64, u64, u64, i32, f64, vp]
        lib.dg_ranks.argtypes = [u64, u64, u64, i32, f64, vp]
        lib.dg_values.argtypes = [u64, u64, u64, i64, i64, vp]
        lib.dg_r16.argtypes = [u64, u64, u64, i32, f64, i64, i64, vp]
        lib.dg_r24.argtypes = [u64, u64, u64, i32, f64, i64, i64, vp]
        lib.dg_loguniform.argtypes = [u64, u64, u64, f64, f64, vp]
        lib.dg_uniform_f64.argtypes = [u64, u64, u64, f64, f64, vp]
        for f in (lib.dg_keys, lib.dg_ranks, lib.dg_values, lib.dg_r16, lib.dg_r24, lib.dg_loguniform, lib.dg_uniform_f64):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int):
    if rc != 0:
        raise ValueError("datagen: invalid arguments")


def keys(seed: int, n: int, d: int, dist: int = UNIFORM, s: float = 0.0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(_load().dg_keys(seed, n, d, dist, s, _ptr(out)))
    return out


def ranks(seed: int, n: int, d: int, dist: int = UNIFORM, s: float = 0.0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(_load().dg_ranks(seed, n, d, dist, s, _ptr(out)))
    return out


def values(seed: int, tag: int, n: int, lo: int, hi: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _check(_load().dg_values(seed, tag, n, lo, hi, _ptr(out)))
    return out


def r16(seed: int, n: int, d: int, dist: int = UNIFORM, s: float = 0.0, lo: int = 0, hi: int = 999,
        out: np.ndarray | None = None) -> np.ndarray:
    """n R16 records {u64 key, i64 v}; exactly d distinct keys; v uniform in [lo, hi]."""
    if out is None:
        out = np.empty(n, dtype=R16)
    assert out.dtype == R16 and out.size >= n and out.flags.c_contiguous
    if n:
        _check(_load().dg_r16(seed, n, d, dist, s, lo, hi, _ptr(out)))
    return out[:n]


def r24(seed: int, n: int, d: int, dist: int = UNIFORM, s: float = 0.0, lo1: int = -10**9, hi1: int = 10**9,
        out: np.ndarray | None = None) -> np.ndarray:
    """n R24 records {u32 k1, u32 k2, i64 v1, i32 v2, i32 v3}; exactly d distinct (k1, k2)."""
    if out is None:
        out = np.empty(n, dtype=R24)
    assert out.dtype == R24 and out.size >= n and out.flags.c_contiguous
    if n:
        _check(_load().dg_r24(seed, n, d, dist, s, lo1, hi1, _ptr(out)))
    return out[:n]


def loguniform_ints(seed: int, tag: int, n: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(_load().dg_loguniform(seed, tag, n, lo, hi, _ptr(out)))
    return out


def uniform_f64(seed: int, tag: int, n: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _check(_load().dg_uniform_f64(seed, tag, n, lo, hi, _ptr(out)))
    return out


def checksum(buf: np.ndarray) -> str:
    """Order-sensitive 64-bit digest of the raw bytes (logged so that runs can be compared)."""
    import hashlib
    return hashlib.blake2b(memoryview(np.ascontiguousarray(buf)).cast("B"), digest_size=8).hexdigest()
