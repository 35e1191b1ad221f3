"""ORACLE -- test infrastructure only.

A plain CPU group-by (C, sort-then-scan, `oracle.c`) and the paper's analytic
formulas, used to check the GPU library.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package; the library and
its Python binding never do, and the two share no code.

Contents:
  groupby(records, spec)        -- the result rows (the paper, Sec. 3.1; method of Sec. 4.1, Phase 2)
  groupby_par(records, spec)    -- the same rows on all host threads (the sort split by leading key bits)
  host_threads(), cpu_model()   -- the thread count groupby_par uses by default, and the host CPU's name
  rows_for_keys(records, spec, keys) -- the rows of chosen keys by one scan (sampled checks at full size)
  totals(records, spec)         -- whole-input COUNT / wrap-around SUM / MIN / MAX (invariants)
  yao_i_key, yao_i_raw          -- Appendix, input component (Yao's formula, draws without replacement)
  hybrid_hash_partitions        -- Sec. 4.3, Formula (1)
  spilled_fraction              -- Sec. 5.3.1 / 5.3.4 I/O model: share of records spilled, 1 - K/G_t
  slot_filter_false_positive    -- Sec. 4.3.4 / 5.3.4: alpha of a one-byte filter per hash-table slot

A spec here is the oracle's own plain description:
  {"record_bytes": int, "keys": [(offset, type)], "aggs": [(op, offset, type)]}
with type in {"u32","u64","i32","i64"} and op in {"COUNT","SUM","MIN","MAX"}.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_TYPES = {"u32": 0, "u64": 1, "i32": 2, "i64": 3}
_OPS = {"COUNT": 0, "SUM": 1, "MIN": 2, "MAX": 3}

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc -O2; pthreads for groupby_par) next to its source."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        lib.oracle_groupby.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, u64, vp, vp]
        lib.oracle_groupby.restype = ctypes.c_int64
        lib.oracle_groupby_par.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, u64, vp, vp, u32, u32]
        lib.oracle_groupby_par.restype = ctypes.c_int64
        lib.oracle_rows_for_keys.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, vp, u64, vp, vp]
        lib.oracle_rows_for_keys.restype = ctypes.c_int
        lib.oracle_totals.argtypes = [vp, u64, u32, u32, vp, vp, vp, vp]
        lib.oracle_totals.restype = ctypes.c_int
        _lib = lib
    return _lib


def _u32(xs) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))


def _spec_arrays(spec):
    koff = _u32([o for o, _ in spec["keys"]])
    ktype = _u32([_TYPES[t] for _, t in spec["keys"]])
    op = _u32([_OPS[o] for o, _, _ in spec["aggs"]])
    ioff = _u32([off for _, off, _ in spec["aggs"]])
    itype = _u32([_TYPES[t] for _, _, t in spec["aggs"]])
    return koff, ktype, op, ioff, itype


def _raw(records: np.ndarray, rb: int) -> np.ndarray:
    buf = np.ascontiguousarray(records).view(np.uint8).reshape(-1)
    if buf.size % rb:
        raise ValueError("record buffer is not a whole number of records")
    return buf


def groupby(records: np.ndarray, spec) -> tuple[np.ndarray, np.ndarray]:
    """Rows sorted by key: (keys u64[G], cols i64[n_aggs, G])."""
    rb = spec["record_bytes"]
    buf = _raw(records, rb)
    n = buf.size // rb
    koff, ktype, op, ioff, itype = _spec_arrays(spec)
    na = len(spec["aggs"])
    cap = max(n, 1)
    keys = np.empty(cap, dtype=np.uint64)
    cols = np.empty((na, cap), dtype=np.int64)
    rows = _load().oracle_groupby(buf.ctypes.data, n, rb, len(spec["keys"]), koff.ctypes.data, ktype.ctypes.data, na,
                                  op.ctypes.data, ioff.ctypes.data, itype.ctypes.data, cap, keys.ctypes.data,
                                  cols.ctypes.data)
    if rows < 0:
        raise ValueError("oracle: invalid spec")
    return keys[:rows].copy(), cols[:, :rows].copy()


def host_threads() -> int:
    """Threads for groupby_par: OMP_NUM_THREADS when set (the host's share of cores), else the
    cores this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def groupby_par(records: np.ndarray, spec, threads: int | None = None, bits: int = 12):
    """The rows of groupby (sorted by key), computed on `threads` threads (default host_threads()).
    `bits` is the width of the leading-key-bits digit that splits the sort (1..16)."""
    rb = spec["record_bytes"]
    buf = _raw(records, rb)
    n = buf.size // rb
    koff, ktype, op, ioff, itype = _spec_arrays(spec)
    na = len(spec["aggs"])
    cap = max(n, 1)
    keys = np.empty(cap, dtype=np.uint64)
    cols = np.empty((na, cap), dtype=np.int64)
    t = host_threads() if threads is None else threads
    rows = _load().oracle_groupby_par(buf.ctypes.data, n, rb, len(spec["keys"]), koff.ctypes.data, ktype.ctypes.data,
                                      na, op.ctypes.data, ioff.ctypes.data, itype.ctypes.data, cap, keys.ctypes.data,
                                      cols.ctypes.data, t, bits)
    if rows < 0:
        raise ValueError("oracle: invalid spec, thread count or digit width, or out of memory")
    return keys[:rows], cols[:, :rows]


def rows_for_keys(records: np.ndarray, spec, qkeys) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(sorted query keys, record counts per key, cols i64[n_aggs, nq]) by one scan of all records."""
    rb = spec["record_bytes"]
    buf = _raw(records, rb)
    n = buf.size // rb
    q = np.unique(np.asarray(qkeys, dtype=np.uint64))
    koff, ktype, op, ioff, itype = _spec_arrays(spec)
    na = len(spec["aggs"])
    found = np.zeros(q.size, dtype=np.uint64)
    cols = np.zeros((na, max(q.size, 1)), dtype=np.int64)
    rc = _load().oracle_rows_for_keys(buf.ctypes.data, n, rb, len(spec["keys"]), koff.ctypes.data, ktype.ctypes.data,
                                      na, op.ctypes.data, ioff.ctypes.data, itype.ctypes.data, q.ctypes.data, q.size,
                                      found.ctypes.data, cols.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid spec")
    return q, found, cols[:, :q.size]


def totals(records: np.ndarray, spec) -> np.ndarray:
    """Per aggregate: COUNT -> n, SUM -> wrap-around total, MIN/MAX -> global extreme."""
    rb = spec["record_bytes"]
    buf = _raw(records, rb)
    n = buf.size // rb
    _, _, op, ioff, itype = _spec_arrays(spec)
    out = np.zeros(len(spec["aggs"]), dtype=np.int64)
    _load().oracle_totals(buf.ctypes.data, n, rb, len(spec["aggs"]), op.ctypes.data, ioff.ctypes.data,
                          itype.ctypes.data, out.ctypes.data)
    return out


# ---- the paper's analytic quantities -------------------------------------------------------------

def yao_i_key(r: float, n: float, m: float) -> float:
    """Appendix, input component, Eq. (key_dep): expected distinct keys among r records drawn
    without replacement from a dataset of n records holding m distinct keys: m(1 - (1 - r/n)^(n/m))."""
    return m * (1.0 - (1.0 - r / n) ** (n / m))


def yao_i_raw(k: float, n: float, m: float) -> float:
    """Appendix, input component, Eq. (raw_dep): expected records drawn until k distinct keys
    have been seen: n(1 - (1 - k/m)^(m/n))."""
    return n * (1.0 - (1.0 - k / m) ** (m / n))


def hybrid_hash_partitions(G: float, M: float, F: float = 1.2) -> int:
    """Sec. 4.3, Formula (1): spilling partitions P = (G*F - M) / (M - 2), read as
    max(0, ceil(.)) -- P = 0 means everything is aggregated in memory.  Needs M > 2."""
    if M <= 2:
        raise ValueError("Formula (1) needs M > 2")
    return max(0, math.ceil((G * F - M) / (M - 2)))


def slot_filter_false_positive(K: float, H: float, bits: int = 8) -> float:
    """Sec. 4.3.4 / 5.3.4: the false-positive ratio alpha of a filter of `bits` bits per slot of
    a table of H slots holding K keys, where each key sets one bit (chosen by its hash) in the
    filter of its home slot.  An absent key tests the bit its own hash chooses in its own home
    slot's filter; with independent uniform hashes that bit is set with probability
    1 - (1 - 1/(bits H))^K."""
    return 1.0 - (1.0 - 1.0 / (bits * H)) ** K


def spilled_fraction(K: float, G_t: float) -> float:
    """Sec. 5.3.1 / 5.3.4: with K groups resident out of G_t (uniform keys), the share of input
    records that is spilled, from C_IO = R + (R - K/G_t * R)."""
    return max(0.0, 1.0 - K / G_t)
