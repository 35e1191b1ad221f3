"""Test-side helpers: workload -> spec conversions and the brute-force pin.

The oracle and the library each take their own spec; these helpers build both
from one workload description so a test can feed the same bytes to each.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def oracle_spec(wl) -> dict:
    return {"record_bytes": wl.record_bytes, "keys": list(wl.key_fields), "aggs": list(wl.aggs)}


def make_spec(record_bytes, keys, aggs) -> dict:
    return {"record_bytes": record_bytes, "keys": list(keys), "aggs": list(aggs)}


def _read(rec: bytes, off: int, typ: str) -> int:
    if typ == "u32":
        return int.from_bytes(rec[off:off + 4], "little", signed=False)
    if typ == "i32":
        return int.from_bytes(rec[off:off + 4], "little", signed=True)
    if typ == "u64":
        return int.from_bytes(rec[off:off + 8], "little", signed=False)
    return int.from_bytes(rec[off:off + 8], "little", signed=True)


def brute_force(records: np.ndarray, spec: dict):
    """Python dict group-by, written independently of the oracle (pure Python ints).

    Keys: one field, or two u32 fields combined as k1 * 2^32 + k2.  COUNT counts,
    SUM wraps modulo 2^64, MIN/MAX use the input's signedness; 32-bit inputs
    widen to 64 bits.  Returns rows sorted by key as (keys, cols) like the oracle.
    """
    rb = spec["record_bytes"]
    raw = np.ascontiguousarray(records).view(np.uint8).tobytes()
    n = len(raw) // rb
    groups: dict[int, list] = {}
    for i in range(n):
        rec = raw[i * rb:(i + 1) * rb]
        ks = [_read(rec, o, t) for o, t in spec["keys"]]
        k = ks[0] if len(ks) == 1 else (ks[0] << 32) + ks[1]
        k &= MASK64
        st = groups.get(k)
        vals = [_read(rec, o, t) for _, o, t in spec["aggs"]]
        if st is None:
            st = []
            for (op, _, _), v in zip(spec["aggs"], vals):
                st.append(1 if op == "COUNT" else v)
            groups[k] = st
            continue
        for j, ((op, _, _), v) in enumerate(zip(spec["aggs"], vals)):
            if op == "COUNT":
                st[j] += 1
            elif op == "SUM":
                st[j] = (st[j] + v) & MASK64
            elif op == "MIN":
                st[j] = min(st[j], v)
            else:
                st[j] = max(st[j], v)
    keys = sorted(groups)
    cols = np.zeros((len(spec["aggs"]), len(keys)), dtype=np.int64)
    for r, k in enumerate(keys):
        for j, v in enumerate(groups[k]):
            v &= MASK64
            cols[j, r] = np.int64(v - (1 << 64) if v >= (1 << 63) else v)
    return np.array(keys, dtype=np.uint64), cols


def canonical_keys(records: np.ndarray, layout: str) -> np.ndarray:
    if layout == "R16":
        return records["key"].astype(np.uint64)
    return (records["k1"].astype(np.uint64) << np.uint64(32)) | records["k2"].astype(np.uint64)


def sort_rows(keys: np.ndarray, cols: np.ndarray):
    order = np.argsort(keys, kind="stable")
    return keys[order], cols[:, order]
