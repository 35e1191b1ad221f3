"""Helpers for the GPU parity tests: run the library through the C ABI and
compare its rows with the oracle's, element by element after sorting by key."""
from __future__ import annotations

import numpy as np

import oracle


def lib_spec_args(wl):
    return dict(record_bytes=wl.record_bytes, keys=list(wl.key_fields), aggs=list(wl.aggs))


def run_lib(records: np.ndarray, record_bytes: int, keys, aggs, batches: int = 1, **kw):
    """Upload `records`, aggregate them in `batches` consume calls, return (keys u64, cols, stats)."""
    import torch
    import paper_1311_0059_amd as P

    raw = np.ascontiguousarray(records).view(np.uint8).reshape(-1)
    n = raw.size // record_bytes
    dev = torch.from_numpy(raw.copy()).to("cuda") if raw.size else torch.empty(16, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()  # the library works on its own stream
    spec = P.make_spec(record_bytes, keys, aggs, **kw)
    with P.GroupBy(spec) as g:
        bounds = np.linspace(0, n, batches + 1).astype(np.int64)
        for b in range(batches):
            lo, hi = int(bounds[b]), int(bounds[b + 1])
            if hi > lo:
                g.consume_ptr(dev.data_ptr() + lo * record_bytes, hi - lo)
        g.finish()
        k, c = g.rows("cpu")
        st = g.stats()
    torch.cuda.synchronize()
    keys_u = k.numpy().view(np.uint64)
    cols = c.numpy()
    order = np.argsort(keys_u, kind="stable")
    return keys_u[order], cols[:, order], st


def assert_rows_equal(got_keys, got_cols, want_keys, want_cols, label=""):
    assert got_keys.shape == want_keys.shape, f"{label}: {got_keys.size} rows vs oracle {want_keys.size}"
    if not np.array_equal(got_keys, want_keys):
        bad = np.nonzero(got_keys != want_keys)[0][:5]
        raise AssertionError(f"{label}: keys differ at {bad.tolist()}")
    for a in range(want_cols.shape[0]):
        if not np.array_equal(got_cols[a], want_cols[a]):
            bad = np.nonzero(got_cols[a] != want_cols[a])[0][:5]
            raise AssertionError(f"{label}: aggregate {a} differs at rows {bad.tolist()}: "
                                 f"{got_cols[a][bad].tolist()} vs {want_cols[a][bad].tolist()}")


def check_against_oracle(records, spec_oracle, got_keys, got_cols, label=""):
    want_keys, want_cols = oracle.groupby(records, spec_oracle)
    assert_rows_equal(got_keys, got_cols, want_keys, want_cols, label)
