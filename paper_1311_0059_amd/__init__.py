"""aggx: bounded-memory hash GROUP BY on AMD MI355X (gfx950).

A thin binding of the C ABI in include/aggx.h.  Every step of the operator runs
in the native library's HIP kernels; this module only marshals arguments.
PyTorch supplies device memory and streams (torch is imported first so that the
library binds to the same HIP runtime).  There is no CPU fallback: without the
built library, or without a GPU, the calls raise.
"""
from __future__ import annotations

import ctypes

import torch  # noqa: F401  (must be loaded before the native library)

from . import _native as N

__all__ = ["AggError", "GroupBy", "Batch", "Server", "make_spec", "load_library", "min_budget", "query_noalloc",
           "EXPORTS"]

EXPORTS = N.EXPORTS


class AggError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        name = N.STATUS.get(status, str(status))
        msg = load_library().agg_strerror(status).decode()
        super().__init__(f"{what}: {name} ({msg})" if what else f"{name} ({msg})")


def load_library():
    return N.load()


def _check(rc: int, what: str):
    if rc != 0:
        raise AggError(rc, what)


def make_spec(record_bytes: int, keys, aggs, budget: int = 0, est_groups: int = 0, workspace=None,
              stream=None, fanout_bits: int = 0, load_pct: int = 0, policy: str = "destage",
              preagg: str = "auto", engine: str = "auto") -> N.Spec:
    """keys: [(offset, type)]; aggs: [(op, offset, type)]; types "u32","u64","i32","i64";
    ops "COUNT","SUM","MIN","MAX".  workspace: optional device tensor of >= budget bytes."""
    s = N.Spec()
    s.record_bytes = record_bytes
    s.n_keys = len(keys)
    for i, (off, t) in enumerate(keys):
        s.keys[i].offset = off
        s.keys[i].type = N.TYPES[t]
    s.n_aggs = len(aggs)
    for i, (op, off, t) in enumerate(aggs):
        s.aggs[i].op = N.OPS[op]
        s.aggs[i].in_.offset = off
        s.aggs[i].in_.type = N.TYPES[t]
    s.budget_bytes = budget
    s.est_groups = est_groups
    if workspace is not None:
        s.device_workspace = workspace.data_ptr()
        s.workspace_bytes = workspace.numel() * workspace.element_size()
    if stream is not None:
        s.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    s.fanout_bits = fanout_bits
    s.load_pct = load_pct
    s.policy = N.POLICIES[policy]
    s.preagg = {"auto": 0, "on": 1, "off": 2}[preagg]
    s.engine = {"auto": 0, "tables": 1, "lds": 2, "owner": 3, "sorted": 4, "onchip": 5}[engine]
    return s


def min_budget(spec: N.Spec) -> int:
    return int(load_library().agg_min_budget(ctypes.byref(spec)))


_hip = None


def _hip_rt():
    """The HIP runtime already loaded by torch (same soname), for device copies of results."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


class GroupBy:
    """One GROUP BY query: create -> consume(batch)* -> finish -> rows."""

    def __init__(self, spec: N.Spec):
        self._lib = load_library()
        self._spec = spec
        self._h = ctypes.c_void_p()
        _check(self._lib.agg_create(ctypes.byref(spec), ctypes.byref(self._h)), "agg_create")
        self._res = None

    @classmethod
    def from_args(cls, *args, **kw) -> "GroupBy":
        return cls(make_spec(*args, **kw))

    def consume(self, records: torch.Tensor, n: int | None = None):
        """records: contiguous device tensor holding n packed records (any dtype)."""
        if not records.is_cuda:
            raise ValueError("records must be a device tensor")
        if not records.is_contiguous():
            raise ValueError("records must be contiguous")
        nbytes = records.numel() * records.element_size()
        rb = self._spec.record_bytes
        if n is None:
            n = nbytes // rb
        if n * rb > nbytes:
            raise ValueError("tensor holds fewer than n records")
        _check(self._lib.agg_consume(self._h, ctypes.c_void_p(records.data_ptr()), n), "agg_consume")

    def consume_ptr(self, ptr: int, n: int):
        _check(self._lib.agg_consume(self._h, ctypes.c_void_p(ptr), n), "agg_consume")

    def first_result(self) -> N.Result:
        """agg_first_rows: descriptor of the rows finished in memory at level 0 (device
        memory owned by the handle), before the recursion over spilled partitions."""
        res = N.Result()
        _check(self._lib.agg_first_rows(self._h, ctypes.byref(res)), "agg_first_rows")
        return res

    def first_rows(self, device: str = "cpu"):
        """The level-0 rows copied out: (keys as int64 view of u64, cols [n_aggs, n])."""
        return _copy_rows(self.first_result(), self._spec.n_aggs, device)

    def finish(self) -> N.Result:
        res = N.Result()
        _check(self._lib.agg_finish(self._h, ctypes.byref(res)), "agg_finish")
        self._res = res
        return res

    def stats(self) -> dict:
        st = N.Stats()
        _check(self._lib.agg_get_stats(self._h, ctypes.byref(st)), "agg_get_stats")
        return st.as_dict()

    def rows(self, device: str = "cpu"):
        """(keys int64 tensor holding the u64 bit patterns, cols int64 tensor [n_aggs, rows])."""
        res = self._res if self._res is not None else self.finish()
        n = int(res.n_rows)
        na = self._spec.n_aggs
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        cols = torch.empty((na, n), dtype=torch.int64, device="cuda")
        if n:
            rt = _hip_rt()
            torch.cuda.synchronize()
            _check(rt.hipMemcpy(keys.data_ptr(), res.d_keys, n * 8, 3), "hipMemcpy")
            for a in range(na):
                _check(rt.hipMemcpy(cols[a].data_ptr(), res.d_cols[a], n * 8, 3), "hipMemcpy")
        return keys.to(device), cols.to(device)

    def close(self):
        if self._h:
            self._lib.agg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_rows(res, na: int, device: str):
    n = int(res.n_rows)
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    cols = torch.empty((na, n), dtype=torch.int64, device="cuda")
    if n:
        rt = _hip_rt()
        torch.cuda.synchronize()
        _check(rt.hipMemcpy(keys.data_ptr(), res.d_keys, n * 8, 3), "hipMemcpy")
        for a in range(na):
            _check(rt.hipMemcpy(cols[a].data_ptr(), res.d_cols[a], n * 8, 3), "hipMemcpy")
    return keys.to(device), cols.to(device)


def query_noalloc(spec: N.Spec, ptr: int, n: int, out_keys, out_cols) -> int:
    """One whole query through agg_query_noalloc (no allocation in the library): `out_keys`
    (int64 device tensor) and `out_cols` (int64 device tensor [n_aggs, cap]) receive the rows;
    returns the row count.  Raises AggError (its .status) on a library error."""
    cap = out_keys.numel()
    if out_cols.shape[0] != spec.n_aggs or out_cols.shape[1] != cap or not out_cols.is_contiguous():
        raise ValueError("out_cols must be a contiguous [n_aggs, len(out_keys)] tensor")
    cols = (ctypes.c_void_p * max(1, spec.n_aggs))(*[out_cols[a].data_ptr() for a in range(spec.n_aggs)])
    rows = ctypes.c_uint64()
    rc = load_library().agg_query_noalloc(ctypes.byref(spec), ctypes.c_void_p(ptr), n,
                                          ctypes.c_void_p(out_keys.data_ptr()), cols, cap, ctypes.byref(rows))
    if rc != 0:
        err = AggError(rc, "agg_query_noalloc")
        err.rows = rows.value
        raise err
    return rows.value


class Batch:
    """Many independent instances in one persistent launch (agg_batch_*)."""

    def __init__(self, spec: N.Spec, instances):
        """instances: iterable of (device pointer, n records, estimated groups or 0)."""
        self._lib = load_library()
        self._spec = spec
        inst = list(instances)
        arr = (N.Instance * max(len(inst), 1))()
        for i, (ptr, n, est) in enumerate(inst):
            arr[i].d_records = ptr
            arr[i].n = n
            arr[i].est_groups = est
        self._n = len(inst)
        self._b = ctypes.c_void_p()
        _check(self._lib.agg_batch_create(ctypes.byref(spec), arr, len(inst), ctypes.byref(self._b)),
               "agg_batch_create")

    def run(self):
        _check(self._lib.agg_batch_run(self._b), "agg_batch_run")

    def result(self, i: int) -> N.Result:
        res = N.Result()
        _check(self._lib.agg_batch_result(self._b, i, ctypes.byref(res)), "agg_batch_result")
        return res

    def rows(self, i: int, device: str = "cpu"):
        return _copy_rows(self.result(i), self._spec.n_aggs, device)

    def stats(self) -> dict:
        st = N.BatchStats()
        _check(self._lib.agg_batch_get_stats(self._b, ctypes.byref(st)), "agg_batch_get_stats")
        return st.as_dict()

    def close(self):
        if self._b:
            self._lib.agg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Served mode (agg_server_*): submit requests, the native loop admits them by budget."""

    def __init__(self, pool_bytes: int, max_inflight: int = 6):
        self._lib = load_library()
        cfg = N.ServerConfig()
        cfg.pool_bytes = pool_bytes
        cfg.max_inflight = max_inflight
        self._s = ctypes.c_void_p()
        _check(self._lib.agg_server_create(ctypes.byref(cfg), ctypes.byref(self._s)), "agg_server_create")
        self._na = {}

    def submit(self, spec: N.Spec, ptr: int, n: int) -> int:
        t = ctypes.c_uint64()
        _check(self._lib.agg_server_submit(self._s, ctypes.byref(spec), ctypes.c_void_p(ptr), n, ctypes.byref(t)),
               "agg_server_submit")
        self._na[t.value] = spec.n_aggs
        return t.value

    def wait(self, ticket: int):
        """(result, info dict) once the request finished."""
        res, info = N.Result(), N.RequestInfo()
        rc = self._lib.agg_server_wait(self._s, ticket, ctypes.byref(res), ctypes.byref(info))
        _check(rc, "agg_server_wait")
        d = {"queue_ms": info.queue_ms, "run_ms": info.run_ms, "latency_ms": info.latency_ms,
             "pool_offset": info.pool_offset, "stats": info.stats.as_dict()}
        return res, d

    def rows(self, ticket: int, device: str = "cpu"):
        res, _ = self.wait(ticket)
        return _copy_rows(res, self._na[ticket], device)

    def release(self, ticket: int):
        _check(self._lib.agg_server_release(self._s, ticket), "agg_server_release")
        self._na.pop(ticket, None)

    def stats(self) -> dict:
        st = N.ServerStats()
        _check(self._lib.agg_server_get_stats(self._s, ctypes.byref(st)), "agg_server_get_stats")
        return st.as_dict()

    def close(self):
        if self._s:
            self._lib.agg_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
