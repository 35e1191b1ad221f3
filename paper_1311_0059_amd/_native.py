"""ctypes declarations of the C ABI in include/aggx.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaggx.so")

MAX_AGGS = 8

STATUS = {0: "AGG_OK", -1: "AGG_E_INVALID", -2: "AGG_E_BUDGET", -3: "AGG_E_DEVICE", -4: "AGG_E_STATE",
          -5: "AGG_E_NOMEM", -6: "AGG_E_INTERNAL"}
TYPES = {"u32": 0, "u64": 1, "i32": 2, "i64": 3}
OPS = {"COUNT": 0, "SUM": 1, "MIN": 2, "MAX": 3}
POLICIES = {"destage": 0, "prepart": 1, "hashsort": 2}


class Field(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint32), ("type", ctypes.c_uint32)]


class Fn(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("in_", Field)]


class Spec(ctypes.Structure):
    _fields_ = [
        ("record_bytes", ctypes.c_uint32),
        ("n_keys", ctypes.c_uint32),
        ("keys", Field * 2),
        ("n_aggs", ctypes.c_uint32),
        ("aggs", Fn * MAX_AGGS),
        ("budget_bytes", ctypes.c_uint64),
        ("est_groups", ctypes.c_uint64),
        ("device_workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("fanout_bits", ctypes.c_uint32),
        ("load_pct", ctypes.c_uint32),
        ("policy", ctypes.c_uint32),
        ("preagg", ctypes.c_uint32),
        ("engine", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class Result(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_uint64), ("d_keys", ctypes.c_void_p), ("d_cols", ctypes.c_void_p * MAX_AGGS)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("records_in", ctypes.c_uint64),
        ("groups_out", ctypes.c_uint64),
        ("resident_groups_l0", ctypes.c_uint64),
        ("records_spilled", ctypes.c_uint64),
        ("states_spilled", ctypes.c_uint64),
        ("bytes_spilled_d2h", ctypes.c_uint64),
        ("bytes_reloaded_h2d", ctypes.c_uint64),
        ("levels", ctypes.c_uint32),
        ("partitions", ctypes.c_uint32),
        ("partitions_spilled", ctypes.c_uint32),
        ("guard_trips", ctypes.c_uint32),
        ("preagg", ctypes.c_uint32),
        ("engine", ctypes.c_uint32),
        ("pool_high_water", ctypes.c_uint64),
        ("pool_bytes", ctypes.c_uint64),
        ("update_launches", ctypes.c_uint64),
        ("update_records", ctypes.c_uint64),
        ("update_ms", ctypes.c_double),
        ("update_launches_l0", ctypes.c_uint64),
        ("update_records_l0", ctypes.c_uint64),
        ("update_ms_l0", ctypes.c_double),
        ("flush_launches", ctypes.c_uint64),
        ("flush_ms", ctypes.c_double),
        ("lds_launches", ctypes.c_uint64),
        ("lds_ms", ctypes.c_double),
        ("partition_ms", ctypes.c_double),
        ("sorted_ms", ctypes.c_double),
        ("lds_sweeps", ctypes.c_uint32),
        ("lds_passes", ctypes.c_uint32),
        ("scatter_launches", ctypes.c_uint64),
        ("scatter_ms", ctypes.c_double),
        ("lds_hot_keys", ctypes.c_uint32),
        ("lds_narrow", ctypes.c_uint32),
        ("scatter_records", ctypes.c_uint64),
        ("onchip_classes", ctypes.c_uint32),
        ("onchip_workers", ctypes.c_uint32),
        ("onchip_ms", ctypes.c_double),
        ("onchip_fallbacks", ctypes.c_uint32),
        ("onchip_kernel16", ctypes.c_uint32),
        ("onchip_direct", ctypes.c_uint64),
        ("records_spilled_l0", ctypes.c_uint64),
        ("first_full_record", ctypes.c_uint64),
        ("filter_rejects", ctypes.c_uint64),
        ("filter_false", ctypes.c_uint64),
        ("partitions_filtered", ctypes.c_uint32),
        ("reserved_stats2", ctypes.c_uint32),
        ("table_slots_l0", ctypes.c_uint64),
        ("hashsort_runs", ctypes.c_uint64),
        ("hashsort_windows", ctypes.c_uint64),
        ("hashsort_fallbacks", ctypes.c_uint32),
        ("partitions_grown", ctypes.c_uint32),
        ("records_refed", ctypes.c_uint64),
        ("cost_onchip_ms", ctypes.c_double),
        ("cost_lds_ms", ctypes.c_double),
        ("cost_tables_ms", ctypes.c_double),
        ("cost_spilled_records", ctypes.c_uint64),
        ("cost_levels", ctypes.c_uint32),
        ("onchip_retries", ctypes.c_uint32),
        ("pinned_peak_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("d_records", ctypes.c_void_p), ("n", ctypes.c_uint64), ("est_groups", ctypes.c_uint64)]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("instances", ctypes.c_uint32),
        ("solo_instances", ctypes.c_uint32),
        ("partitioned_instances", ctypes.c_uint32),
        ("recomputed_instances", ctypes.c_uint32),
        ("items", ctypes.c_uint64),
        ("partitions", ctypes.c_uint64),
        ("records", ctypes.c_uint64),
        ("tuned_candidate", ctypes.c_uint32),
        ("blocks", ctypes.c_uint32),
        ("last_run_ms", ctypes.c_double),
        ("tune_ms", ctypes.c_double * 4),
        ("predict_ms", ctypes.c_double * 4),
        ("trial_part_records", ctypes.c_uint64 * 4),
        ("trial_chunk_records", ctypes.c_uint64 * 4),
        ("trial_solo_max", ctypes.c_uint64 * 4),
        ("candidates_priced", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]
    _ARRAYS = ("tune_ms", "predict_ms", "trial_part_records", "trial_chunk_records", "trial_solo_max")

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in self._ARRAYS}
        for k in self._ARRAYS:
            d[k] = list(getattr(self, k))
        return d


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("reserved", ctypes.c_uint32), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("pool_offset", ctypes.c_uint64),
                ("stats", Stats)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint32), ("running", ctypes.c_uint32), ("peak_running", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("pool_bytes", ctypes.c_uint64), ("pool_in_use", ctypes.c_uint64),
                ("pool_peak", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# every symbol include/aggx.h declares
EXPORTS = ["agg_create", "agg_consume", "agg_first_rows", "agg_finish", "agg_get_stats", "agg_destroy", "agg_strerror",
           "agg_min_budget", "agg_batch_create", "agg_batch_run", "agg_batch_result", "agg_batch_get_stats",
           "agg_batch_destroy", "agg_server_create", "agg_server_submit", "agg_server_wait",
           "agg_server_release", "agg_server_get_stats", "agg_server_destroy", "agg_query_noalloc"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libaggx.so; raises if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1311_0059_amd.build` (needs hipcc)")
    lib = ctypes.CDLL(path)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.agg_create.argtypes = [ctypes.POINTER(Spec), ctypes.POINTER(vp)]
    lib.agg_create.restype = ctypes.c_int
    lib.agg_consume.argtypes = [vp, vp, u64]
    lib.agg_consume.restype = ctypes.c_int
    lib.agg_finish.argtypes = [vp, ctypes.POINTER(Result)]
    lib.agg_finish.restype = ctypes.c_int
    lib.agg_first_rows.argtypes = [vp, ctypes.POINTER(Result)]
    lib.agg_first_rows.restype = ctypes.c_int
    lib.agg_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.agg_get_stats.restype = ctypes.c_int
    lib.agg_destroy.argtypes = [vp]
    lib.agg_destroy.restype = None
    lib.agg_strerror.argtypes = [ctypes.c_int]
    lib.agg_strerror.restype = ctypes.c_char_p
    lib.agg_min_budget.argtypes = [ctypes.POINTER(Spec)]
    lib.agg_min_budget.restype = u64
    lib.agg_batch_create.argtypes = [ctypes.POINTER(Spec), ctypes.POINTER(Instance), ctypes.c_uint32,
                                     ctypes.POINTER(vp)]
    lib.agg_batch_create.restype = ctypes.c_int
    lib.agg_batch_run.argtypes = [vp]
    lib.agg_batch_run.restype = ctypes.c_int
    lib.agg_batch_result.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(Result)]
    lib.agg_batch_result.restype = ctypes.c_int
    lib.agg_batch_get_stats.argtypes = [vp, ctypes.POINTER(BatchStats)]
    lib.agg_batch_get_stats.restype = ctypes.c_int
    lib.agg_batch_destroy.argtypes = [vp]
    lib.agg_batch_destroy.restype = None
    lib.agg_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.agg_server_create.restype = ctypes.c_int
    lib.agg_server_submit.argtypes = [vp, ctypes.POINTER(Spec), vp, u64, ctypes.POINTER(u64)]
    lib.agg_server_submit.restype = ctypes.c_int
    lib.agg_server_wait.argtypes = [vp, u64, ctypes.POINTER(Result), ctypes.POINTER(RequestInfo)]
    lib.agg_server_wait.restype = ctypes.c_int
    lib.agg_server_release.argtypes = [vp, u64]
    lib.agg_server_release.restype = ctypes.c_int
    lib.agg_query_noalloc.argtypes = [ctypes.POINTER(Spec), vp, u64, vp, ctypes.POINTER(vp), u64, ctypes.POINTER(u64)]
    lib.agg_query_noalloc.restype = ctypes.c_int
    lib.agg_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.agg_server_get_stats.restype = ctypes.c_int
    lib.agg_server_destroy.argtypes = [vp]
    lib.agg_server_destroy.restype = None
    _lib = lib
    return lib
