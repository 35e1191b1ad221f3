"""GPU parity of the on-chip engine (one pass, key classes aggregated in LDS,
folded into the level-0 HBM tables), against the oracle row by row.

Cases: the 1M-record / 10k-key workload in its default configuration, narrow
and wide LDS columns, two-field keys, the reserved key values, one key only,
keys that all fall in one class (the class's LDS table overflows into the HBM
tables), an estimate too low for the tables (the batch runs again on another
engine), later batches on the same tables, a budget, and tiny inputs.
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_R24, _pool, _rand_r24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
SPEC_R16 = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": workloads.AGGS_R16_ALL}


def _r16(keys, vals):
    rec = np.zeros(len(keys), dtype=datagen.R16)
    rec["key"] = np.asarray(keys, dtype=np.uint64)
    rec["v"] = np.asarray(vals, dtype=np.int64)
    return rec


def test_uniform_1m_10k_and_automatic_choice():
    """The 1M-record / 10k-key workload on the on-chip engine; AUTO takes this engine where the
    cost model prices it below the partition-first engine (40M records over 2k keys), not at
    100 records per group."""
    wl = workloads.uniform_small()
    rec = wl.generate()
    print("case: onchip uniform-1M-10k", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, "onchip 1M/10k")
    assert st["engine"] == 5 and st["onchip_fallbacks"] == 0 and st["onchip_classes"] >= 2
    assert st["records_spilled"] == 0 and st["levels"] == 1
    _, _, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    assert st["engine"] == 2
    wl = workloads.uniform_small().scaled(40_000_000, 2_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "auto onchip")
    assert st["engine"] == 5 and st["cost_onchip_ms"] < st["cost_lds_ms"]


@pytest.mark.parametrize("n,d", [(1, 1), (100, 7), (5000, 5000), (300_000, 2500), (3_000_000, 3000),
                                 (400_000, 25_000), (2_500_000, 27_000)])
def test_sizes(n, d):
    """From one record to enough records for eight or more workers per class (XCD-aware roles),
    and up to eight classes (a wave's own class then a small share of what it reads)."""
    wl = workloads.uniform_small().scaled(n, d)
    rec = wl.generate()
    print(f"case: onchip n={n} d={d}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=d, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"onchip n={n}")
    assert st["engine"] == 5


def test_r24_narrow_and_extremes():
    """Two-field keys, MIN/MAX of int32 fields at their extremes in 4-byte LDS columns."""
    rng = np.random.default_rng(11)
    # 12k groups: narrow columns save classes (six of 8-byte columns at two thirds load, four of narrow ones)
    rec = _rand_r24(rng, 300_000, _pool(rng, 11_900))
    print("case: onchip R24", flush=True)
    k, c, st = run_lib(rec, 24, SPEC_R24["keys"], SPEC_R24["aggs"], est_groups=12_000, engine="onchip")
    check_against_oracle(rec, SPEC_R24, k, c, "onchip R24")
    assert st["engine"] == 5 and st["lds_narrow"] == 1 and st["onchip_classes"] == 4


def test_reserved_keys_and_one_key():
    rng = np.random.default_rng(5)
    keys = rng.choice(np.array([0, 1, 2**63, 2**64 - 1, 2**64 - 2, 12345], dtype=np.uint64), size=50_000)
    vals = rng.integers(-2**63, 2**63 - 1, size=keys.size, dtype=np.int64)
    rec = _r16(keys, vals)
    print("case: onchip reserved keys", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=6, engine="onchip")
    check_against_oracle(rec, SPEC_R16, k, c, "onchip reserved")
    assert st["engine"] == 5
    one = _r16(np.full(70_000, 77, dtype=np.uint64), rng.integers(-10**9, 10**9, size=70_000))
    # (one key is also sorted input: the on-chip engine is asked for)
    k, c, st = run_lib(one, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=1, engine="onchip")
    check_against_oracle(one, SPEC_R16, k, c, "onchip one key")
    assert st["engine"] == 5


def test_one_class_overflows_into_tables():
    """Keys x * 2^32 + x share their class (the class hash folds the two halves), so one
    class's LDS table overflows: the staged kernel leaves the batch to the general kernel,
    where the class's extra keys go straight to the HBM tables."""
    rng = np.random.default_rng(9)
    x = rng.choice(2**31, size=9000, replace=False).astype(np.uint64)
    pool = (x << np.uint64(32)) | x
    keys = pool[rng.integers(0, pool.size, size=400_000)]
    rec = _r16(keys, rng.integers(-10**6, 10**6, size=keys.size))
    print("case: onchip one class", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=9000, engine="onchip")
    check_against_oracle(rec, SPEC_R16, k, c, "onchip one class")
    assert st["engine"] == 5 and st["onchip_classes"] > 1 and st["onchip_fallbacks"] == 0
    assert st["onchip_retries"] == 1 and st["onchip_kernel16"] == 0 and st["onchip_direct"] > 0


def test_low_estimate_runs_the_batch_again():
    """50k keys with an estimate of 2k: the tables planned for the estimate overflow, the
    on-chip result is dropped and the batch runs on another engine."""
    wl = workloads.uniform_small().scaled(1_000_000, 50_000)
    rec = wl.generate()
    print("case: onchip low estimate", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=2000, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, "onchip low estimate")
    assert st["onchip_fallbacks"] == 1 and st["engine"] != 5


def test_later_batches_and_budget():
    """Three batches (the first on-chip, the others into the same HBM tables), under a budget."""
    wl = workloads.uniform_small().scaled(600_000, 8000)
    rec = wl.generate()
    print("case: onchip three batches", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), batches=3, est_groups=wl.d, budget=4 << 20, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, "onchip batches")
    assert st["engine"] == 5 and st["pool_high_water"] <= 4 << 20


R16_SWAPPED = np.dtype([("v", "<i8"), ("key", "<u8")])


@pytest.mark.parametrize("d,aggs", [(1500, workloads.AGGS_R16_ALL), (9000, workloads.AGGS_R16_ALL),
                                    (8000, workloads.AGGS_R16_CS)])
def test_kernel16_one_class_and_staged(d, aggs):
    """16-byte (key, value) records whose groups fit one LDS table take the one-class kernel
    (every lane folds every record it loads); with more groups, the staged kernel (a ring of
    whole records per wave).  COUNT+SUM and all four aggregates."""
    wl = workloads.uniform_small().scaled(2_000_000, d)
    rec = wl.generate()
    spec = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": aggs}
    print(f"case: onchip kernel16 d={d} na={len(aggs)}", flush=True)
    k, c, st = run_lib(rec, 16, spec["keys"], aggs, est_groups=d, engine="onchip")
    check_against_oracle(rec, spec, k, c, f"kernel16 d={d}")
    assert st["engine"] == 5 and st["onchip_fallbacks"] == 0 and st["onchip_retries"] == 0
    assert st["onchip_kernel16"] == (1 if d == 1500 else 2) and (st["onchip_classes"] == 1) == (d == 1500)


def test_kernel16_key_in_second_half_signed_extremes():
    """The key in the record's second 8 bytes, signed int64 values at both extremes (MIN/MAX
    kept as unsigned maxima of a transformed value), and the two reserved key values."""
    rng = np.random.default_rng(23)
    pool = rng.integers(0, 2**63, size=2000, dtype=np.int64).astype(np.uint64)
    pool[:2] = [2**64 - 1, 2**64 - 2]
    rec = np.zeros(600_000, dtype=R16_SWAPPED)
    rec["key"] = pool[rng.integers(0, pool.size, size=rec.size)]
    rec["v"] = rng.integers(-2**63, 2**63 - 1, size=rec.size, dtype=np.int64)
    rec["v"][:20] = -2**63
    rec["v"][20:40] = 2**63 - 1
    aggs = [("COUNT", 0, "i64"), ("SUM", 0, "i64"), ("MIN", 0, "i64"), ("MAX", 0, "i64")]
    spec = {"record_bytes": 16, "keys": [(8, "u64")], "aggs": aggs}
    print("case: onchip kernel16 key second", flush=True)
    k, c, st = run_lib(rec, 16, spec["keys"], aggs, est_groups=2000, engine="onchip")
    check_against_oracle(rec, spec, k, c, "kernel16 key second")
    assert st["engine"] == 5 and st["onchip_kernel16"] == 1


def test_unaligned_input_takes_the_general_kernel():
    """Records that start 8 bytes past a 16-byte boundary: the general kernel, the same rows."""
    import torch
    import paper_1311_0059_amd as P
    wl = workloads.uniform_small().scaled(500_000, 5000)
    rec = wl.generate()
    raw = np.zeros(rec.size * 16 + 8, dtype=np.uint8)
    raw[8:] = rec.view(np.uint8).reshape(-1)
    dev = torch.from_numpy(raw).cuda()
    torch.cuda.synchronize()
    print("case: onchip unaligned", flush=True)
    spec = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=wl.d, engine="onchip")
    with P.GroupBy(spec) as g:
        g.consume_ptr(dev.data_ptr() + 8, rec.size)
        g.finish()
        k, c = g.rows("cpu")
        st = g.stats()
    torch.cuda.synchronize()
    keys = k.numpy().view(np.uint64)
    order = np.argsort(keys)
    check_against_oracle(rec, oracle_spec(wl), keys[order], c.numpy()[:, order], "onchip unaligned")
    assert st["engine"] == 5 and st["onchip_kernel16"] == 0


def test_kernel16_other_field_takes_the_general_kernel():
    """An aggregate of a 32-bit field does not fit the 16-byte record kernel's form."""
    rng = np.random.default_rng(29)
    rec = _r16(rng.integers(0, 500, size=300_000).astype(np.uint64), rng.integers(-10**6, 10**6, size=300_000))
    aggs = [("COUNT", 0, "i64"), ("MIN", 8, "i32"), ("MAX", 12, "i32")]
    spec = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": aggs}
    print("case: onchip kernel16 not applicable", flush=True)
    k, c, st = run_lib(rec, 16, spec["keys"], aggs, est_groups=500, engine="onchip")
    check_against_oracle(rec, spec, k, c, "onchip i32 fields")
    assert st["engine"] == 5 and st["onchip_kernel16"] == 0


def test_staged_reserved_keys_go_to_the_general_kernel():
    """A reserved key value among several classes: the staged kernel leaves the batch to the
    general kernel (side groups), with the same rows as the oracle."""
    wl = workloads.uniform_small().scaled(1_500_000, 9000)
    rec = wl.generate()
    rec["key"][::1001] = np.uint64(2**64 - 1)
    rec["key"][5::1003] = np.uint64(2**64 - 2)
    print("case: onchip staged reserved", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=9002, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, "staged reserved")
    assert st["engine"] == 5 and st["onchip_retries"] == 1 and st["onchip_kernel16"] == 0


@pytest.mark.parametrize("n,d", [(4097, 3000), (1_000_003, 6000), (3_000_001, 17_000)])
def test_staged_sizes_and_ragged_tails(n, d):
    """The staged kernel over ragged last tiles (a ring's carry across tiles, the last partial
    wave) and up to eight classes."""
    wl = workloads.uniform_small().scaled(n, d)
    rec = wl.generate()
    print(f"case: onchip staged n={n} d={d}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=d, engine="onchip")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"staged n={n}")
    assert st["engine"] == 5 and st["onchip_kernel16"] == 2 and st["onchip_retries"] == 0
