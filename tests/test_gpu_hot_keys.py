"""GPU parity of the LDS engine with frequent keys taken out of the partitions.

When a sample of the first batch shows a dominant key, the keys seen at least
three times in it are aggregated apart: the count pass folds their records into
per-workgroup LDS accumulators, the scatter skips them, and each becomes one row.
Every case compares all rows with the CPU oracle: Zipf keys (R16 and composite
R24), a heavy hitter, with and without budget passes, the reserved key values,
a forced overflow of the partitions' tables (spill and recursion), and more
batches after the first.
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_R16
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


def _zipf_r16(seed, n, d, s):
    return workloads.Workload("zipf-r16", "R16", n, d, datagen.ZIPF, s, -10**6, 10**6, workloads.AGGS_R16_ALL, 0,
                              seed)


@pytest.mark.parametrize("n,d,s,budget_mib", [(1_500_000, 150_000, 1.2, 0), (2_000_000, 400_000, 1.0, 16),
                                              (600_000, 5_000, 0.8, 0)])
def test_zipf_hot_keys_exact(n, d, s, budget_mib):
    wl = _zipf_r16(workloads.SEED_BASE + 21 + n % 7, n, d, s)
    rec = wl.generate()
    print(f"case: hot keys zipf n={n} d={d} s={s} budget={budget_mib}MiB", flush=True)
    # (5k keys alone would take the on-chip engine: the LDS engine is asked for)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget_mib * MIB, est_groups=d,
                       engine="lds" if d < 30_000 else "auto")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"hot zipf {n} {d} {s}")
    assert st["engine"] == 2 and st["lds_hot_keys"] > 0 and st["records_spilled"] == 0
    if budget_mib:
        assert st["lds_passes"] >= 2 and st["pool_high_water"] <= budget_mib * MIB


def test_zipf_composite_hot_keys_in_passes():
    wl = workloads.zipf_composite().scaled(2_000_000, 200_000)
    rec = wl.generate()
    print("case: hot keys R24 passes", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=24 * MIB, est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "hot R24")
    assert st["engine"] == 2 and st["lds_hot_keys"] > 0 and st["lds_passes"] >= 2


@pytest.mark.parametrize("budget_mib", [0, 8])
def test_heavy_hitter_hot_key(budget_mib):
    wl = workloads.heavy_hitter(1_000_000, 50_000, budget_mib * MIB)
    rec = wl.generate()
    print(f"case: heavy hitter budget={budget_mib}MiB", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget_mib * MIB, est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "heavy hitter")
    assert st["engine"] == 2 and st["lds_hot_keys"] >= 1


def test_hot_keys_with_reserved_values_and_overflow():
    """Frequent keys apart, the reserved key values in their side groups, and too few
    partitions for the other keys (an explicit fan-out): those spill and recurse."""
    rec = _zipf_r16(workloads.SEED_BASE + 29, 2_000_000, 600_000, 1.1).generate().copy()
    rec["key"][::997] = np.uint64((1 << 64) - 1)
    rec["key"][3::1999] = np.uint64((1 << 64) - 2)
    print("case: hot keys + reserved + overflow", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=20_000, engine="lds",
                       fanout_bits=4)
    check_against_oracle(rec, SPEC_R16, k, c, "hot reserved overflow")
    assert st["engine"] == 2 and st["lds_hot_keys"] > 0 and st["levels"] >= 2 and st["records_spilled"] > 0


def test_hot_keys_then_more_batches():
    wl = _zipf_r16(workloads.SEED_BASE + 31, 1_800_000, 200_000, 1.2)
    rec = wl.generate()
    print("case: hot keys + batches", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=16 * MIB, est_groups=wl.d, batches=4)
    check_against_oracle(rec, oracle_spec(wl), k, c, "hot batches")
    assert st["engine"] == 2 and st["lds_hot_keys"] > 0
