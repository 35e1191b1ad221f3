"""GPU parity of the sorted-run path (engine 4): a first batch whose keys are in
non-decreasing order becomes one row per run of equal keys, with no tables.

Every case compares all rows with the CPU oracle: runs of many lengths
(all-unique, one key for the whole batch, runs spanning many 1024-record
tiles), composite keys, the two reserved key values (they sort last and go to
side groups), sizes that are not tile multiples, a second batch (the rows are
then merged into HBM tables), and unsorted input with the path forced (it must
fall back to the hash engines).
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import check_against_oracle, run_lib
from tests.test_oracle import SPEC_R16, SPEC_R24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


def _sorted_r16(seed, n, d, dist=datagen.UNIFORM, s=0.0):
    rec = datagen.r16(seed, n, d, dist, s, -10**6, 10**6)
    return rec[np.argsort(rec["key"], kind="stable")]


@pytest.mark.parametrize("n,d", [(1, 1), (1023, 100), (1024, 1024), (1025, 1), (100_000, 100_000),
                                 (2_000_000, 200_000), (3_000_001, 7), (500_000, 1)])
def test_sorted_runs_exact(n, d):
    rec = _sorted_r16(300 + n % 97, n, d)
    print(f"case: sorted n={n} d={d}", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=d, engine="sorted")
    check_against_oracle(rec, SPEC_R16, k, c, f"sorted {n} {d}")
    assert st["engine"] == 4 and st["levels"] == 1 and st["records_spilled"] == 0


def test_sorted_zipf_long_runs_and_budget():
    """Zipf ranks sorted by key: a few very long runs among short ones; a small budget
    does not matter (no tables)."""
    rec = _sorted_r16(311, 2_500_000, 300_000, datagen.ZIPF, 1.1)
    print("case: sorted zipf", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=16 * MIB, est_groups=300_000)
    check_against_oracle(rec, SPEC_R16, k, c, "sorted zipf")
    assert st["engine"] == 4


def test_sorted_composite_keys():
    wl = workloads.zipf_composite().scaled(1_200_000, 90_000)
    rec = wl.generate()
    key = (rec["k1"].astype(np.uint64) << np.uint64(32)) | rec["k2"].astype(np.uint64)
    rec = rec[np.argsort(key, kind="stable")]
    print("case: sorted R24", flush=True)
    k, c, st = run_lib(rec, **{"record_bytes": 24, "keys": wl.key_fields, "aggs": wl.aggs}, est_groups=wl.d)
    check_against_oracle(rec, SPEC_R24, k, c, "sorted R24")
    assert st["engine"] == 4


def test_sorted_with_reserved_keys():
    rec = _sorted_r16(313, 700_000, 50_000)
    rec = rec.copy()
    rec["key"][-5000:-2000] = np.uint64((1 << 64) - 2)
    rec["key"][-2000:] = np.uint64((1 << 64) - 1)
    print("case: sorted + reserved keys", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=50_000)
    check_against_oracle(rec, SPEC_R16, k, c, "sorted reserved")
    assert st["engine"] == 4


@pytest.mark.parametrize("budget", [0, 8 * MIB])
def test_sorted_then_more_batches(budget):
    """A sorted first batch, then more batches: the rows become states in HBM tables."""
    rec = _sorted_r16(317, 900_000, 120_000)
    print(f"case: sorted + batches budget={budget}", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=budget, est_groups=120_000, batches=4)
    check_against_oracle(rec, SPEC_R16, k, c, "sorted batches")
    assert st["engine"] == 4


def test_unsorted_input_falls_back():
    rec = _sorted_r16(319, 400_000, 40_000).copy()
    rec[[1000, 350_000]] = rec[[350_000, 1000]]  # one swap: the sample may still look sorted
    print("case: unsorted forced", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=40_000, engine="sorted")
    check_against_oracle(rec, SPEC_R16, k, c, "unsorted fallback")
    assert st["engine"] != 4
    rnd = datagen.r16(321, 300_000, 30_000)
    k, c, st = run_lib(rnd, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=4 * MIB, est_groups=30_000)
    check_against_oracle(rnd, SPEC_R16, k, c, "random input")
    assert st["engine"] != 4
