"""GPU parity of the LDS engine's sweeps and passes.

Sweeps: a partition with more groups than one LDS table is aggregated in 2-4
sweeps over its records, each sweep taking the keys of one value of the hash
bits below the partition digit.  Passes: when the budget holds only part of
the partitioned batch, runs of consecutive partitions are partitioned and
aggregated one after the other, each run in one pass over the batch.

Every case compares all rows with the CPU oracle: sweeps forced by a small
explicit fan-out (R16 and composite R24 keys), the two reserved key values
(folded by the first sweep only, and in exactly one pass), overflow of a
table (spill and recursion, with sweeps and with passes), more batches after
a swept or passed first batch, passes and sweeps together, and the automatic
choice of 2^13 partitions for a batch whose groups need more than 2^12.
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


@pytest.mark.parametrize("n,d,bits,sweeps,parts", [(1_500_000, 150_000, 4, 4, 16), (1_000_000, 60_000, 4, 2, 16),
                                                   (777_777, 40_000, 2, 4, 4), (3000, 2999, 0, 1, 2)])
def test_sweeps_exact(n, d, bits, sweeps, parts):
    wl = workloads.uniform_spill().scaled(n, d)
    rec = wl.generate()
    print(f"case: sweeps n={n} d={d} bits={bits}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=d, engine="lds", fanout_bits=bits)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"sweeps {n} {d}")
    assert st["engine"] == 2 and st["levels"] == 1 and st["records_spilled"] == 0
    assert st["lds_sweeps"] == sweeps and st["partitions"] == parts


def test_sweeps_composite_keys():
    wl = workloads.zipf_composite().scaled(1_200_000, 100_000)
    rec = wl.generate()
    print("case: sweeps R24", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="lds", fanout_bits=4)
    check_against_oracle(rec, oracle_spec(wl), k, c, "sweeps R24")
    assert st["engine"] == 2 and st["lds_sweeps"] > 1


def test_sweeps_reserved_keys_counted_once():
    rec = datagen.r16(401, 900_000, 70_000, lo=-10**6, hi=10**6).copy()
    rec["key"][::777] = np.uint64((1 << 64) - 1)
    rec["key"][5::1009] = np.uint64((1 << 64) - 2)
    print("case: sweeps + reserved keys", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=70_000, engine="lds",
                       fanout_bits=3)
    check_against_oracle(rec, SPEC_R16, k, c, "sweeps reserved keys")
    assert st["engine"] == 2 and st["lds_sweeps"] == 4


def test_sweep_overflow_spills_and_recurses():
    """An estimate far below the true count: each sweep's table fills, new keys spill
    raw and are aggregated at the next level."""
    wl = workloads.uniform_spill().scaled(2_000_000, 400_000)
    rec = wl.generate()
    print("case: sweeps overflow", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=120_000, engine="lds", fanout_bits=4)
    check_against_oracle(rec, oracle_spec(wl), k, c, "sweeps overflow")
    assert st["engine"] == 2 and st["lds_sweeps"] == 4 and st["levels"] >= 2 and st["records_spilled"] > 0


def test_sweeps_then_more_batches():
    wl = workloads.uniform_spill().scaled(1_600_000, 120_000)
    rec = wl.generate()
    print("case: sweeps + batches", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="lds", fanout_bits=4, batches=3)
    check_against_oracle(rec, oracle_spec(wl), k, c, "sweeps batches")
    assert st["engine"] == 2 and st["lds_sweeps"] == 4


def test_automatic_fanout_beyond_table_engine_limit():
    """12M groups need more than 2^12 one-table partitions: the automatic choice keeps the
    LDS engine with 2^13 partitions, one sweep each (unlimited budget, no hot key)."""
    wl = workloads.uniform_spill().scaled(24_000_000, 12_000_000)
    rec = wl.generate()
    print("case: automatic 24M/12M", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=0, est_groups=wl.d)
    assert st["engine"] == 2 and st["lds_sweeps"] == 1 and st["partitions"] == 8192
    check_against_oracle(rec, oracle_spec(wl), k, c, "automatic 2^13 partitions")


@pytest.mark.parametrize("n,d,budget_mib", [(3_000_000, 300_000, 16), (2_000_000, 50_000, 9), (1_500_000, 1, 8)])
def test_passes_exact(n, d, budget_mib):
    wl = workloads.uniform_spill().scaled(n, d)
    rec = wl.generate()
    print(f"case: passes n={n} d={d} budget={budget_mib}MiB", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget_mib * MIB, est_groups=d)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"passes {n} {d}")
    if d > 1:
        assert st["engine"] == 2 and st["lds_passes"] >= 2 and st["levels"] == 1 and st["records_spilled"] == 0
    assert st["pool_high_water"] <= budget_mib * MIB


def test_passes_composite_keys_and_reserved_values():
    wl = workloads.zipf_composite().scaled(1_500_000, 120_000)
    rec = wl.generate().copy()
    print("case: passes R24", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=12 * MIB, est_groups=wl.d, engine="lds")
    check_against_oracle(rec, oracle_spec(wl), k, c, "passes R24")
    assert st["engine"] == 2 and st["lds_passes"] >= 2
    r16 = datagen.r16(409, 2_000_000, 100_000, lo=-10**6, hi=10**6).copy()
    r16["key"][::333] = np.uint64((1 << 64) - 1)
    r16["key"][1::777] = np.uint64((1 << 64) - 2)
    print("case: passes + reserved keys", flush=True)
    k, c, st = run_lib(r16, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=12 * MIB, est_groups=100_000)
    check_against_oracle(r16, SPEC_R16, k, c, "passes reserved keys")
    assert st["engine"] == 2 and st["lds_passes"] >= 2


@pytest.mark.parametrize("policy", ["destage", "prepart"])
def test_passes_with_overflow_spill_and_recursion(policy):
    """Too few partitions for the groups (a low estimate with an explicit fan-out): the LDS
    tables of every pass fill, new keys spill raw and are aggregated at the next level inside
    the same budget."""
    wl = workloads.uniform_spill().scaled(2_500_000, 1_200_000)
    rec = wl.generate()
    print(f"case: passes overflow {policy}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=16 * MIB, est_groups=60_000, engine="lds", policy=policy,
                       fanout_bits=6)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"passes overflow {policy}")
    assert st["engine"] == 2 and st["lds_passes"] >= 2 and st["levels"] >= 2 and st["records_spilled"] > 0
    assert st["pool_high_water"] <= 16 * MIB


def test_passes_with_sweeps_then_more_batches():
    wl = workloads.uniform_spill().scaled(2_400_000, 200_000)
    rec = wl.generate()
    print("case: passes + sweeps + batches", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=10 * MIB, est_groups=wl.d, engine="lds", fanout_bits=5,
                       batches=3)
    check_against_oracle(rec, oracle_spec(wl), k, c, "passes sweeps batches")
    assert st["engine"] == 2 and st["lds_passes"] >= 2 and st["lds_sweeps"] >= 2


def test_block_counts_beyond_16_bits():
    """The count kernel stores each workgroup's partition counts in 16 bits; a workgroup
    whose count of a partition is larger counts its chunk again in the scatter.  Sorted
    keys, 2000 records each, over two partitions: about a third of the 256 workgroups
    (125k records each) hold more than 65535 records of one partition, the others fewer."""
    wl = workloads.Workload("sorted-blocks", "R16", 32_000_000, 16_000, datagen.UNIFORM, 0.0, -10**6, 10**6,
                            workloads.AGGS_R16_ALL, 0, workloads.SEED_BASE + 43)
    rec = wl.generate()
    rec = rec[np.argsort(rec["key"], kind="stable")]
    print("case: 16-bit block counts", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="lds", fanout_bits=1)
    check_against_oracle(rec, oracle_spec(wl), k, c, "16-bit block counts")
    assert st["engine"] == 2 and st["partitions"] == 2 and st["levels"] == 1
