"""GPU parity of the partition-first LDS engine and of the engine choice.

Every case compares all rows with the CPU oracle.  The LDS engine is forced on
for the edge-case layouts, driven into LDS-table overflow (spill + recursion)
by an underestimated group count, continued with more batches (its rows are
then merged into HBM tables), and refused when the budget cannot hold the
partitioned batch.
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import assert_rows_equal, check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_MIX, SPEC_R16, SPEC_R24, _pool, _rand_mix, _rand_r16, _rand_r24
from tests.wl import make_spec, oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


def _lib_args(spec):
    return dict(record_bytes=spec["record_bytes"], keys=spec["keys"], aggs=spec["aggs"])


@pytest.mark.parametrize("n,d", [(1_000_000, 10_000), (777_777, 123_457), (513, 500), (70_000, 1)])
def test_lds_engine_exact(n, d):
    wl = workloads.uniform_small().scaled(n, d)
    rec = wl.generate()
    print(f"case: lds n={n} d={d}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="lds")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"lds {n} {d}")
    assert st["engine"] == 2 and st["levels"] == 1


@pytest.mark.parametrize("layout", ["R16", "R24", "MIX"])
def test_lds_engine_edge_layouts(layout):
    rng = np.random.default_rng(99)
    gen, spec = {"R16": (_rand_r16, SPEC_R16), "R24": (_rand_r24, SPEC_R24), "MIX": (_rand_mix, SPEC_MIX)}[layout]
    for case in range(8):
        n = int(rng.integers(1, 5000))
        rec = gen(rng, n, _pool(rng, int(rng.integers(1, 60))))
        k, c, st = run_lib(rec, **_lib_args(spec), est_groups=int(rng.integers(1, 100)), engine="lds")
        check_against_oracle(rec, spec, k, c, f"lds {layout} {case}")
        assert st["engine"] == 2


@pytest.mark.parametrize("layout", ["R24", "MIX"])
def test_lds_narrow_columns(layout):
    """COUNT and MIN/MAX of 32-bit fields in 4-byte table columns, with the fields'
    extreme values: a plan where the narrow columns save a sweep."""
    rng = np.random.default_rng(7)
    # two partitions; each one's expected groups fit a table of narrow slots but not of 8-byte ones
    gen, spec, est = {"R24": (_rand_r24, SPEC_R24, 6400), "MIX": (_rand_mix, SPEC_MIX, 4800)}[layout]
    rec = gen(rng, 40_000, _pool(rng, est - 100))
    print(f"case: lds narrow {layout}", flush=True)
    k, c, st = run_lib(rec, **_lib_args(spec), est_groups=est, engine="lds", fanout_bits=1)
    check_against_oracle(rec, spec, k, c, f"lds narrow {layout}")
    assert st["engine"] == 2 and st["lds_narrow"] == 1 and st["lds_sweeps"] == 1


@pytest.mark.parametrize("engine", ["lds", "tables"])
@pytest.mark.parametrize("rb,keys,voff,vtype", [
    (12, [(0, "u32"), (4, "u32")], 8, "i32"),   # 12-byte records: the key's fields are read one by one
    (16, [(4, "u32"), (0, "u32")], 8, "i64"),   # fields in the other order: one by one
    (16, [(8, "u32"), (12, "u32")], 0, "i64"),  # adjacent at an 8-byte offset: one 8-byte load
])
def test_composite_key_layouts(rb, keys, voff, vtype, engine):
    """Two-field keys in several record layouts, against the oracle."""
    rng = np.random.default_rng(rb + 31 * keys[0][0])
    n = 60_000
    dt = np.dtype({"names": ["ka", "kb", "v"], "formats": ["<u4", "<u4", "<i4" if vtype == "i32" else "<i8"],
                   "offsets": [keys[0][0], keys[1][0], voff], "itemsize": rb})
    pool = rng.integers(0, 1 << 32, size=(4000, 2), dtype=np.uint64)
    pool[:3] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0xFFFFFFFF, 0xFFFFFFFE]]  # incl. the reserved key values
    pick = pool[rng.integers(0, len(pool), size=n)]
    rec = np.zeros(n, dtype=dt)
    rec["ka"], rec["kb"] = pick[:, 0].astype(np.uint32), pick[:, 1].astype(np.uint32)
    rec["v"] = rng.integers(-(1 << 31), (1 << 31) - 1, size=n)
    aggs = [("COUNT", 0, "i64"), ("SUM", voff, vtype), ("MIN", voff, vtype), ("MAX", voff, vtype)]
    spec = make_spec(rb, keys, aggs)
    print(f"case: composite key rb={rb} keys={keys} {engine}", flush=True)
    k, c, st = run_lib(rec, rb, keys, aggs, est_groups=4000, engine=engine)
    check_against_oracle(rec, spec, k, c, f"composite key {rb} {keys} {engine}")
    assert st["engine"] == (2 if engine == "lds" else 1)


@pytest.mark.parametrize("bits", [2, 6])
def test_lds_overflow_spills_and_recurses(bits):
    """Too few partitions for the groups (an explicit fan-out, so that the low estimate is
    taken as given): LDS tables fill, new keys spill raw and are re-aggregated at the
    next level."""
    wl = workloads.uniform_spill().scaled(1_500_000, 1_200_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d // 400, engine="lds", fanout_bits=bits)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"lds overflow {bits}")
    assert st["engine"] == 2 and st["levels"] >= 2 and st["records_spilled"] > 0


def test_lds_low_estimate_plans_enough_partitions():
    """Without an explicit fan-out, an estimate 400x too low still gets enough partitions:
    nothing spills."""
    wl = workloads.uniform_spill().scaled(1_500_000, 1_200_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d // 400)
    check_against_oracle(rec, oracle_spec(wl), k, c, "lds low estimate")
    assert st["engine"] == 2 and st["levels"] == 1 and st["records_spilled"] == 0


@pytest.mark.parametrize("budget", [0, 64 * MIB])
def test_lds_then_more_batches(budget):
    """Rows of the first (LDS) batch become states in HBM tables when more batches come."""
    wl = workloads.uniform_spill().scaled(900_000, 90_000)
    rec = wl.generate()
    a = run_lib(rec, **lib_spec_args(wl), budget=budget, est_groups=wl.d, batches=5, engine="lds")
    check_against_oracle(rec, oracle_spec(wl), a[0], a[1], "lds + batches")
    assert a[2]["engine"] == 2


def test_lds_passes_or_refused_by_budget():
    """A budget that holds part of the partitioned batch: the LDS engine reads the batch in
    passes; one that would need more than eight passes: the HBM tables take the batch."""
    wl = workloads.uniform_spill().scaled(1_000_000, 100_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=8 * MIB, est_groups=wl.d, engine="lds")
    check_against_oracle(rec, oracle_spec(wl), k, c, "lds passes")
    assert st["engine"] == 2 and st["lds_passes"] >= 2 and st["pool_high_water"] <= 8 * MIB
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=2 * MIB, est_groups=wl.d, engine="lds")
    check_against_oracle(rec, oracle_spec(wl), k, c, "lds refused")
    assert st["engine"] == 1


def test_automatic_engine_choice():
    """Uniform keys with an ample budget take the partition-first LDS engine (10k keys at 100
    records each, 300k keys), with a heavy hitter's key aggregated apart from the partitions."""
    wl = workloads.uniform_small()
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "auto uniform")
    assert st["engine"] == 2
    wl = workloads.uniform_small().scaled(1_000_000, 300_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "auto uniform 300k")
    assert st["engine"] == 2, "uniform keys with an ample budget should take the LDS engine"
    hh = workloads.heavy_hitter(400_000, 100_000)
    rec = hh.generate()
    k, c, st = run_lib(rec, **lib_spec_args(hh), est_groups=hh.d)
    check_against_oracle(rec, oracle_spec(hh), k, c, "auto heavy hitter")
    assert st["engine"] == 2 and st["lds_hot_keys"] >= 1, "a heavy hitter should be aggregated apart from the partitions"


def test_engines_agree():
    wl = workloads.uniform_spill().scaled(500_000, 60_000)
    rec = wl.generate()
    a = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="lds")
    b = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d, engine="tables")
    assert a[2]["engine"] == 2 and b[2]["engine"] == 1
    assert_rows_equal(a[0], a[1], b[0], b[1], "lds vs tables")
