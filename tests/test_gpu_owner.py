"""GPU parity of the owner-computed table engine (engine 3).

Sub-chunks are radix-partitioned into a buffer inside the budget and one
workgroup owns each partition's HBM table.  Every case compares all rows with
the CPU oracle: fitting and spilling budgets, an underestimated group count
(tables overflow; both spill policies), several batches, skewed keys forced
onto the engine, the edge-case record layouts (reserved key values included),
and agreement with the atomic-table engine.
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import assert_rows_equal, check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_MIX, SPEC_R16, SPEC_R24, _pool, _rand_mix, _rand_r16, _rand_r24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


@pytest.mark.parametrize("n,d,budget", [(1_000_000, 10_000, 0), (2_000_000, 400_000, 24 * MIB),
                                        (777_777, 123_457, 64 * MIB), (513, 500, 0), (70_000, 1, 0)])
def test_owner_engine_exact(n, d, budget):
    wl = workloads.uniform_spill().scaled(n, d)
    rec = wl.generate()
    print(f"case: owner n={n} d={d} budget={budget}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget, est_groups=wl.d, engine="owner")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"owner {n} {d} {budget}")
    assert st["engine"] == 3


@pytest.mark.parametrize("layout", ["R16", "R24", "MIX"])
def test_owner_engine_edge_layouts(layout):
    rng = np.random.default_rng(123)
    gen, spec = {"R16": (_rand_r16, SPEC_R16), "R24": (_rand_r24, SPEC_R24), "MIX": (_rand_mix, SPEC_MIX)}[layout]
    for case in range(8):
        n = int(rng.integers(1, 5000))
        rec = gen(rng, n, _pool(rng, int(rng.integers(1, 60))))
        print(f"case: owner {layout} {case} n={n}", flush=True)
        k, c, st = run_lib(rec, record_bytes=spec["record_bytes"], keys=spec["keys"], aggs=spec["aggs"],
                           est_groups=int(rng.integers(1, 100)), engine="owner")
        check_against_oracle(rec, spec, k, c, f"owner {layout} {case}")
        assert st["engine"] == 3


@pytest.mark.parametrize("policy", ["destage", "prepart"])
def test_owner_overflow_spills_and_recurses(policy):
    """An estimate far below the true group count: tables fill mid-batch; Dynamic
    Destaging spills the full partitions' states, Pre-Partitioning keeps them."""
    wl = workloads.uniform_spill().scaled(3_000_000, 1_200_000)
    rec = wl.generate()
    print(f"case: owner overflow {policy}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=40 * MIB, est_groups=wl.d // 8, engine="owner",
                       policy=policy)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"owner overflow {policy}")
    assert st["engine"] == 3 and st["levels"] >= 2 and st["records_spilled"] > 0
    if policy == "destage":
        assert st["states_spilled"] > 0


def test_owner_many_batches():
    wl = workloads.uniform_spill().scaled(2_500_000, 300_000)
    rec = wl.generate()
    print("case: owner 5 batches", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=64 * MIB, est_groups=wl.d, batches=5, engine="owner")
    check_against_oracle(rec, oracle_spec(wl), k, c, "owner batches")
    assert st["engine"] == 3


def test_owner_skewed_keys_forced():
    wl = workloads.zipf_composite().scaled(1_500_000, 150_000)
    rec = wl.generate()
    print("case: owner zipf R24", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=64 * MIB, est_groups=wl.d, engine="owner")
    check_against_oracle(rec, oracle_spec(wl), k, c, "owner zipf")
    assert st["engine"] == 3


def test_owner_reserved_keys_in_spilled_partitions():
    """Records with the two reserved key values land in partitions that are spilled
    from the start; they still end in their side groups."""
    rec = datagen.r16(5150, 2_000_000, 600_000, lo=-10**6, hi=10**6).copy()
    rec["key"][::501] = np.uint64((1 << 64) - 1)
    rec["key"][7::1003] = np.uint64((1 << 64) - 2)
    print("case: owner reserved keys + planned spill", flush=True)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=20 * MIB, est_groups=600_000,
                       engine="owner")
    check_against_oracle(rec, SPEC_R16, k, c, "owner reserved keys")
    assert st["engine"] == 3 and st["partitions_spilled"] > 0


def test_owner_agrees_with_tables():
    """A large uniform batch that the budget cannot hold partitioned whole: the owner
    engine's rows equal the atomic-table engine's and the oracle's."""
    wl = workloads.uniform_spill().scaled(5_000_000, 1_000_000)
    rec = wl.generate()
    print("case: owner vs tables", flush=True)
    a = run_lib(rec, **lib_spec_args(wl), budget=48 * MIB, est_groups=wl.d, engine="owner")
    b = run_lib(rec, **lib_spec_args(wl), budget=48 * MIB, est_groups=wl.d, engine="tables")
    assert a[2]["engine"] == 3 and b[2]["engine"] == 1
    assert_rows_equal(a[0], a[1], b[0], b[1], "owner vs tables")
    check_against_oracle(rec, oracle_spec(wl), a[0], a[1], "owner 5M")
