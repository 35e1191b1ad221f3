"""Dynamic Destaging (Sec. 4.3.3) on the HBM tables, against the oracle row by row.

Every partition starts resident with a table from a pool of frames (none is
spilled from the estimate); a table that fills gets one twice as large from
the pool, its groups moved there, and the records that found it full are fed
again; while the pool has no room, the largest resident partition is spilled
and its frames recycled.
"""
import numpy as np
import pytest

from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_R24, _pool, _rand_r24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


@pytest.mark.parametrize("scale", [64, 4096])
def test_overestimate_keeps_every_partition_resident(scale):
    """An estimate far above the groups: the groups fit the budget, so nothing spills."""
    wl = workloads.uniform_spill().scaled(1_000_000, 200_000)
    rec = wl.generate()
    print(f"case: destage overestimate x{scale}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=24 * MIB, est_groups=wl.d * scale, engine="tables")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"destage x{scale}")
    assert st["levels"] == 1 and st["partitions_spilled"] == 0 and st["records_spilled"] == 0
    assert st["pool_high_water"] <= 24 * MIB


def test_tables_grow_from_the_pool():
    """Ten batches: level 0 is planned from the first (100k records), the tables fill as
    later batches bring more keys, and they grow from the rest of the pool -- no spill."""
    wl = workloads.uniform_spill().scaled(1_000_000, 200_000)
    rec = wl.generate()
    print("case: destage growth", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=24 * MIB, est_groups=20_000, engine="tables", batches=10)
    check_against_oracle(rec, oracle_spec(wl), k, c, "destage growth")
    assert st["partitions_grown"] > 0 and st["records_refed"] >= 0
    assert st["levels"] == 1 and st["partitions_spilled"] == 0 and st["records_spilled"] == 0


@pytest.mark.parametrize("budget_mib,est_scale", [(6, 1.0), (6, 1 / 64), (3, 16.0)])
def test_budget_below_the_groups(budget_mib, est_scale):
    """More groups than the budget holds: the largest resident partitions are spilled (their
    frames recycled for the tables that grow), and the recursion finishes them."""
    wl = workloads.uniform_spill().scaled(1_000_000, 200_000)
    rec = wl.generate()
    print(f"case: destage budget={budget_mib}MiB est x{est_scale}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget_mib * MIB, est_groups=int(wl.d * est_scale),
                       engine="tables", batches=4)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"destage {budget_mib} {est_scale}")
    assert st["levels"] >= 2 and st["partitions_spilled"] > 0 and st["states_spilled"] > 0
    assert st["pool_high_water"] <= budget_mib * MIB


def test_r24_batches_and_reserved_keys():
    rng = np.random.default_rng(33)
    rec = _rand_r24(rng, 800_000, _pool(rng, 120_000))
    rec["k1"][:30] = 0xFFFFFFFF
    rec["k2"][:30] = 0xFFFFFFFE
    rng.shuffle(rec)
    print("case: destage R24", flush=True)
    k, c, st = run_lib(rec, 24, SPEC_R24["keys"], SPEC_R24["aggs"], budget=4 * MIB, est_groups=30_000,
                       engine="tables", batches=6)
    check_against_oracle(rec, SPEC_R24, k, c, "destage R24")
    assert st["partitions_spilled"] > 0 or st["partitions_grown"] > 0
