"""Hash-Sort (Sec. 4.2) on the GPU, as the policy and as the fallback of Sec. 4.3
(Phase 2), against the oracle row by row.

As the policy, one table takes the whole budget; each time it is full its
groups are written as a run in hash order and it is emptied; the runs are then
merged range by range.  The paper's heavy-hitter set (one key with most of the
records, every other key once) is where it collapses most; a uniform set with
far more keys than the table holds makes many runs and ranges.

As the fallback, a sub-run of a level's grace split that kept more than 80% of
the run it was split from (a frequent key spilled whole) goes to Hash-Sort.
"""
import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_R24, _pool, _rand_r24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20
SPEC_R16 = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": workloads.AGGS_R16_ALL}


@pytest.mark.parametrize("n,d,budget_mib", [(2_000_000, 400_000, 4), (3_000_000, 30_000, 1)])
def test_policy_heavy_hitter(n, d, budget_mib):
    """Heavy hitter: the frequent key collapses into one group of every run."""
    wl = workloads.heavy_hitter(n, d, budget_mib * MIB)
    rec = wl.generate()
    print(f"case: hashsort heavy n={n} d={d} budget={budget_mib}MiB", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=wl.budget, est_groups=d, policy="hashsort")
    check_against_oracle(rec, oracle_spec(wl), k, c, "hashsort heavy")
    assert st["hashsort_runs"] >= 2  # more groups than one table holds
    assert st["engine"] == 1 and st["pool_high_water"] <= wl.budget
    assert st["levels"] == (2 if st["hashsort_runs"] else 1)


def test_policy_many_runs_and_ranges():
    """400k distinct uniform keys through a 1 MiB budget: tens of runs, a range merge over all of them."""
    wl = workloads.uniform_spill().scaled(1_200_000, 400_000)
    rec = wl.generate()
    print("case: hashsort uniform many runs", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=1 * MIB, est_groups=wl.d, policy="hashsort", batches=3)
    check_against_oracle(rec, oracle_spec(wl), k, c, "hashsort many runs")
    assert st["hashsort_runs"] >= 20 and st["hashsort_windows"] >= 20 and st["hashsort_fallbacks"] == 0


def test_policy_fits_in_one_table():
    wl = workloads.uniform_small().scaled(300_000, 5_000)
    rec = wl.generate()
    print("case: hashsort fits", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=8 * MIB, est_groups=wl.d, policy="hashsort")
    check_against_oracle(rec, oracle_spec(wl), k, c, "hashsort fits")
    assert st["hashsort_runs"] == 0 and st["levels"] == 1


def test_policy_r24_reserved_keys_batches():
    """Two-field keys, MIN/MAX of int32 at their extremes, the two reserved key values, five batches."""
    rng = np.random.default_rng(21)
    rec = _rand_r24(rng, 600_000, _pool(rng, 150_000))
    # a few records whose canonical key is one of the reserved values
    rec["k1"][:50] = 0xFFFFFFFF
    rec["k2"][:50] = 0xFFFFFFFF
    rec["k1"][50:90] = 0xFFFFFFFF
    rec["k2"][50:90] = 0xFFFFFFFE
    rng.shuffle(rec)
    print("case: hashsort R24", flush=True)
    k, c, st = run_lib(rec, 24, SPEC_R24["keys"], SPEC_R24["aggs"], budget=2 * MIB, est_groups=150_000,
                       policy="hashsort", batches=5)
    check_against_oracle(rec, SPEC_R24, k, c, "hashsort R24")
    assert st["hashsort_runs"] >= 2


def test_fallback_when_a_split_does_not_divide_the_run():
    """Pre-Partitioning fills its tables with the keys of the first part of the input; a
    frequent key that only arrives afterwards is spilled whole, with a few hundred thousand
    other keys.  The next level's grace split cannot divide that key's records (over 80% of
    its input), so that sub-run goes to Hash-Sort, whose table collapses the key at once."""
    rng = np.random.default_rng(workloads.SEED_BASE + 61)
    pool = np.unique(rng.integers(0, 2**63 - 2, size=450_000, dtype=np.int64).astype(np.uint64))
    first, late, heavy = pool[:300_000], pool[300_000:400_000], pool[400_000]
    part1 = rng.permutation(np.repeat(first, 2))
    part2 = rng.permutation(np.concatenate([np.full(5_000_000, heavy, dtype=np.uint64), np.repeat(late, 2)]))
    rec = np.empty(part1.size + part2.size, dtype=datagen.R16)
    rec["key"] = np.concatenate([part1, part2])
    rec["v"] = rng.integers(-10**6, 10**6, size=rec.size)
    spec = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": workloads.AGGS_R16_ALL}
    print("case: hashsort fallback after a split", flush=True)
    k, c, st = run_lib(rec, 16, spec["keys"], spec["aggs"], budget=4 * MIB, est_groups=400_001, policy="prepart",
                       engine="tables")
    check_against_oracle(rec, spec, k, c, "hashsort fallback")
    assert st["records_spilled_l0"] > 5_000_000
    assert st["hashsort_fallbacks"] >= 1 and st["levels"] >= 2


def test_first_rows_under_hashsort():
    """Under the policy every row is final once the runs are merged: first_rows returns them all."""
    import torch
    import paper_1311_0059_amd as P

    wl = workloads.heavy_hitter(1_000_000, 200_000, 2 * MIB)
    rec = wl.generate()
    raw = torch.from_numpy(rec.view(np.uint8).reshape(-1).copy()).cuda()
    torch.cuda.synchronize()
    print("case: hashsort first rows", flush=True)
    spec = P.make_spec(wl.record_bytes, list(wl.key_fields), list(wl.aggs), budget=wl.budget, est_groups=wl.d,
                       policy="hashsort")
    with P.GroupBy(spec) as g:
        g.consume_ptr(raw.data_ptr(), rec.size)
        fk, fc = g.first_rows("cpu")
        g.finish()
        k, c = g.rows("cpu")
    torch.cuda.synchronize()
    # the reserved keys' side rows come last, at finish; none here
    assert fk.shape[0] == k.shape[0]
    keys = k.numpy().view(np.uint64)
    order = np.argsort(keys)
    check_against_oracle(rec, oracle_spec(wl), keys[order], c.numpy()[:, order], "hashsort first rows")
