"""GPU parity: the library (called through its C ABI) against the CPU oracle.

Results must be bit-exact: integer keys and 64-bit aggregates, rows compared
element by element after sorting by key.  Sizes span several tiles, ragged
tails, budgets that force spilling and 2-3 recursion levels, both spill
policies, wrong distinct-count estimates, many batches, and the paper's
special datasets (heavy hitter, sorted, all-unique, single key).
"""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.golden import load_edge_rows
from tests.gpu_util import assert_rows_equal, check_against_oracle, lib_spec_args, run_lib
from tests.test_oracle import SPEC_MIX, SPEC_R16, SPEC_R24, _pool, _rand_mix, _rand_r16, _rand_r24
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu

MIB = 1 << 20


def _lib_args(spec):
    return dict(record_bytes=spec["record_bytes"], keys=spec["keys"], aggs=spec["aggs"])


def test_small_workload_exact():
    """1M records, 10k uniform keys, unlimited budget: every row equal to the oracle's."""
    wl = workloads.uniform_small()
    rec = wl.generate()
    print("case: uniform-1M-10k", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "uniform-1M-10k")
    assert st["levels"] == 1 and st["records_spilled"] == 0


def test_small_workload_without_estimate():
    wl = workloads.uniform_small()
    rec = wl.generate()
    k, c, _ = run_lib(rec, **lib_spec_args(wl))
    check_against_oracle(rec, oracle_spec(wl), k, c, "no-estimate")


@pytest.mark.parametrize("layout", ["R16", "R24", "MIX"])
def test_edge_values_and_keys(layout):
    """Tiny inputs with keys 0, 2^63, 2^64-1 (the value tables use as 'empty') and extreme values."""
    rng = np.random.default_rng(77)
    gen, spec = {"R16": (_rand_r16, SPEC_R16), "R24": (_rand_r24, SPEC_R24), "MIX": (_rand_mix, SPEC_MIX)}[layout]
    for case in range(12):
        n = int(rng.integers(1, 3000))
        rec = gen(rng, n, _pool(rng, int(rng.integers(1, 50))))
        print(f"case: edge {layout} #{case} n={n}", flush=True)
        k, c, _ = run_lib(rec, **_lib_args(spec), est_groups=int(rng.integers(0, 100)))
        check_against_oracle(rec, spec, k, c, f"{layout} case {case}")


def test_golden_edge_rows():
    rec, keys, cols = load_edge_rows()
    k, c, _ = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL)
    assert_rows_equal(k, c, keys, cols, "golden")


def test_empty_input():
    rec = np.empty(0, dtype=datagen.R16)
    k, c, st = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=10)
    assert k.size == 0 and c.shape[1] == 0 and st["groups_out"] == 0


@pytest.mark.parametrize("policy", ["destage", "prepart"])
@pytest.mark.parametrize("budget_mib,est_scale", [(4, 1.0), (2, 1.0), (4, 1 / 16), (4, 16.0), (3, 0.0)])
def test_spill_and_recursion(policy, budget_mib, est_scale):
    """Budgets far below the table size: partitions of the HBM tables spill to host memory and
    are re-aggregated (the table engine is asked for: the LDS engine would read the batch in
    passes instead of spilling)."""
    wl = workloads.uniform_spill().scaled(2_000_000, 400_000)
    rec = wl.generate()
    est = int(wl.d * est_scale)
    print(f"case: spill budget={budget_mib}MiB est={est} policy={policy}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=budget_mib * MIB, est_groups=est, policy=policy,
                       engine="tables")
    check_against_oracle(rec, oracle_spec(wl), k, c, f"spill {budget_mib} {est_scale} {policy}")
    assert st["levels"] >= 2
    assert st["records_spilled"] + st["states_spilled"] > 0
    assert st["pool_high_water"] <= budget_mib * MIB


def test_many_batches_equal_one_batch():
    wl = workloads.uniform_spill().scaled(600_000, 60_000)
    rec = wl.generate()
    a = run_lib(rec, **lib_spec_args(wl), budget=2 * MIB, est_groups=wl.d, batches=1)
    b = run_lib(rec, **lib_spec_args(wl), budget=2 * MIB, est_groups=wl.d, batches=97)
    assert_rows_equal(a[0], a[1], b[0], b[1], "batches")
    check_against_oracle(rec, oracle_spec(wl), a[0], a[1], "batches")


@pytest.mark.parametrize("budget", [0, 2 * MIB])
def test_heavy_hitter(budget):
    wl = workloads.heavy_hitter(500_000, 20_000, budget)
    rec = wl.generate()
    k, c, _ = run_lib(rec, **lib_spec_args(wl), budget=budget, est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "heavy")


def test_sorted_all_unique_single_key():
    rec = datagen.r16(11, 300_000, 30_000, lo=-5, hi=5)
    srt = rec[np.argsort(rec["key"], kind="stable")]
    k, c, _ = run_lib(srt, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=2 * MIB, est_groups=30_000)
    check_against_oracle(srt, SPEC_R16, k, c, "sorted")
    uniq = datagen.r16(12, 200_000, 200_000)
    k, c, _ = run_lib(uniq, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=3 * MIB, est_groups=200_000)
    check_against_oracle(uniq, SPEC_R16, k, c, "all-unique")
    single = datagen.r16(13, 100_000, 1)
    k, c, _ = run_lib(single, 16, [(0, "u64")], workloads.AGGS_R16_ALL, est_groups=1)
    check_against_oracle(single, SPEC_R16, k, c, "single")


def test_composite_zipf_scaled():
    wl = workloads.zipf_composite().scaled(3_000_000, 300_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=8 * MIB, est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "zipf composite")
    assert st["preagg"] == 1, "skewed input should switch the hot-key cache on"


@pytest.mark.parametrize("policy", ["destage", "prepart"])
@pytest.mark.parametrize("s_exp,preagg", [(0.5, "on"), (1.2, "auto"), (0.0, "on"), (1.2, "off")])
def test_zipf_hot_key_cache_with_spill(policy, s_exp, preagg):
    """Hot-key pre-aggregation together with overflow, spill and recursion (the cache forced on
    also for mild and no skew, and off for strong skew, so both kernel paths see every case)."""
    wl = workloads.Workload("zipf-spill", "R16", 1_500_000, 300_000, datagen.ZIPF if s_exp else datagen.UNIFORM,
                            s_exp, -10**6, 10**6, workloads.AGGS_R16_ALL, 3 * MIB, workloads.SEED_BASE + 11)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=wl.budget, est_groups=wl.d // 4, policy=policy,
                       preagg=preagg)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"zipf {s_exp} {policy} {preagg}")
    assert st["preagg"] == (0 if preagg == "off" else 1) and st["levels"] >= 2


def test_uniform_large_keys_space_keeps_cache_off():
    wl = workloads.uniform_spill().scaled(1_000_000, 900_000)
    rec = wl.generate()
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=wl.d)
    check_against_oracle(rec, oracle_spec(wl), k, c, "uniform no cache")
    assert st["preagg"] == 0


def test_sum_wraps():
    rec = np.zeros(1000, dtype=datagen.R16)
    rec["key"] = np.arange(1000) % 3
    rec["v"] = (1 << 62) + np.arange(1000)
    k, c, _ = run_lib(rec, 16, [(0, "u64")], workloads.AGGS_R16_ALL)
    check_against_oracle(rec, SPEC_R16, k, c, "wrap")


@pytest.mark.slow
@pytest.mark.parametrize("factor", [1 / 4096, 16])
def test_full_size_uniform_spill_wrong_estimate(factor):
    """The 200M-record / 20M-key / 1 GiB workload with the distinct-key estimate 4096x too low
    and 16x too high (more groups than the records), every row against the oracle: the LDS
    engine plans enough partitions, and for the high estimate its largest plan (four sweeps)
    with no overflow."""
    wl = workloads.uniform_spill()
    rec = wl.generate()
    print(f"case: full uniform-200M-20M-1GiB, estimate x{factor}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), budget=wl.budget, est_groups=max(1, int(wl.d * factor)))
    want_k, want_c = oracle.groupby_par(rec, oracle_spec(wl))
    assert_rows_equal(k, c, want_k, want_c, f"estimate x{factor}")
    assert st["pool_high_water"] <= wl.budget and st["engine"] == 2 and st["records_spilled"] == 0
    assert st["lds_sweeps"] == (4 if factor > 1 else 1)
