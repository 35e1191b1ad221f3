"""The spill logic's counters against the paper's models (Pre-Partitioning on
the HBM tables).

Input: D keys that each occur exactly c times, in a seeded random order -- the
draws without replacement from a dataset of n records over m keys that Yao's
formula describes (Appendix, input component).  Under Pre-Partitioning
(Sec. 4.3.4) the first K keys that find room stay resident and every record
of any other key is spilled raw, so

  * records spilled at level 0 = R (1 - K / G_t) records (Secs. 5.3.1, 5.3.4:
    C_IO = R + (R - K/G_t R)), exactly, with K the resident groups;
  * the records consumed before the first table is full follow
    I_raw(K, n, m) = n (1 - (1 - K/m)^(m/n)) (Appendix), within 3%.

The input goes in batches of 4000 records: a launch works on its records
concurrently, so "consumed before" is resolved to the batch in which the first
table filled (4000 records, against I_raw values of 110k and 288k records here).
The rows are checked against the oracle as well.
"""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.gpu_util import check_against_oracle, run_lib

pytestmark = pytest.mark.gpu
SPEC = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": workloads.AGGS_R16_CS}
MIB = 1 << 20


def _equal_counts(seed, d, c):
    """d distinct keys scattered over 2^64, each exactly c times, in a seeded random order."""
    rng = np.random.default_rng(seed)
    keys = np.unique(rng.integers(0, 2**63 - 2, size=d + d // 10, dtype=np.int64).astype(np.uint64))[:d]
    assert keys.size == d
    rec = np.empty(d * c, dtype=datagen.R16)
    rec["key"] = rng.permutation(np.repeat(keys, c))
    rec["v"] = rng.integers(-10**6, 10**6, size=rec.size)
    return rec


@pytest.mark.parametrize("d,c,budget_mib", [(400_000, 10, 6), (300_000, 20, 3)])
def test_prepartitioning_spill_counters_follow_the_models(d, c, budget_mib):
    rec = _equal_counts(workloads.SEED_BASE + 51 + c, d, c)
    n = rec.size
    print(f"case: spill stats d={d} c={c} budget={budget_mib}MiB", flush=True)
    k, cols, st = run_lib(rec, 16, SPEC["keys"], SPEC["aggs"], budget=budget_mib * MIB, est_groups=d,
                          engine="tables", policy="prepart", fanout_bits=1, batches=n // 4000)
    check_against_oracle(rec, SPEC, k, cols, "spill stats")
    K = st["resident_groups_l0"]
    assert 0 < K < d and st["levels"] >= 2
    # every record of a key that stayed out was spilled, and only those
    assert st["records_spilled_l0"] == n - c * K == round(n * oracle.spilled_fraction(K, d))
    want = oracle.yao_i_raw(K, n, d)
    got = st["first_full_record"]
    print(f"  K={K} ({K / d:.3f} of the keys), first full at {got} records, I_raw {want:.0f}", flush=True)
    assert abs(got - want) <= 0.03 * want


def test_prepartitioning_slot_filter_false_positives():
    """Sec. 4.3.4: once a table is full, Pre-Partitioning consults a one-byte filter per slot
    before probing it, and a record whose key the filter shows absent spills with no probe.
    The rows match the oracle, and the share of absent keys' records that pass the filter (its
    false positives, the alpha of Sec. 5.3.4) matches 1 - (1 - 1/(8H))^K within 5%, with K the
    resident groups and H the table slots (every partition's table full)."""
    d, c = 400_000, 10
    rec = _equal_counts(workloads.SEED_BASE + 71, d, c)
    print("case: slot filter", flush=True)
    k, cols, st = run_lib(rec, 16, SPEC["keys"], SPEC["aggs"], budget=6 * MIB, est_groups=d, engine="tables",
                          policy="prepart", batches=20)
    check_against_oracle(rec, SPEC, k, cols, "slot filter")
    assert st["partitions_filtered"] >= st["partitions"] and st["filter_rejects"] > 0
    K, H = st["resident_groups_l0"], st["table_slots_l0"]
    got = st["filter_false"] / (st["filter_rejects"] + st["filter_false"])
    want = oracle.slot_filter_false_positive(K, H)
    print(f"  K={K} H={H} filter passes of absent keys {got:.4f}, model {want:.4f}", flush=True)
    assert abs(got - want) <= 0.05 * want
