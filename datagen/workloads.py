"""Workload recipes: the synthetic inputs that stand in for the paper's datasets.

The paper measures on a synthetic UserVisits table (string key, double revenue,
1e9 records) and on skewed variants (uniform, Zipf, heavy hitter, sorted) from
its skew study.  Those files are not available; these recipes keep the
structure that matters to the method (record count, exact number of distinct
keys, key-frequency distribution, memory budget) with integer keys and int64
aggregates.  Each recipe is a plain description; the generator in
`datagen/__init__.py` turns it into bytes.

Seeds are 0x1311005900000000 + workload number, with a sub-index per instance or
request for the batched and served mixes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import HEAVY, UNIFORM, ZIPF, R16, R24, r16, r24, loguniform_ints, uniform_f64

SEED_BASE = 0x1311005900000000
GIB = 1 << 30
MIB = 1 << 20

# record layouts: name -> (record bytes, key fields [(offset, type)], numpy dtype)
# types: "u32", "u64", "i32", "i64"
LAYOUTS = {
    "R16": (16, [(0, "u64")], R16),
    "R24": (24, [(0, "u32"), (4, "u32")], R24),
}

# aggregate sets: list of (op, field offset, field type); COUNT ignores the field
AGGS_R16_ALL = [("COUNT", 0, "i64"), ("SUM", 8, "i64"), ("MIN", 8, "i64"), ("MAX", 8, "i64")]
AGGS_R16_CS = [("COUNT", 0, "i64"), ("SUM", 8, "i64")]
AGGS_R24 = [("SUM", 8, "i64"), ("MIN", 16, "i32"), ("MAX", 20, "i32"), ("COUNT", 0, "i64")]


@dataclass
class Workload:
    name: str
    layout: str
    n: int
    d: int
    dist: int
    s: float
    lo: int
    hi: int
    aggs: list
    budget: int          # device working-memory budget in bytes; 0 = unlimited
    seed: int
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def record_bytes(self) -> int:
        return LAYOUTS[self.layout][0]

    @property
    def key_fields(self):
        return LAYOUTS[self.layout][1]

    def generate(self, out: np.ndarray | None = None) -> np.ndarray:
        if self.layout == "R16":
            return r16(self.seed, self.n, self.d, self.dist, self.s, self.lo, self.hi, out=out)
        return r24(self.seed, self.n, self.d, self.dist, self.s, self.lo, self.hi, out=out)

    def scaled(self, n: int, d: int | None = None, budget: int | None = None, name: str | None = None) -> "Workload":
        """Same distribution at another size (keeps the records-per-key ratio unless d is given)."""
        if d is None:
            d = max(1, int(round(self.d * n / self.n)))
        return Workload(name or f"{self.name}@{n}", self.layout, n, min(d, max(n, 1)), self.dist, self.s, self.lo,
                        self.hi, self.aggs, self.budget if budget is None else budget, self.seed, self.note)


def uniform_small() -> Workload:
    """1M R16 records, 10,000 uniform keys, v in [0, 1000), COUNT+SUM+MIN+MAX, unlimited budget."""
    return Workload("uniform-1M-10k", "R16", 1_000_000, 10_000, UNIFORM, 0.0, 0, 999, AGGS_R16_ALL, 0,
                    SEED_BASE + 1)


def uniform_small_1g() -> Workload:
    """The 1M-record workload's distribution at 1e9 records (16 GB): 10,000 uniform keys,
    v in [0, 1000), COUNT+SUM+MIN+MAX, unlimited budget -- its bandwidth regime."""
    return Workload("uniform-1G-10k", "R16", 1_000_000_000, 10_000, UNIFORM, 0.0, 0, 999, AGGS_R16_ALL, 0,
                    SEED_BASE + 1)


def uniform_spill() -> Workload:
    """200M R16 records, 20M uniform keys, v in [-1e6, 1e6], all four aggregates, 1 GiB budget."""
    return Workload("uniform-200M-20M-1GiB", "R16", 200_000_000, 20_000_000, UNIFORM, 0.0, -1_000_000, 1_000_000,
                    AGGS_R16_ALL, 1 * GIB, SEED_BASE + 2)


def uniform_inmem() -> Workload:
    """The same 200M records as uniform_spill (same seed), with an unlimited budget: nothing spills."""
    return Workload("uniform-200M-20M-unlimited", "R16", 200_000_000, 20_000_000, UNIFORM, 0.0, -1_000_000,
                    1_000_000, AGGS_R16_ALL, 0, SEED_BASE + 2)


def zipf_composite() -> Workload:
    """500M R24 records, 50M composite keys Zipf s=1.0, SUM(v1) MIN(v2) MAX(v3) COUNT, 4 GiB budget."""
    return Workload("zipf1-500M-50M-4GiB", "R24", 500_000_000, 50_000_000, ZIPF, 1.0, -1_000_000_000,
                    1_000_000_000, AGGS_R24, 4 * GIB, SEED_BASE + 3)


def heavy_hitter(n: int, d: int, budget: int = 0) -> Workload:
    """One key carries n-(d-1) records, every other key exactly one (the paper's heavy-hitter set)."""
    return Workload(f"heavy-{n}-{d}", "R16", n, d, HEAVY, 0.0, -1_000_000, 1_000_000, AGGS_R16_ALL, budget,
                    SEED_BASE + 7)


# --- batched instance mix: 4096 instances, sizes log-uniform 1k..4M, distinct 1%..50% ---
def batched_mix(n_inst: int = 4096, lo: float = 1e3, hi: float = 4e6):
    seed = SEED_BASE + 4
    sizes = loguniform_ints(seed, 0, n_inst, lo, hi).astype(np.int64)
    frac = uniform_f64(seed, 1, n_inst, 0.01, 0.50)
    d = np.maximum(1, np.rint(frac * sizes)).astype(np.int64)
    d = np.minimum(d, sizes)
    return [Workload(f"inst{i}", "R16", int(sizes[i]), int(d[i]), UNIFORM, 0.0, -1_000_000, 1_000_000, AGGS_R16_CS,
                     0, SEED_BASE + 0x40000000 + i) for i in range(n_inst)]


# --- served request mix: Poisson arrivals, sizes log-uniform 1e4..5e7, Zipf s in [0, 1.2] ---
def served_mix(n_req: int = 1000, lo: float = 1e4, hi: float = 5e7, budget_lo: int = 16 * MIB,
               budget_hi: int = 2 * GIB):
    seed = SEED_BASE + 5
    sizes = loguniform_ints(seed, 0, n_req, lo, hi).astype(np.int64)
    frac = uniform_f64(seed, 1, n_req, 0.01, 0.50)
    svals = uniform_f64(seed, 2, n_req, 0.0, 1.2)
    budgets = loguniform_ints(seed, 3, n_req, float(budget_lo), float(budget_hi)).astype(np.int64)
    gaps = -np.log1p(-uniform_f64(seed, 4, n_req, 0.0, 1.0))  # unit-mean exponential inter-arrival gaps
    out = []
    for i in range(n_req):
        n = int(sizes[i])
        d = int(min(n, max(1, round(frac[i] * n))))
        s = float(svals[i])
        out.append(Workload(f"req{i}", "R16", n, d, ZIPF if s > 0 else UNIFORM, s, -1_000_000, 1_000_000,
                            AGGS_R16_ALL, int(budgets[i]), SEED_BASE + 0x50000000 + i,
                            extra={"gap": float(gaps[i])}))
    return out
