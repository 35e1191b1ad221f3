"""The cost model that picks the engine of an AUTO first batch (each engine priced
by a fixed part and a part per byte of its passes, at rates measured on this
GPU; the HBM tables also by the paper's I/O term for what they spill).

Checked: AUTO takes the engine the model prices lowest; the predicted times of
the partition-first and on-chip engines are within a factor of two of their
measured query times; the predicted level-0 spill of the HBM tables follows
R - (K/G) R (Secs. 5.3.1, 5.3.4) as measured; and the rows stay the oracle's.
"""
import time

import numpy as np
import pytest

import datagen
from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args, run_lib
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


@pytest.mark.parametrize("n,d,want", [(1_000_000, 10_000, 2), (3_000_000, 5_000, 2), (10_000_000, 10_000, 2),
                                      (40_000_000, 2_000, 5)])
def test_auto_takes_the_engine_priced_lowest(n, d, want):
    wl = workloads.uniform_small().scaled(n, d)
    rec = wl.generate()
    print(f"case: cost model n={n} d={d}", flush=True)
    k, c, st = run_lib(rec, **lib_spec_args(wl), est_groups=d)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"cost {n} {d}")
    assert st["engine"] == want
    priced = {2: st["cost_lds_ms"], 5: st["cost_onchip_ms"]}
    assert priced[want] == min(v for v in priced.values() if v > 0)


def _query_ms(raw, wl, engine, reps=4):
    import torch
    import paper_1311_0059_amd as P

    spec = P.make_spec(wl.record_bytes, list(wl.key_fields), list(wl.aggs), est_groups=wl.d, engine=engine)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with P.GroupBy(spec) as g:
            g.consume_ptr(raw.data_ptr(), wl.n)
            g.finish()
            st = g.stats()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return 1e3 * float(np.median(ts[1:] if len(ts) > 1 else ts)), st


@pytest.mark.parametrize("n,d", [(10_000_000, 10_000), (40_000_000, 2_000)])
def test_predicted_times_track_measured(n, d):
    import torch

    wl = workloads.uniform_small().scaled(n, d)
    rec = wl.generate()
    raw = torch.from_numpy(rec.view(np.uint8).reshape(-1).copy()).cuda()
    print(f"case: cost model timing n={n} d={d}", flush=True)
    _, st = _query_ms(raw, wl, "auto", reps=1)
    for engine, key in (("lds", "cost_lds_ms"), ("onchip", "cost_onchip_ms")):
        ms, st_e = _query_ms(raw, wl, engine)
        pred = st[key]
        print(f"  {engine}: measured {ms:.3f} ms, predicted {pred:.3f} ms", flush=True)
        assert pred > 0 and 0.5 * ms <= pred <= 2.0 * ms


def test_spill_prediction_follows_the_io_model():
    """HBM tables under Pre-Partitioning with a budget below the groups: the predicted level-0
    spill R - (K/G) R is within 10% of the input of the measured one."""
    rng = np.random.default_rng(workloads.SEED_BASE + 91)
    d, c = 400_000, 10
    keys = np.unique(rng.integers(0, 2**63 - 2, size=d + d // 10, dtype=np.int64).astype(np.uint64))[:d]
    rec = np.empty(d * c, dtype=datagen.R16)
    rec["key"] = rng.permutation(np.repeat(keys, c))
    rec["v"] = rng.integers(-10**6, 10**6, size=rec.size)
    spec = {"record_bytes": 16, "keys": [(0, "u64")], "aggs": workloads.AGGS_R16_CS}
    print("case: cost model spill", flush=True)
    k, cols, st = run_lib(rec, 16, spec["keys"], spec["aggs"], budget=6 * MIB, est_groups=d, engine="tables",
                          policy="prepart")
    check_against_oracle(rec, spec, k, cols, "cost spill")
    pred, got = st["cost_spilled_records"], st["records_spilled_l0"]
    print(f"  spilled {got}, predicted {pred}, levels {st['levels']} (predicted {st['cost_levels']})", flush=True)
    assert abs(pred - got) <= 0.1 * rec.size and st["cost_levels"] >= 2 and st["levels"] >= 2
