"""GPU parity of the batched mode: every instance's rows against the oracle.

The mix spans whole-instance (one workgroup) and partitioned instances, the
autotuner's trial runs, graph replays, empty and one-record instances, and the
fallback that recomputes an instance alone (underestimated groups overflowing
the LDS tables, reserved key values).
"""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.gpu_util import assert_rows_equal, run_lib
from tests.wl import make_spec

pytestmark = pytest.mark.gpu
SPEC = make_spec(16, [(0, "u64")], workloads.AGGS_R16_CS)


def _upload(recs):
    import torch
    offs, total = [], 0
    for r in recs:
        offs.append(total)
        total += (r.size * 16 + 255) // 256 * 256
    host = np.zeros(max(total, 256), dtype=np.uint8)
    for r, o in zip(recs, offs):
        host[o:o + r.size * 16] = r.view(np.uint8)
    dev = torch.from_numpy(host).to("cuda")
    torch.cuda.synchronize()
    return dev, offs


def _run_batch(recs, ests, **kw):
    import torch
    import paper_1311_0059_amd as P
    dev, offs = _upload(recs)
    spec = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_CS, **kw)
    inst = [(dev.data_ptr() + o, r.size, e) for r, o, e in zip(recs, offs, ests)]
    out = []
    with P.Batch(spec, inst) as b:
        b.run()
        for rep in range(2):  # a graph replay must give the same rows
            if rep:
                b.run()
            rows = []
            for i in range(len(recs)):
                k, c = b.rows(i, "cpu")
                keys = k.numpy().view(np.uint64)
                order = np.argsort(keys, kind="stable")
                rows.append((keys[order], c.numpy()[:, order]))
            out.append(rows)
        st = b.stats()
    torch.cuda.synchronize()
    assert all(np.array_equal(a[0], b_[0]) and np.array_equal(a[1], b_[1]) for a, b_ in zip(out[0], out[1]))
    return out[0], st


def _mix(seed, n_inst, lo, hi):
    sizes = datagen.loguniform_ints(seed, 0, n_inst, lo, hi).astype(np.int64)
    fr = datagen.uniform_f64(seed, 1, n_inst, 0.01, 0.5)
    recs, ds = [], []
    for i in range(n_inst):
        n = int(sizes[i])
        d = int(min(n, max(1, round(fr[i] * n))))
        recs.append(datagen.r16(seed * 1000 + i, n, d, lo=-10**6, hi=10**6))
        ds.append(d)
    return recs, ds


def test_batch_mix_exact():
    recs, ds = _mix(41, 160, 1e3, 3e5)
    recs += [np.empty(0, dtype=datagen.R16), datagen.r16(5, 1, 1)]
    ds += [0, 1]
    rows, st = _run_batch(recs, ds)
    for i, r in enumerate(recs):
        wk, wc = oracle.groupby(r, SPEC)
        assert_rows_equal(rows[i][0], rows[i][1], wk, wc, f"instance {i}")
    assert st["solo_instances"] > 0 and st["partitioned_instances"] > 0
    assert st["recomputed_instances"] == 0


def test_batch_fallback_recomputes_overflowing_instances():
    recs, ds = _mix(43, 24, 2e4, 4e5)
    ests = [max(1, d // 200) if i % 3 == 0 else d for i, d in enumerate(ds)]  # some far too low
    # a reserved key value in one instance
    recs[1] = recs[1].copy()
    recs[1]["key"][::7] = np.uint64((1 << 64) - 1)
    rows, st = _run_batch(recs, ests)
    for i, r in enumerate(recs):
        wk, wc = oracle.groupby(r, SPEC)
        assert_rows_equal(rows[i][0], rows[i][1], wk, wc, f"instance {i}")
    assert st["recomputed_instances"] >= 1


def test_batch_equals_instances_alone():
    recs, ds = _mix(47, 12, 5e3, 2e5)
    rows, _ = _run_batch(recs, ds)
    for i, r in enumerate(recs):
        k, c, _ = run_lib(r, 16, [(0, "u64")], workloads.AGGS_R16_CS, est_groups=ds[i])
        assert_rows_equal(rows[i][0], rows[i][1], k, c, f"alone {i}")


def test_batch_large_instances():
    """A few instances at the top of the size range (partitioned into many LDS partitions)."""
    recs = [datagen.r16(900 + i, n, d, lo=-10**6, hi=10**6)
            for i, (n, d) in enumerate([(4_000_000, 2_000_000), (3_000_000, 30_000), (1_000_000, 500_000)])]
    ds = [2_000_000, 30_000, 500_000]
    rows, st = _run_batch(recs, ds)
    for i, r in enumerate(recs):
        wk, wc = oracle.groupby(r, SPEC)
        assert_rows_equal(rows[i][0], rows[i][1], wk, wc, f"large {i}")
    assert st["partitioned_instances"] == 3


def test_autotuner_times_the_four_candidates_the_cost_model_prices_lowest():
    """The cost model prices all 27 candidate layouts; the four cheapest are timed in price
    order and the fastest is kept.  A second batch of the same shape reuses that choice
    untimed, with the same rows."""
    recs, ds = _mix(53, 37, 2e4, 6e5)
    rows, st = _run_batch(recs, ds)
    for i, r in enumerate(recs):
        wk, wc = oracle.groupby(r, SPEC)
        assert_rows_equal(rows[i][0], rows[i][1], wk, wc, f"tuned {i}")
    print(f"  predicted {st['predict_ms']} timed {st['tune_ms']} chose {st['tuned_candidate']}", flush=True)
    assert st["candidates_priced"] == 27
    assert st["predict_ms"] == sorted(st["predict_ms"]) and st["predict_ms"][0] > 0
    assert all(t > 0 for t in st["tune_ms"])
    assert st["tune_ms"][st["tuned_candidate"]] == min(st["tune_ms"])
    cands = set(zip(st["trial_part_records"], st["trial_chunk_records"], st["trial_solo_max"]))
    assert len(cands) == 4
    chosen = (st["trial_part_records"][st["tuned_candidate"]], st["trial_chunk_records"][st["tuned_candidate"]],
              st["trial_solo_max"][st["tuned_candidate"]])
    rows2, st2 = _run_batch(recs, ds)
    assert st2["candidates_priced"] == 0 and st2["tuned_candidate"] == 0 and st2["tune_ms"] == [0.0] * 4
    assert (st2["trial_part_records"][0], st2["trial_chunk_records"][0], st2["trial_solo_max"][0]) == chosen
    for i in range(len(recs)):
        assert np.array_equal(rows[i][0], rows2[i][0]) and np.array_equal(rows[i][1], rows2[i][1])
