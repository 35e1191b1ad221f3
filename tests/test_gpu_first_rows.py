"""GPU tests of early output (agg_first_rows): the rows level 0 finished in memory
are final, and agg_finish returns them first, unchanged and in the same order.

Each first row is checked against the oracle's row for its key; the whole final
result against the oracle; on a spilling budget (atomic-table and owner-computed
engines) and on engines that spill nothing (every non-reserved row comes first).
"""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.gpu_util import check_against_oracle
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20


def _run(rec, wl, budget, engine, est=None, policy="destage"):
    import torch
    import paper_1311_0059_amd as P
    dev = torch.from_numpy(rec.view(np.uint8).reshape(-1).copy()).to("cuda")
    torch.cuda.synchronize()
    spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, budget=budget,
                       est_groups=wl.d if est is None else est, engine=engine, policy=policy)
    with P.GroupBy(spec) as g:
        g.consume_ptr(dev.data_ptr(), rec.size)
        fk, fc = g.first_rows("cpu")
        fk2, fc2 = g.first_rows("cpu")
        with pytest.raises(P.AggError):
            g.consume_ptr(dev.data_ptr(), rec.size)
        g.finish()
        k, c = g.rows("cpu")
        st = g.stats()
    torch.cuda.synchronize()
    assert np.array_equal(fk.numpy(), fk2.numpy()) and np.array_equal(fc.numpy(), fc2.numpy())
    return fk.numpy().view(np.uint64), fc.numpy(), k.numpy().view(np.uint64), c.numpy(), st


def _check(rec, wl, first_k, first_c, k, c, label):
    n1 = first_k.size
    assert np.array_equal(k[:n1], first_k) and np.array_equal(c[:, :n1], first_c), f"{label}: first rows moved"
    if n1:
        q, found, qcols = oracle.rows_for_keys(rec, oracle_spec(wl), first_k)
        assert np.all(found > 0)
        order = np.argsort(first_k)
        assert np.array_equal(q, first_k[order]) and np.array_equal(qcols, first_c[:, order]), f"{label}: first rows"
    o = np.argsort(k, kind="stable")
    check_against_oracle(rec, oracle_spec(wl), k[o], c[:, o], label)


@pytest.mark.parametrize("engine,policy", [("tables", "destage"), ("tables", "prepart"), ("owner", "destage")])
def test_first_rows_with_spill(engine, policy):
    wl = workloads.uniform_spill().scaled(2_000_000, 600_000)
    rec = wl.generate()
    print(f"case: first rows {engine} {policy}", flush=True)
    fk, fc, k, c, st = _run(rec, wl, 20 * MIB, engine, policy=policy)
    _check(rec, wl, fk, fc, k, c, f"first rows {engine}")
    assert st["levels"] >= 2 and 0 < fk.size < k.size and fk.size == st["resident_groups_l0"]
    assert st["engine"] == (3 if engine == "owner" else 1)


def test_first_rows_with_frequent_keys():
    """Zipf keys on the LDS engine: the frequent keys' rows are final at level 0 too."""
    wl = workloads.Workload("zipf-first", "R16", 1_200_000, 100_000, datagen.ZIPF, 1.2, -10**6, 10**6,
                            workloads.AGGS_R16_ALL, 0, workloads.SEED_BASE + 41)
    rec = wl.generate()
    print("case: first rows with frequent keys", flush=True)
    fk, fc, k, c, st = _run(rec, wl, 0, "auto")
    _check(rec, wl, fk, fc, k, c, "first rows frequent keys")
    assert st["engine"] == 2 and st["lds_hot_keys"] > 0 and fk.size == k.size


@pytest.mark.parametrize("engine", ["lds", "sorted"])
def test_first_rows_without_spill(engine):
    wl = workloads.uniform_spill().scaled(600_000, 50_000)
    rec = wl.generate()
    if engine == "sorted":
        rec = rec[np.argsort(rec["key"], kind="stable")]
    rec = rec.copy()
    rec["key"][::4999] = np.uint64((1 << 64) - 1)  # a reserved key: its row comes only with agg_finish
    if engine == "sorted":
        rec = rec[np.argsort(rec["key"], kind="stable")]
    print(f"case: first rows {engine}", flush=True)
    fk, fc, k, c, st = _run(rec, wl, 0, engine)
    _check(rec, wl, fk, fc, k, c, f"first rows {engine}")
    assert st["levels"] == 1 and fk.size == k.size - 1
