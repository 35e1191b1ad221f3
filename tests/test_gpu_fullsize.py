"""Full-size parity: every row of the large workloads against the oracle.

The 200M-record uniform query under its 1 GiB budget, the 500M-record Zipf
composite-key query under 4 GiB, the 1M-record workload's distribution at 1e9
records (the on-chip engine's bandwidth regime), all 4096 instances of the batched mix in one
persistent launch, and every request of the served trace are compared row by
row (keys and every aggregate, after sorting by key) with the oracle's
parallel sort-then-scan.  The inputs, engines, budgets and launch shapes are
the ones the benchmark times.  Integer results: the tolerance is zero.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from datagen import workloads
from tests.gpu_util import assert_rows_equal
from tests.wl import oracle_spec

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(msg):
    print(msg, flush=True)


def _sorted(k, c):
    keys = k.numpy().view(np.uint64)
    o = np.argsort(keys, kind="stable")
    return keys[o], c.numpy()[:, o]


def _query(wl):
    """Run one workload as the benchmark does (budget as a caller workspace, est_groups = D)."""
    import torch
    import paper_1311_0059_amd as P
    host = wl.generate()
    dev = torch.from_numpy(host.view(np.uint8).reshape(-1)).to("cuda")
    ws = torch.empty(wl.budget, dtype=torch.uint8, device="cuda") if wl.budget else None
    torch.cuda.synchronize()
    spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, budget=wl.budget, est_groups=wl.d, workspace=ws)
    with P.GroupBy(spec) as g:
        g.consume_ptr(dev.data_ptr(), wl.n)
        g.finish()
        k, c = g.rows("cpu")
        st = g.stats()
    del dev, ws
    torch.cuda.empty_cache()
    return host, _sorted(k, c), st


@pytest.mark.parametrize("name", ["uniform_spill", "zipf_composite"])
def test_full_query_rows_equal_oracle(name):
    wl = getattr(workloads, name)()
    _say(f"case: full-size {wl.name} ({wl.n} records, {wl.d} keys, budget {wl.budget})")
    host, (keys, cols), st = _query(wl)
    _say(f"  library: {keys.size} rows, engine {st['engine']}, passes {st['lds_passes']}, levels {st['levels']}")
    want_k, want_c = oracle.groupby_par(host, oracle_spec(wl))
    assert keys.size == wl.d
    assert_rows_equal(keys, cols, want_k, want_c, wl.name)
    assert st["pool_high_water"] <= wl.budget and st["engine"] == 2
    if wl.dist == workloads.ZIPF:
        assert st["lds_hot_keys"] > 0  # the frequent keys were aggregated apart


def test_onchip_1g_records_rows_equal_oracle():
    """The 1M-record workload's distribution at 1e9 records (16 GB, 10k keys): the on-chip
    engine in one pass, every row against the oracle."""
    wl = workloads.uniform_small_1g()
    _say(f"case: full-size {wl.name} ({wl.n} records, {wl.d} keys)")
    host, (keys, cols), st = _query(wl)
    _say(f"  library: {keys.size} rows, engine {st['engine']}, classes {st['onchip_classes']}, "
         f"workers {st['onchip_workers']}, {st['onchip_ms']:.2f} ms")
    want_k, want_c = oracle.groupby_par(host, oracle_spec(wl))
    assert keys.size == wl.d and st["engine"] == 5
    assert_rows_equal(keys, cols, want_k, want_c, wl.name)


def _bank(ws, rb=16):
    """Generate the workloads one after another into one host buffer (256-byte aligned slots)."""
    offs, total = [], 0
    for w in ws:
        offs.append(total)
        total += (w.n * rb + 255) // 256 * 256
    host = np.empty(max(total, 256), dtype=np.uint8)
    for w, o in zip(ws, offs):
        w.generate(out=host[o:o + w.n * rb].view(workloads.R16))
    return host, offs


def _oracle_many(host, offs, ws, spec):
    """The oracle's rows of every workload, computed on the host's cores (one instance per thread)."""
    def one(i):
        w, o = ws[i], offs[i]
        return oracle.groupby(host[o:o + w.n * 16].view(workloads.R16), spec)
    with ThreadPoolExecutor(max_workers=oracle.host_threads()) as ex:
        return list(ex.map(one, range(len(ws))))


def test_batched_all_4096_instances_equal_oracle():
    import torch
    import paper_1311_0059_amd as P
    insts = workloads.batched_mix()
    _say(f"case: batched mix, {len(insts)} instances, {sum(w.n for w in insts)} records")
    host, offs = _bank(insts)
    dev = torch.empty(host.size, dtype=torch.uint8, device="cuda")
    chunk = 1 << 30
    for o in range(0, host.size, chunk):
        dev[o:o + chunk].copy_(torch.from_numpy(host[o:o + chunk]))
    torch.cuda.synchronize()
    spec = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_CS)
    got = []
    with P.Batch(spec, [(dev.data_ptr() + o, w.n, w.d) for w, o in zip(insts, offs)]) as b:
        b.run()
        b.run()  # the rows of a graph replay
        for i in range(len(insts)):
            got.append(_sorted(*b.rows(i, "cpu")))
        st = b.stats()
    del dev
    torch.cuda.empty_cache()
    _say(f"  batch: {st['solo_instances']} whole, {st['partitioned_instances']} partitioned, "
         f"{st['recomputed_instances']} recomputed alone")
    want = _oracle_many(host, offs, insts, oracle_spec(insts[0]))
    for i, ((k, c), (wk, wc)) in enumerate(zip(got, want)):
        assert k.size == insts[i].d, f"instance {i}: {k.size} rows, {insts[i].d} keys"
        assert_rows_equal(k, c, wk, wc, f"instance {i}")


def test_served_trace_every_request_equals_oracle():
    """The benchmark's 120-request served trace (sizes 1e4-5e7, Zipf s in [0, 1.2], budgets
    16 MiB-2 GiB, 64 GiB pool), every request queued at once, the most requests in flight the
    server accepts."""
    import torch
    import paper_1311_0059_amd as P
    reqs = workloads.served_mix(120)
    _say(f"case: served trace, {len(reqs)} requests, {sum(w.n for w in reqs)} records")
    host, offs = _bank(reqs)
    dev = torch.empty(host.size, dtype=torch.uint8, device="cuda")
    chunk = 1 << 30
    for o in range(0, host.size, chunk):
        dev[o:o + chunk].copy_(torch.from_numpy(host[o:o + chunk]))
    torch.cuda.synchronize()
    got = []
    with P.Server(pool_bytes=64 << 30, max_inflight=6) as srv:
        tickets = [srv.submit(P.make_spec(16, [(0, "u64")], w.aggs, budget=w.budget, est_groups=w.d),
                              dev.data_ptr() + o, w.n) for w, o in zip(reqs, offs)]
        for t in tickets:
            got.append(_sorted(*srv.rows(t)))
            srv.release(t)
        sst = srv.stats()
    del dev
    torch.cuda.empty_cache()
    _say(f"  server: peak {sst['peak_running']} running, pool peak {sst['pool_peak']} bytes")
    want = _oracle_many(host, offs, reqs, oracle_spec(reqs[0]))
    for i, ((k, c), (wk, wc)) in enumerate(zip(got, want)):
        assert k.size == reqs[i].d, f"request {i}: {k.size} rows, {reqs[i].d} keys"
        assert_rows_equal(k, c, wk, wc, f"request {i}")
