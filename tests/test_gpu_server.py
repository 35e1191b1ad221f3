"""GPU tests of the served mode: memory admission, overlap, and results that are
the same alone and in the mix (bit-exact, so the tolerance is zero)."""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.gpu_util import assert_rows_equal, run_lib
from tests.wl import make_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20
SPEC = make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL)


def _requests(seed, count):
    sizes = datagen.loguniform_ints(seed, 0, count, 1e4, 2e6).astype(np.int64)
    fr = datagen.uniform_f64(seed, 1, count, 0.01, 0.5)
    ss = datagen.uniform_f64(seed, 2, count, 0.0, 1.2)
    budgets = datagen.loguniform_ints(seed, 3, count, 2 * MIB, 96 * MIB).astype(np.int64)
    out = []
    for i in range(count):
        n = int(sizes[i])
        d = int(min(n, max(1, round(fr[i] * n))))
        dist = datagen.ZIPF if ss[i] > 0.05 else datagen.UNIFORM
        out.append((datagen.r16(seed * 100 + i, n, d, dist, float(ss[i]), -10**6, 10**6), d, int(budgets[i])))
    return out


def _sorted_rows(k, c):
    keys = k.numpy().view(np.uint64)
    o = np.argsort(keys, kind="stable")
    return keys[o], c.numpy()[:, o]


def test_served_mix_equals_alone_and_oracle():
    import torch
    import paper_1311_0059_amd as P
    reqs = _requests(61, 40)
    devs = [torch.from_numpy(r.view(np.uint8).copy()).to("cuda") for r, _, _ in reqs]
    torch.cuda.synchronize()
    with P.Server(pool_bytes=512 * MIB, max_inflight=6) as srv:
        tickets = []
        for (r, d, b), dev in zip(reqs, devs):
            spec = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=b, est_groups=d)
            tickets.append(srv.submit(spec, dev.data_ptr(), r.size))
        got = []
        for t in tickets:
            got.append(_sorted_rows(*srv.rows(t)))
            _, info = srv.wait(t)
            assert info["latency_ms"] >= info["run_ms"] >= 0
        st = srv.stats()
        for t in tickets:
            srv.release(t)
    assert st["peak_running"] > 1, "requests should overlap on the device"
    assert st["pool_peak"] <= 512 * MIB
    for i, (r, d, b) in enumerate(reqs):
        if r.size <= 600_000:
            wk, wc = oracle.groupby(r, SPEC)
            assert_rows_equal(got[i][0], got[i][1], wk, wc, f"request {i} vs oracle")
        k, c, _ = run_lib(r, 16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=b, est_groups=d)
        assert_rows_equal(got[i][0], got[i][1], k, c, f"request {i} alone vs mix")


def test_admission_waits_for_memory_and_rejects_oversize():
    import torch
    import paper_1311_0059_amd as P
    r = datagen.r16(7, 300_000, 30_000)
    dev = torch.from_numpy(r.view(np.uint8).copy()).to("cuda")
    torch.cuda.synchronize()
    pool = 64 * MIB
    with P.Server(pool_bytes=pool, max_inflight=4) as srv:
        big = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=pool, est_groups=30_000)
        small = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=8 * MIB, est_groups=30_000)
        ts = [srv.submit(small, dev.data_ptr(), r.size) for _ in range(3)]
        tb = srv.submit(big, dev.data_ptr(), r.size)  # must wait until the small ones are done
        ts += [srv.submit(small, dev.data_ptr(), r.size) for _ in range(3)]
        rows = [_sorted_rows(*srv.rows(t)) for t in ts + [tb]]
        st = srv.stats()
        with pytest.raises(P.AggError):
            srv.submit(P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=pool + MIB), dev.data_ptr(),
                       r.size)
    assert st["pool_peak"] <= pool
    wk, wc = oracle.groupby(r, SPEC)
    for k, c in rows:
        assert_rows_equal(k, c, wk, wc, "admission")


def test_destroy_with_queued_requests():
    """Closing a server with requests still queued frees each of them once (no
    release needed); a new server afterwards gives the oracle's rows."""
    import torch
    import paper_1311_0059_amd as P
    r = datagen.r16(11, 200_000, 20_000)
    dev = torch.from_numpy(r.view(np.uint8).copy()).to("cuda")
    torch.cuda.synchronize()
    spec = P.make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL, budget=16 * MIB, est_groups=20_000)
    for _ in range(3):
        srv = P.Server(pool_bytes=64 * MIB, max_inflight=1)
        for _ in range(30):
            srv.submit(spec, dev.data_ptr(), r.size)
        srv.close()
    with P.Server(pool_bytes=64 * MIB, max_inflight=2) as srv:
        t = srv.submit(spec, dev.data_ptr(), r.size)
        k, c = _sorted_rows(*srv.rows(t))
        srv.release(t)
    wk, wc = oracle.groupby(r, SPEC)
    assert_rows_equal(k, c, wk, wc, "after destroy with queued requests")
