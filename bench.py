#!/usr/bin/env python3
"""Benchmark of the bounded-memory hash GROUP BY on one MI355X.

A step is one whole query through the C ABI over one batch that is already
resident in HBM: agg_create (on a preallocated workspace of the budget's size)
+ agg_consume + agg_finish (every recursion level, result rows in HBM) +
agg_destroy.

Default workload: 500M R24 records {u32 k1, u32 k2, i64 v1, i32 v2, i32 v3},
50M distinct composite keys drawn Zipf s=1.0, SUM(v1) MIN(v2) MAX(v3) COUNT,
4 GiB device budget -- the largest single query.  Beside it, under "extra",
the 200M-record R16 query with 20M uniform keys and a 1 GiB budget (too small
for the partitioned batch: the library reads the batch in passes of
partitions).

Prints one JSON line.  `roofline` describes the kernel that took the most
device time, timed with HIP events recorded by the library on the stream it
launches on; its algorithmic bytes are the query's algorithmic bytes per record
(input read once + result rows written once, divided by the records) times the
records its launches processed.  `step_frac` is the whole step's algorithmic
bytes over its wall time, against the same peak.  `cpu_baseline` is the
oracle's parallel sort-then-scan over the whole input on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "input records/s + % HBM peak (bit-exact); served p50/p99 latency vs plain path"

DEFAULT_WORKLOAD = "zipf-composite"  # 500M R24 records, 50M Zipf keys, 4 GiB: the largest single query
EXTRA_WORKLOAD = "uniform-spill"     # 200M R16 records, 20M uniform keys, 1 GiB

WORKLOADS = {
    "uniform-spill": "uniform_spill",
    "uniform-small": "uniform_small",
    "uniform-1g": "uniform_small_1g",
    "uniform-inmem": "uniform_inmem",
    "zipf-composite": "zipf_composite",
    "batched": "batched_mix",
    "served": "served_mix",
    "g-sweep": "uniform_spill",
    "uniform-sorted": "uniform_spill",
    "first-rows": "uniform_spill",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help=f"with the default workload, skip the {EXTRA_WORKLOAD} query reported under 'extra'")
    ap.add_argument("--policy", default="destage", choices=["destage", "prepart"])
    ap.add_argument("--engine", default="auto", choices=["auto", "tables", "lds", "owner", "sorted", "onchip"],
                    help="engine for the first batch (auto = the library's choice)")
    ap.add_argument("--cpu-runs", type=int, default=3,
                    help="runs of the CPU oracle over the whole input (median reported; 0 = skip)")
    ap.add_argument("--requests", type=int, default=120, help="served: requests in the trace")
    ap.add_argument("--load", type=float, default=0.8, help="served: offered load vs the plain path's capacity")
    ap.add_argument("--loads", default="", help="served: comma-separated offered loads to sweep (the first is reported "
                                                  "at the top level; default: --load alone)")
    ap.add_argument("--inflight", type=int, default=6, help="served: requests running at once (the library accepts at most 6)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy kernel (counter calibration for the traffic figure)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding the aggregation over several GPUs is not built", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    if args.calibrate_copy:
        return calibrate_copy(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "g-sweep":
        return bench_g_sweep(args)
    if args.workload == "first-rows":
        return bench_first_rows(args)
    if args.workload == "served":
        return bench_served(args)
    out = bench_query(args, args.workload, with_cpu=rank == 0 and args.cpu_runs > 0)
    if args.extra and args.workload == DEFAULT_WORKLOAD:
        # the 200M-record / 1 GiB query beside the headline one, on the same GPU
        extra = bench_query(args, EXTRA_WORKLOAD, with_cpu=False)
        out["extra"] = {k: extra[k] for k in ("value", "unit", "ms_per_step", "config", "gbps_algorithmic",
                                              "pct_hbm_peak", "rows_ok", "per_step", "roofline")}
    if rank == 0:
        print(json.dumps(out), flush=True)


def dominant_kernel(agg, steps, n, alg_per_record):
    """The kernel that took the most device time in the steps, its launches, HIP-event time and
    algorithmic bytes: the per-record algorithmic bytes of the query times the records the
    launches processed (records they partitioned, aggregated or routed)."""
    engine = agg["engine"] // steps
    if engine == 5:  # on-chip engine: one pass reads every record once
        return "k_onchip", steps, agg["onchip_ms"], n * steps * alg_per_record
    if engine == 4:  # sorted runs: the check/count pass and the run reduction read every record
        return "k_run_heads+k_run_reduce", steps, agg["sorted_ms"], n * steps * alg_per_record
    if agg["update_launches_l0"]:
        kname = "k_owner_update" if engine == 3 else f"k_update<0, {1 if agg['preagg'] else 0}>"
        return kname, agg["update_launches_l0"], agg["update_ms_l0"], agg["update_records_l0"] * alg_per_record
    # the partition-first LDS engine: each scatter launch reads the batch and writes one run of
    # partitions; each aggregation launch reads that run back.  Both are charged the records of
    # the run (every non-frequent record once per step), not the rest of the batch they skip.
    recs = agg["scatter_records"]
    if agg["scatter_ms"] > agg["lds_ms"]:
        return "k_part_scatter", agg["scatter_launches"], agg["scatter_ms"], recs * alg_per_record
    return "k_lds_agg", agg["lds_launches"], agg["lds_ms"], recs * alg_per_record


def cpu_oracle_baseline(args, host, wl):
    """The oracle (parallel sort-then-scan) on the whole input on this host's cores: median of
    `--cpu-runs` runs, generation excluded."""
    import oracle
    from tests.wl import oracle_spec  # the oracle's own spec format
    threads = oracle.host_threads()
    times = []
    for i in range(args.cpu_runs):
        tc = time.perf_counter()
        k, _ = oracle.groupby_par(host, oracle_spec(wl), threads=threads)
        times.append(time.perf_counter() - tc)
        log(args, f"[bench] CPU oracle run {i}: {times[-1]:.2f}s on {threads} threads, {k.size} rows")
        del k
    dt = sorted(times)[len(times) // 2]
    return {"value": round(wl.n / dt, 1), "unit": "records/s", "cores": threads, "kind": "oracle",
            "cpu_model": oracle.cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"whole input ({wl.n} records), median of {len(times)} runs "
                      f"({', '.join(f'{t:.2f}' for t in times)} s); parallel sort-then-scan on {threads} threads"}


def bench_query(args, workload, with_cpu):
    """One query workload: a step is agg_create + agg_consume + agg_finish + agg_destroy over
    the whole batch, resident in HBM before the timed region."""
    import numpy as np
    import torch

    import datagen
    import paper_1311_0059_amd as P
    from datagen import workloads

    wl = getattr(workloads, WORKLOADS[workload])()
    log(args, f"[bench] generating {wl.name}: {wl.n} records x {wl.record_bytes} B, {wl.d} keys")
    t = time.perf_counter()
    host = wl.generate()
    raw = host.view(np.uint8).reshape(-1)
    log(args, f"[bench] generated in {time.perf_counter() - t:.1f}s, checksum {datagen.checksum(raw[: 1 << 24])}")
    dev = torch.empty(raw.size, dtype=torch.uint8, device="cuda")
    dev.copy_(torch.from_numpy(raw))
    if workload == "uniform-sorted":
        # the same records in non-decreasing key order (the paper's sorted dataset), sorted on the
        # device before timing; int64 order of key ^ 2^63 is the unsigned order of the key
        assert wl.record_bytes == 16
        words = dev.view(torch.int64).view(-1, 2)
        flip = torch.tensor(-(1 << 63), dtype=torch.int64, device="cuda")
        keys, vals = words[:, 0].contiguous(), words[:, 1].contiguous()
        perm = torch.argsort(keys ^ flip)
        # gather the two 1-D columns and interleave them (a row gather of the whole
        # 3.2 GB two-column tensor returned wrong rows on this torch build)
        sk, sv = keys[perm], vals[perm]
        out = torch.stack([sk, sv], dim=1).contiguous()
        ok = bool(((out[1:, 0] ^ flip) >= (out[:-1, 0] ^ flip)).all().item())
        ok &= int(out[:, 0].sum().item()) == int(keys.sum().item()) and int(out[:, 1].sum().item()) == int(vals.sum().item())
        if not ok:
            sys.exit("bench.py: building the sorted input on the device failed its checks")
        dev = out.view(torch.uint8).view(-1)
        del words, keys, vals, perm, sk, sv
        host = dev.cpu().numpy().view(workloads.R16) if with_cpu else host
        wl = workloads.Workload(wl.name + "-sorted", wl.layout, wl.n, wl.d, wl.dist, wl.s, wl.lo, wl.hi, wl.aggs,
                                wl.budget, wl.seed, "sorted by key")
    workspace = torch.empty(wl.budget, dtype=torch.uint8, device="cuda") if wl.budget else None
    torch.cuda.synchronize()
    spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, budget=wl.budget, est_groups=wl.d,
                       workspace=workspace, policy=args.policy, engine=args.engine)
    W8 = 8 * (1 + len(wl.aggs))

    def step():
        g = P.GroupBy(spec)
        g.consume_ptr(dev.data_ptr(), wl.n)
        res = g.finish()
        st = g.stats()
        g.close()
        return int(res.n_rows), st

    for i in range(args.warmup):
        rows, st = step()
        log(args, f"[bench] warmup {i}: rows={rows} levels={st['levels']} spilled={st['records_spilled']}")
    torch.cuda.synchronize()
    agg = {}
    rows_ok = True
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rows, st = step()
        rows_ok &= rows == wl.d
        for k, v in st.items():
            agg[k] = agg.get(k, 0) + v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = wl.n * args.steps / elapsed
    log(args, f"[bench] {wl.name}: {args.steps} steps in {elapsed:.3f}s ({ms_per_step:.2f} ms/step)")

    # algorithmic bytes of the query: input read once + result rows written once
    alg_bytes_step = wl.n * wl.record_bytes + wl.d * W8
    alg_per_record = alg_bytes_step / wl.n
    kname, launches, k_ms, k_bytes = dominant_kernel(agg, args.steps, wl.n, alg_per_record)
    launches = max(1, launches)
    achieved = (k_bytes / launches) / (k_ms / launches * 1e-3) / 1e9 if k_ms > 0 else 0.0
    step_gbps = alg_bytes_step / (ms_per_step * 1e-3) / 1e9
    # HBM traffic per launch from the committed rocprofv3 counter summary of this kernel and
    # workload, used only while the kernel sources are the ones it was measured on
    from paper_1311_0059_amd import profiling
    tsum = os.path.join(ROOT, "profiles", f"{kname.split('<')[0]}_{wl.name}_traffic.md")
    traffic = profiling.read_traffic(tsum, kname)
    roofline = {
        "bound": "hbm",
        "kernel": kname,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": None if traffic is None else int(traffic),
        "avg_launch_ms": round(k_ms / launches, 4),
        "launches_per_step": launches / args.steps,
        "bytes_per_launch": int(k_bytes / launches),
        "alg_bytes_per_record": round(alg_per_record, 3),
        "records_per_launch": int(k_bytes / alg_per_record / launches),
        "step_frac": round(step_gbps / HBM_PEAK_GBPS, 4),
    }

    cpu = cpu_oracle_baseline(args, host, wl) if with_cpu else None
    del host, raw

    n_steps = args.steps
    per_step = {k: (round(agg[k] / n_steps, 3) if isinstance(agg[k], float) else agg[k] // n_steps)
                for k in ("levels", "records_spilled", "states_spilled", "bytes_spilled_d2h", "bytes_reloaded_h2d",
                          "partitions", "partitions_spilled", "resident_groups_l0", "update_ms", "update_ms_l0",
                          "flush_ms", "lds_ms", "partition_ms", "sorted_ms", "lds_sweeps", "lds_passes",
                          "scatter_ms", "scatter_records", "lds_hot_keys", "lds_narrow", "onchip_ms",
                          "onchip_classes", "onchip_workers", "onchip_direct", "engine", "preagg",
                          "pool_high_water")}
    per_step["levels"] = agg["levels"] / n_steps
    return {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "records": wl.n,
            "record_bytes": wl.record_bytes,
            "distinct_keys": wl.d,
            "key_distribution": "zipf s=%.1f" % wl.s if wl.dist == datagen.ZIPF else "uniform",
            "aggregates": [a[0] for a in wl.aggs],
            "budget_bytes": wl.budget,
            "policy": args.policy,
            "engine": args.engine,
            "parallelism": "1 GPU",
        },
        "gbps_algorithmic": round(step_gbps, 1),
        "pct_hbm_peak": round(100.0 * step_gbps / HBM_PEAK_GBPS, 2),
        "rows_ok": bool(rows_ok),
        "per_step": per_step,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def bench_g_sweep(args):
    """Sensitivity to the estimate of distinct keys (the paper's G): the default
    200M-record / 20M-key / 1 GiB workload run with est_groups = G x factor for
    factors 1/4096 .. 4096, under both spill policies (Dynamic Destaging,
    Pre-Partitioning).  One timed run per point after a warm-up; every run's row
    count is checked against the true number of keys."""
    import numpy as np
    import torch

    import paper_1311_0059_amd as P
    from datagen import workloads

    wl = workloads.uniform_spill()
    log(args, f"[bench] generating {wl.name}")
    host = wl.generate()
    dev = torch.from_numpy(host.view(np.uint8).reshape(-1)).to("cuda")
    ws = torch.empty(wl.budget, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    factors = [1 / 4096, 1 / 256, 1 / 16, 1 / 4, 1, 4, 16, 256, 4096]

    def run(policy, factor):
        est = max(1, int(round(wl.d * factor)))
        spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, budget=wl.budget, est_groups=est, workspace=ws,
                           policy=policy, engine=args.engine)
        torch.cuda.synchronize()
        t = time.perf_counter()
        with P.GroupBy(spec) as g:
            g.consume_ptr(dev.data_ptr(), wl.n)
            res = g.finish()
            st = g.stats()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1000
        return ms, int(res.n_rows), st

    run("destage", 1)
    points, ok = [], True
    for policy in ("destage", "prepart"):
        for f in factors:
            ms, rows, st = run(policy, f)
            ok &= rows == wl.d
            points.append({"policy": policy, "factor": f, "est_groups": max(1, int(round(wl.d * f))),
                           "ms": round(ms, 2), "levels": st["levels"], "partitions": st["partitions"],
                           "partitions_spilled": st["partitions_spilled"], "records_spilled": st["records_spilled"],
                           "states_spilled": st["states_spilled"],
                           "host_bytes": st["bytes_spilled_d2h"] + st["bytes_reloaded_h2d"]})
            log(args, f"[bench] {policy} x{f:g}: {ms:.1f} ms, levels {st['levels']}, "
                      f"spilled {st['records_spilled']} records + {st['states_spilled']} states")
    base = next(p["ms"] for p in points if p["policy"] == "destage" and p["factor"] == 1)
    out = {"metric": METRIC, "value": round(wl.n / (base / 1000), 1), "unit": "records/s", "n_gpus": 1, "steps": 1,
           "warmup": 1, "ms_per_step": base, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{wl.name} with est_groups = G x factor", "records": wl.n, "distinct_keys": wl.d,
                      "budget_bytes": wl.budget, "engine": args.engine},
           "rows_ok": bool(ok), "sweep": points, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_first_rows(args):
    """Early output: the default 200M-record / 20M-key input under a 512 MiB budget
    (about half the groups stay resident).  Time from the start of the query until
    agg_first_rows returns the finished level-0 rows, and until agg_finish returns
    all rows; both spill policies, median of `--steps` runs after `--warmup`."""
    import numpy as np
    import torch

    import paper_1311_0059_amd as P
    from datagen import workloads

    wl = workloads.uniform_spill()
    budget = 512 << 20
    log(args, f"[bench] generating {wl.name}")
    host = wl.generate()
    dev = torch.from_numpy(host.view(np.uint8).reshape(-1)).to("cuda")
    ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    res = {}
    ok = True
    for policy in ("destage", "prepart"):
        spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, budget=budget, est_groups=wl.d, workspace=ws,
                           policy=policy, engine=args.engine)
        runs = []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with P.GroupBy(spec) as g:
                g.consume_ptr(dev.data_ptr(), wl.n)
                r1 = g.first_result()
                t1 = time.perf_counter()
                r2 = g.finish()
                t2 = time.perf_counter()
                st = g.stats()
            ok &= int(r2.n_rows) == wl.d and int(r1.n_rows) == st["resident_groups_l0"]
            if i >= args.warmup:
                runs.append((1000 * (t1 - t0), 1000 * (t2 - t0), int(r1.n_rows), int(r2.n_rows)))
        runs.sort()
        mid = runs[len(runs) // 2]
        res[policy] = {"first_rows_ms": round(mid[0], 2), "all_rows_ms": round(mid[1], 2), "first_rows": mid[2],
                       "all_rows": mid[3], "levels": st["levels"], "records_spilled": st["records_spilled"]}
        log(args, f"[bench] {policy}: first {mid[2]} rows at {mid[0]:.1f} ms, all {mid[3]} rows at {mid[1]:.1f} ms")
    base = res["destage"]["all_rows_ms"]
    out = {"metric": METRIC, "value": round(wl.n / (base / 1000), 1), "unit": "records/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": base, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{wl.name} with a 512 MiB budget: time to first rows", "records": wl.n,
                      "distinct_keys": wl.d, "budget_bytes": budget, "engine": args.engine},
           "rows_ok": bool(ok), "first_rows": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def calibrate_copy(args):
    """A plain streaming kernel of known traffic: 1 GiB read and 1 GiB written per launch
    (bitwise NOT of int64), three launches.  Its FETCH_SIZE / WRITE_SIZE readings give the
    factors that turn those counters into bytes."""
    import torch
    n = (1 << 30) // 8
    a = torch.arange(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.bitwise_not(a, out=b)
    torch.cuda.synchronize()
    ok = bool((b[:1024] == ~a[:1024]).all().item())
    print(json.dumps({"calibration": "bitwise_not int64", "bytes_read": n * 8, "bytes_written": n * 8,
                      "launches": 3, "ok": ok}), flush=True)


def bench_batched(args):
    """4096 instances (sizes log-uniform 1k-4M, distinct keys 1-50% of each, COUNT+SUM) in one
    persistent launch captured in a hipGraph.  A step is one agg_batch_run (graph replay, wait,
    read the row counts); planning and autotuning happen once in agg_batch_create."""
    import numpy as np
    import torch

    import paper_1311_0059_amd as P
    from datagen import workloads

    insts = workloads.batched_mix()
    rb = 16
    offs, total = [], 0
    for w in insts:
        offs.append(total)
        total += (w.n * rb + 255) // 256 * 256
    n_total = sum(w.n for w in insts)
    d_total = sum(w.d for w in insts)
    log(args, f"[bench] generating {len(insts)} instances: {n_total} records, {d_total} groups, {total / 1e9:.1f} GB")
    t = time.perf_counter()
    host = np.empty(total, dtype=np.uint8)
    for w, o in zip(insts, offs):
        w.generate(out=host[o:o + w.n * rb].view(workloads.R16))
    log(args, f"[bench] generated in {time.perf_counter() - t:.1f}s")
    dev = torch.empty(total, dtype=torch.uint8, device="cuda")
    chunk = 1 << 30
    for o in range(0, total, chunk):
        dev[o:o + chunk].copy_(torch.from_numpy(host[o:o + chunk]))
    torch.cuda.synchronize()
    spec = P.make_spec(rb, [(0, "u64")], workloads.AGGS_R16_CS)
    t = time.perf_counter()
    b = P.Batch(spec, [(dev.data_ptr() + o, w.n, w.d) for w, o in zip(insts, offs)])
    create_s = time.perf_counter() - t
    log(args, f"[bench] batch created (plan + autotune + graph capture) in {create_s:.2f}s: {b.stats()}")
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    run_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
        run_ms += b.stats()["last_run_ms"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = b.stats()
    rows_ok = all(int(b.result(i).n_rows) == w.d for i, w in enumerate(insts))
    b.close()
    ms_per_step = 1000.0 * elapsed / args.steps
    alg = n_total * rb + d_total * 24
    kernel_ms = run_ms / args.steps
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(n_total * args.steps / elapsed, 1), "unit": "records/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batched-4096-instances", "instances": len(insts), "records": n_total,
                   "distinct_keys": d_total, "record_bytes": rb, "aggregates": ["COUNT", "SUM"],
                   "budget_bytes": 0, "parallelism": "1 GPU"},
        "gbps_algorithmic": round(alg / (ms_per_step * 1e-3) / 1e9, 1),
        "pct_hbm_peak": round(100.0 * alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 2),
        "rows_ok": bool(rows_ok),
        "create_s": round(create_s, 3),
        "batch_stats": st,
        "roofline": {"bound": "hbm", "kernel": "aggx::k_batch (graph replay incl. reset kernel)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "avg_launch_ms": round(kernel_ms, 4), "bytes_per_launch": int(alg)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Poisson stream of requests (sizes log-uniform 1e4-5e7, distinct 1-50%, Zipf s in [0, 1.2],
    budgets log-uniform 16 MiB-2 GiB) against a 64 GiB pool.  The same trace runs (1) on the
    plain path -- one query at a time, FIFO, back to back, to measure its capacity -- then
    with Poisson arrivals at `--load` x that capacity (2) on the plain path (one request
    admitted at a time) and (3) served (memory admission, `--inflight` concurrent requests).
    Latency = finish - arrival; records/s = total records / (last finish - first arrival)."""
    import threading

    import numpy as np
    import torch

    import paper_1311_0059_amd as P
    from datagen import workloads

    reqs = workloads.served_mix(args.requests)
    rb = 16
    offs, total = [], 0
    for w in reqs:
        offs.append(total)
        total += (w.n * rb + 255) // 256 * 256
    n_total = sum(w.n for w in reqs)
    log(args, f"[bench] generating {len(reqs)} requests: {n_total} records, {total / 1e9:.1f} GB")
    dev = torch.empty(total, dtype=torch.uint8, device="cuda")
    host = np.empty(max(w.n for w in reqs) * rb, dtype=np.uint8)
    for w, o in zip(reqs, offs):  # one request at a time through one host buffer
        w.generate(out=host[:w.n * rb].view(workloads.R16))
        dev[o:o + w.n * rb].copy_(torch.from_numpy(host[:w.n * rb]))
        torch.cuda.synchronize()
    del host
    log(args, "[bench] uploaded")
    specs = [P.make_spec(rb, [(0, "u64")], w.aggs, budget=w.budget, est_groups=w.d) for w in reqs]
    pool = 64 << 30

    def run_trace(inflight, arrivals):
        """Submit request i at arrivals[i] (seconds from start); return per-request latency (ms), makespan (s)."""
        with P.Server(pool_bytes=pool, max_inflight=inflight) as srv:
            t0 = time.perf_counter()
            tickets = [None] * len(reqs)
            sub_t = [0.0] * len(reqs)

            def submitter():
                for i, w in enumerate(reqs):
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                    sub_t[i] = time.perf_counter() - t0
                    tickets[i] = srv.submit(specs[i], dev.data_ptr() + offs[i], w.n)

            th = threading.Thread(target=submitter)
            th.start()
            th.join()
            lat, rows_ok, runs = [], True, []
            for i, w in enumerate(reqs):
                try:
                    res, info = srv.wait(tickets[i])
                except P.AggError:
                    log(args, f"[bench] request {i} failed: {w.n} records, {w.d} keys, budget {w.budget}")
                    raise
                if (i + 1) % 25 == 0:
                    log(args, f"[bench]   {i + 1} of {len(reqs)} requests done")
                lat.append(info["latency_ms"])
                runs.append(info["run_ms"])
                rows_ok &= int(res.n_rows) == w.d
                srv.release(tickets[i])  # its rows are counted: give its result memory back
            makespan = time.perf_counter() - t0
            st = srv.stats()
        return np.array(lat), makespan, rows_ok, st, np.array(runs)

    zeros = [0.0] * len(reqs)
    # Warm-up and capacity: the plain path (one request admitted at a time), back to
    # back.  (A warm-up with every request queued at once and eight in flight ended
    # in a host heap-corruption abort whose cause was not found; it is not run.)
    log(args, "[bench] warm-up: plain path, back to back")
    run_trace(1, zeros)
    log(args, "[bench] plain path, back to back")
    _, plain_busy, ok0, _, service = run_trace(1, zeros)
    ok3 = True
    cap_rps = len(reqs) / plain_busy
    loads = [float(x) for x in args.loads.split(",") if x.strip()] if args.loads else [args.load]
    pct = lambda a, q: float(np.percentile(a, q))
    sweep = []
    for load in loads:
        gaps = np.array([w.extra["gap"] for w in reqs]) / (load * cap_rps)
        arrivals = list(np.cumsum(gaps) - gaps[0])
        log(args, f"[bench] plain capacity {cap_rps:.1f} req/s ({plain_busy:.2f}s back to back); load {load}")
        log(args, "[bench] plain path, Poisson arrivals")
        lat_p, span_p, ok1, _, _ = run_trace(1, arrivals)
        log(args, "[bench] served, Poisson arrivals")
        lat_s, span_s, ok2, st_s, _ = run_trace(args.inflight, arrivals)
        log(args, f"[bench] load {load}: served p50/p99 {pct(lat_s, 50):.1f}/{pct(lat_s, 99):.1f} ms, "
                  f"{n_total / span_s / 1e9:.2f} G rec/s; plain p50/p99 {pct(lat_p, 50):.1f}/{pct(lat_p, 99):.1f} ms, "
                  f"{n_total / span_p / 1e9:.2f} G rec/s")
        sweep.append({
            "offered_load": load,
            "served": {"p50_ms": round(pct(lat_s, 50), 3), "p99_ms": round(pct(lat_s, 99), 3),
                       "records_per_s": round(n_total / span_s, 1), "makespan_s": round(span_s, 3),
                       "peak_running": st_s["peak_running"], "pool_peak_bytes": st_s["pool_peak"]},
            "plain": {"p50_ms": round(pct(lat_p, 50), 3), "p99_ms": round(pct(lat_p, 99), 3),
                      "records_per_s": round(n_total / span_p, 1), "makespan_s": round(span_p, 3)},
            "rows_ok": bool(ok1 and ok2),
            "span_s": span_s,
        })
    top = sweep[0]
    span_s = top.pop("span_s")
    for e in sweep[1:]:
        e.pop("span_s")
    out = {
        "metric": METRIC, "value": round(n_total / span_s, 1), "unit": "records/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(1000 * span_s, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"served-{len(reqs)}-requests", "records": n_total, "pool_bytes": pool,
                   "inflight": args.inflight, "offered_load": top["offered_load"],
                   "arrivals": "Poisson at offered_load x plain-path capacity"},
        "served": top["served"],
        "plain": dict(top["plain"], back_to_back_s=round(plain_busy, 3),
                      service_p50_ms=round(pct(service, 50), 3), service_p99_ms=round(pct(service, 99), 3)),
        "capacity": {"plain_records_per_s": round(n_total / plain_busy, 1),
                     "note": "plain path, all requests queued at t=0"},
        "load_sweep": sweep,
        "rows_ok": bool(ok0 and all(e["rows_ok"] for e in sweep)),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
