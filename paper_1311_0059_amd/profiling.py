"""Summaries of rocprofv3 output for the kernel rooflines.

Two kinds of input:
  * `--kernel-trace --stats` output (`*_kernel_stats.csv`): per-kernel call
    counts and durations;
  * `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` output (`*_counter_collection.csv`):
    per-dispatch HBM kilobytes fetched / written.

HBM traffic of a kernel launch = counter KiB x 1024 x a calibration factor.
The factor comes from a plain copy kernel of known size measured with the
same counter (bytes it must move / bytes the counter reports), so that a
counter that over- or under-counts is corrected by what it reads for a copy.

The summary is a short markdown file; it records a hash of the kernel sources
it was measured on, so a reader can tell when the figure no longer applies.

Usage:
  python -m paper_1311_0059_amd.profiling pmc \\
      --fetch F.csv --write W.csv --calib-fetch CF.csv --calib-write CW.csv \\
      --kernel 'k_update<0, 0>' --first N --alg-bytes B --calib-bytes C \\
      --command '...' --out profiles/<name>.md
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources whose change invalidates a measured traffic figure
KERNEL_SOURCES = ["csrc/aggx_kernels.hip", "csrc/aggx_device.h", "csrc/aggx_internal.h", "csrc/aggx_lds.hip",
                  "csrc/aggx_ldstab.h", "csrc/aggx_onchip.hip", "csrc/aggx_owner.hip", "csrc/aggx_sorted.hip",
                  "csrc/aggx_runtime.cpp"]


def sources_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(path: str, counter: str):
    """[(dispatch_id, kernel_name, value)] in dispatch order for one counter."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def per_dispatch(rows, kernel: str, first: int | None):
    vals = [v for _, name, v in rows if kernel in name]
    return vals[:first] if first else vals


def calib_factor(path: str, counter: str, known_bytes: float) -> tuple[float, str, float]:
    """known_bytes / (counter bytes) for the largest-valued dispatch (the copy kernel)."""
    rows = read_counters(path, counter)
    if not rows:
        raise SystemExit(f"{path}: no {counter} rows")
    _, name, kib = max(rows, key=lambda r: r[2])
    return known_bytes / (kib * 1024.0), name, kib


def summarize_pmc(a) -> str:
    f_rows = read_counters(a.fetch, "FETCH_SIZE")
    w_rows = read_counters(a.write, "WRITE_SIZE")
    f_vals = per_dispatch(f_rows, a.kernel, a.first)
    w_vals = per_dispatch(w_rows, a.kernel, a.first)
    if not f_vals or not w_vals:
        raise SystemExit(f"no dispatches of {a.kernel!r} in the counter files")
    cf, cf_name, cf_kib = calib_factor(a.calib_fetch, "FETCH_SIZE", a.calib_bytes)
    cw, cw_name, cw_kib = calib_factor(a.calib_write, "WRITE_SIZE", a.calib_bytes)
    f_avg = sum(f_vals) / len(f_vals)
    w_avg = sum(w_vals) / len(w_vals)
    traffic = f_avg * 1024.0 * cf + w_avg * 1024.0 * cw
    lines = [
        f"# HBM traffic of `{a.kernel}` ({a.workload})",
        "",
        "Commands (run from the repository root on the GPU host; `cd /tmp && export TMPDIR=/tmp` first):",
        "",
        "```",
        *a.command,
        "```",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| dispatches averaged | {len(f_vals)} (FETCH_SIZE), {len(w_vals)} (WRITE_SIZE) |",
        f"| FETCH_SIZE per dispatch | {f_avg:.1f} KiB |",
        f"| WRITE_SIZE per dispatch | {w_avg:.1f} KiB |",
        f"| copy calibration kernel | `{cf_name[:80]}` |",
        f"| copy: known bytes read = written | {a.calib_bytes:.0f} |",
        f"| copy: FETCH_SIZE / WRITE_SIZE | {cf_kib:.1f} KiB / {cw_kib:.1f} KiB |",
        f"| factor fetch / write | {cf:.4f} / {cw:.4f} |",
        f"| HBM traffic per launch (fetch x factor + write x factor) | {traffic:.0f} B |",
        f"| algorithmic bytes per launch | {a.alg_bytes:.0f} B |",
        f"| traffic / algorithmic | {traffic / a.alg_bytes:.2f} |",
        "",
        f"traffic_bytes_per_launch: {traffic:.0f}",
        f"kernel: {a.kernel}",
        f"sources_sha256: {sources_hash()}",
        "",
    ]
    return "\n".join(lines)


def read_traffic(path: str, kernel: str) -> float | None:
    """Traffic per launch from a summary, or None if absent, for another kernel,
    or measured on sources that have changed since."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    m_k = re.search(r"^kernel: (.+)$", text, re.M)
    m_h = re.search(r"^sources_sha256: ([0-9a-f]+)$", text, re.M)
    if not (m_t and m_k and m_h) or m_k.group(1).strip() != kernel or m_h.group(1) != sources_hash():
        return None
    return float(m_t.group(1))


def summarize_trace(a) -> str:
    """Kernel-trace summary: the stats table, and the per-dispatch durations of one kernel
    split by grid size (launch shape), for comparison with the HIP-event timing."""
    stats = list(csv.DictReader(open(a.stats, newline="")))
    lines = [f"# Kernel trace: {a.workload}", "", "Command (repository root on the GPU host; "
             "`cd /tmp && export TMPDIR=/tmp` first):", "", "```", *a.command, "```", "",
             "| kernel | calls | avg ns | total % |", "|---|---|---|---|"]
    for r in stats[: a.top]:
        lines.append(f"| `{r['Name'][:72]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{float(r['Percentage']):.2f} |")
    by_grid = {}
    with open(a.trace, newline="") as f:
        rows = [r for r in csv.DictReader(f) if a.kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[a.skip:]
    if a.first:
        rows = rows[: a.first]
    for r in rows:
        g = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1)) * int(r.get("Grid_Size_Z", 1))
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        by_grid.setdefault(g, []).append(dt)
    which = f"dispatches {a.skip + 1}-{a.skip + len(rows)} in time order" if a.skip or a.first else "all dispatches"
    lines += ["", f"Per-dispatch durations of `{a.kernel}` (End - Start, {which}), by grid size:", "",
              "| grid (threads) | dispatches | avg ms | min ms | max ms |", "|---|---|---|---|---|"]
    for g in sorted(by_grid, reverse=True):
        v = by_grid[g]
        lines.append(f"| {g} | {len(v)} | {sum(v) / len(v):.4f} | {min(v):.4f} | {max(v):.4f} |")
    if a.note:
        lines += ["", *a.note]
    lines.append("")
    return "\n".join(lines)


def summarize_counters(a) -> str:
    """Per-kernel sums of any counters over one or more `--pmc` runs of the same command
    (each run a `*_counter_collection.csv`), with derived ratios for the SQ counters."""
    tot = {}
    durs = {}
    for path in a.csv:
        for r in csv.DictReader(open(path, newline="")):
            name = r["Kernel_Name"].split("(")[0]
            if not any(k in name for k in a.kernel):
                continue
            key = (path, int(r["Dispatch_Id"]))
            tot.setdefault(name, {})
            tot[name][r["Counter_Name"]] = tot[name].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            durs.setdefault(name, {})[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    lines = [f"# Counters: {a.workload}", "", "Commands (repository root on the GPU host; "
             "`cd /tmp && export TMPDIR=/tmp` first), one run per counter set:", "", "```", *a.command, "```", ""]
    for name, c in tot.items():
        d = durs[name]
        lines += [f"## `{name}`", "", f"dispatches counted: {len(d)} (over {len(a.csv)} runs); "
                  f"average duration under the profiler {sum(d.values()) / len(d):.3f} ms", "",
                  "| counter | sum over the runs' dispatches |", "|---|---|"]
        for k in sorted(c):
            lines.append(f"| {k} | {c[k]:.4g} |")
        derived = []
        if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in c:
            derived.append(f"waiting share of wave time (SQ_WAIT_ANY / SQ_WAVE_CYCLES): {c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.2f}")
        if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_LDS" in c:
            derived.append(f"LDS-wait share (SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES): {c['SQ_WAIT_INST_LDS'] / c['SQ_WAVE_CYCLES']:.3f}")
        if c.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in c:
            derived.append(f"LDS bank-conflict cycles per LDS instruction: {c['SQ_LDS_BANK_CONFLICT'] / c['SQ_INSTS_LDS']:.2f}")
        if c.get("SQ_INSTS_LDS") and "SQ_LDS_ADDR_CONFLICT" in c:
            derived.append(f"LDS address-conflict cycles per LDS instruction: {c['SQ_LDS_ADDR_CONFLICT'] / c['SQ_INSTS_LDS']:.2f}")
        if c.get("SQ_WAVES") and "SQ_INSTS_VALU" in c:
            derived.append(f"VALU instructions per wave: {c['SQ_INSTS_VALU'] / c['SQ_WAVES']:.4g}")
        if "TCC_HIT_sum" in c and c.get("TCC_HIT_sum", 0) + c.get("TCC_MISS_sum", 0):
            derived.append(f"L2 hit rate: {c['TCC_HIT_sum'] / (c['TCC_HIT_sum'] + c.get('TCC_MISS_sum', 0)):.3f}")
        if "SQC_ICACHE_MISSES" in c and c.get("SQC_ICACHE_HITS"):
            derived.append(f"instruction-cache miss rate: {c['SQC_ICACHE_MISSES'] / (c['SQC_ICACHE_HITS'] + c['SQC_ICACHE_MISSES']):.2e}")
        if derived:
            lines += ["", *[f"* {x}" for x in derived]]
        lines.append("")
    if a.note:
        lines += [*a.note, ""]
    lines.append(f"sources_sha256: {sources_hash()}")
    lines.append("")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="paper_1311_0059_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("pmc", help="traffic summary from FETCH_SIZE / WRITE_SIZE runs")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--calib-fetch", required=True)
    p.add_argument("--calib-write", required=True)
    p.add_argument("--calib-bytes", type=float, required=True)
    p.add_argument("--kernel", required=True, help="substring of the kernel name")
    p.add_argument("--first", type=int, default=0, help="use only the first N dispatches of the kernel")
    p.add_argument("--alg-bytes", type=float, required=True, help="algorithmic bytes per launch")
    p.add_argument("--workload", default="")
    p.add_argument("--command", action="append", default=[])
    p.add_argument("--out", required=True)
    t = sub.add_parser("trace", help="summary of a --kernel-trace --stats run")
    t.add_argument("--stats", required=True)
    t.add_argument("--trace", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--top", type=int, default=10)
    t.add_argument("--skip", type=int, default=0, help="leave out the kernel's first N dispatches (time order)")
    t.add_argument("--first", type=int, default=0, help="then use only the next N dispatches")
    t.add_argument("--workload", default="")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--note", action="append", default=[])
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters", help="per-kernel sums of --pmc counter runs")
    c.add_argument("--csv", action="append", required=True, help="a *_counter_collection.csv (repeat per run)")
    c.add_argument("--kernel", action="append", required=True, help="substring of a kernel name (repeatable)")
    c.add_argument("--workload", default="")
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--note", action="append", default=[])
    c.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    text = {"pmc": summarize_pmc, "trace": summarize_trace, "counters": summarize_counters}[a.cmd](a)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    sys.exit(main())
