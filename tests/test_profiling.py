"""Host logic of the rocprofv3 summaries (no GPU): the traffic figure, its copy
calibration, and its invalidation when the kernel sources change."""
import csv
import os

from paper_1311_0059_amd import profiling


def _counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def _summarize(tmp_path, first=0):
    d = str(tmp_path)
    # two dispatches of the kernel (and one of another) in each run
    _counters(os.path.join(d, "f.csv"), "FETCH_SIZE", [("k_a(x)", 100.0), ("k_b(y)", 7.0), ("k_a(x)", 300.0)])
    _counters(os.path.join(d, "w.csv"), "WRITE_SIZE", [("k_a(x)", 50.0), ("k_b(y)", 9.0), ("k_a(x)", 150.0)])
    # a 1 MiB copy: the fetch counter reports half of it, the write counter all of it
    _counters(os.path.join(d, "cf.csv"), "FETCH_SIZE", [("tiny", 1.0), ("copy", 512.0)])
    _counters(os.path.join(d, "cw.csv"), "WRITE_SIZE", [("copy", 1024.0)])
    out = os.path.join(d, "k_a_traffic.md")
    profiling.main(["pmc", "--fetch", os.path.join(d, "f.csv"), "--write", os.path.join(d, "w.csv"),
                    "--calib-fetch", os.path.join(d, "cf.csv"), "--calib-write", os.path.join(d, "cw.csv"),
                    "--calib-bytes", str(1 << 20), "--kernel", "k_a", "--first", str(first),
                    "--alg-bytes", "100000", "--workload", "w", "--command", "cmd", "--out", out])
    return out


def test_traffic_is_calibrated_average_per_dispatch(tmp_path):
    out = _summarize(tmp_path)
    # fetch: mean 200 KiB x 2 (calibration); write: mean 100 KiB x 1
    want = 200 * 1024 * 2 + 100 * 1024
    assert profiling.read_traffic(out, "k_a") == want
    assert "| dispatches averaged | 2 (FETCH_SIZE), 2 (WRITE_SIZE) |" in open(out).read()


def test_first_dispatches_only(tmp_path):
    out = _summarize(tmp_path, first=1)
    assert profiling.read_traffic(out, "k_a") == 100 * 1024 * 2 + 50 * 1024


def test_stale_or_foreign_summary_gives_none(tmp_path):
    out = _summarize(tmp_path)
    assert profiling.read_traffic(out, "k_b") is None  # summary of another kernel
    text = open(out).read().replace(f"sources_sha256: {profiling.sources_hash()}", "sources_sha256: 0000")
    with open(out, "w") as f:
        f.write(text)
    assert profiling.read_traffic(out, "k_a") is None  # measured on other sources
    assert profiling.read_traffic(os.path.join(str(tmp_path), "missing.md"), "k_a") is None
