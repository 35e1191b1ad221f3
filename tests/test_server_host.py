"""The served mode's host code under AddressSanitizer and ThreadSanitizer, on the CPU.

The server's source (csrc/aggx_server.cpp) is compiled with CPU stand-ins for the
HIP runtime and for the single-query calls (tests/server_host/), and driven with the
served benchmark's request trace: its sizes and budgets, a 64 GiB pool, every request
submitted at once by one thread while another waits for them in ticket order and
releases each, with six and with eight (more than the library accepts on a GPU) and
twelve requests in flight; the last round destroys the server with requests still
queued.  A heap error, a data race or a lost request fails the test.
"""
import os
import subprocess

import pytest

from datagen import workloads
from tests.conftest import ROOT

HERE = os.path.join(ROOT, "tests", "server_host")


def _trace(tmp_path, n_req):
    p = tmp_path / "trace.txt"
    p.write_text("".join(f"{w.n} {w.budget}\n" for w in workloads.served_mix(n_req)))
    return str(p)


def _build(tmp_path, san):
    exe = tmp_path / f"harness_{san}"
    flags = {"asan": ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"], "tsan": ["-fsanitize=thread"]}[san]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", *flags, "-I", HERE, "-o", str(exe),
                    os.path.join(HERE, "harness.cpp")], check=True, capture_output=True)
    return str(exe)


@pytest.mark.parametrize("san", ["asan", "tsan"])
def test_served_trace_all_queued(tmp_path, san):
    exe = _build(tmp_path, san)
    trace = _trace(tmp_path, 1000)
    env = dict(os.environ, MALLOC_CHECK_="3", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               TSAN_OPTIONS="halt_on_error=1")
    for inflight in (6, 8, 12):
        r = subprocess.run([exe, trace, str(inflight), "3"], env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, f"{san} {inflight} in flight:\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
        assert "server harness ok" in r.stdout
        assert f"peak {inflight} in flight" in r.stdout or inflight > 8  # the trace keeps them all busy


def test_served_trace_through_the_binding(tmp_path):
    """The same trace driven from Python threads through the binding's Server class, with the
    stand-in library under AddressSanitizer (preloaded into the interpreter)."""
    so = tmp_path / "libharness.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-shared", "-fPIC", "-DAGGX_HARNESS_LIB",
                    "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-I", HERE, "-o", str(so),
                    os.path.join(HERE, "harness.cpp")], check=True, capture_output=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()
    ubsan = subprocess.run(["g++", "-print-file-name=libubsan.so"], check=True, capture_output=True,
                           text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               MALLOC_CHECK_="3")
    r = subprocess.run(["python", os.path.join(HERE, "drive.py"), str(so), "8", "1000", "2"], env=env,
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, f"{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    assert "python driver ok" in r.stdout and "peak 8 in flight" in r.stdout
