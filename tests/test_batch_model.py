"""The batched mode's launch model (a replay of its work queue, host code only) on cases
whose times follow by hand: one item alone, many equal items sharing the device's rate,
an instance's dependency chain, and fewer workgroups than items."""
import subprocess

import pytest

from tests.conftest import ROOT

HARNESS = r"""
#include <cstdio>
#include "%s/paper_1311_0059_amd/csrc/aggx_batch_model.h"
using namespace aggx;
int main() {
  const BatchModelParams m = {1000.0, 100.0, 0.5, 0.01, 0.25, 2.0};
  // one count item of 400 bytes over 8 bins, alone: 0.5 + 0.08 fixed, 400 / 100 streaming
  printf("%%.9f\n", simulate_batch({{SM_COUNT, 0, 8, 400.0}}, {1}, 4, m));
  // 20 solo items of 1000 bytes on 20 workgroups: 0.75 fixed, then each streams at 1000/20 = 50
  std::vector<SimItem> v(20, SimItem{SM_SOLO, 0, 1, 1000.0});
  printf("%%.9f\n", simulate_batch(v, std::vector<uint32_t>(20, 0), 20, m));
  // the same on 10 workgroups: two rounds, each with ten streams at min(100, 1000/10) = 100
  printf("%%.9f\n", simulate_batch(v, std::vector<uint32_t>(20, 0), 10, m));
  // one partitioned instance (2 chunks, 4 bins): two counts of 100 bytes at once, offsets,
  // two scatters of 200 bytes at once, four aggregations of 50 bytes at once
  std::vector<SimItem> c = {{SM_COUNT, 0, 4, 100.0}, {SM_COUNT, 0, 4, 100.0}, {SM_OFFS, 0, 4, 0.0},
                            {SM_SCATTER, 0, 4, 200.0}, {SM_SCATTER, 0, 4, 200.0},
                            {SM_AGG, 0, 4, 50.0}, {SM_AGG, 0, 4, 50.0}, {SM_AGG, 0, 4, 50.0}, {SM_AGG, 0, 4, 50.0}};
  printf("%%.9f\n", simulate_batch(c, {2}, 16, m));
  // nothing to do: the launch alone
  printf("%%.9f\n", simulate_batch({}, {}, 16, m));
  return 0;
}
"""


@pytest.fixture(scope="module")
def model_out(tmp_path_factory):
    d = tmp_path_factory.mktemp("batch_model")
    src, exe = d / "h.cpp", d / "h"
    src.write_text(HARNESS % ROOT)
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", str(exe), str(src)], check=True)
    return [float(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]


def test_single_item(model_out):
    assert model_out[0] == pytest.approx(0.5 + 0.08 + 400 / 100 + 2.0)


def test_shared_device_rate(model_out):
    assert model_out[1] == pytest.approx(0.75 + 1000 / 50 + 2.0)


def test_more_items_than_workgroups(model_out):
    assert model_out[2] == pytest.approx(2 * (0.75 + 1000 / 100) + 2.0)


def test_dependency_chain(model_out):
    count = 0.5 + 0.04 + 100 / 100
    offs = 0.5 + 0.04
    scat = 0.5 + 0.04 + 200 / 100
    agg = 0.75 + 50 / 100
    assert model_out[3] == pytest.approx(count + offs + scat + agg + 2.0)


def test_empty(model_out):
    assert model_out[4] == pytest.approx(2.0)
