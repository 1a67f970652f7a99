"""Host-only test of the serving engine's admission policy (te_sched.h, the
header the server itself uses) with a virtual clock and a fake executor
(tests/sched_sim.cpp): budget never exceeded, one class per round, FIFO
within each class, the oldest waiting request choosing the class, heavy
rounds within the size spread, oversize requests rejected alone, every
other request served; latency percentiles reported."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1209_1910_amd", "csrc")


@pytest.fixture(scope="module")
def sim():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    tmp = tempfile.mkdtemp()
    exe = os.path.join(tmp, "sched_sim")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I", CSRC, "-o", exe,
                           os.path.join(ROOT, "tests", "sched_sim.cpp")])
    yield exe
    shutil.rmtree(tmp)


def _run(exe, *args):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout)


def test_policy_invariants_at_moderate_load(sim):
    out = _run(sim, 400, 2.0, 32 << 30, 3)
    assert out["rejected"] == 0
    assert out["p50_s"] <= out["p99_s"] <= out["makespan_s"]
    assert out["multi_request_rounds"] > 0          # queued requests are batched


def test_policy_under_a_small_budget(sim):
    """A budget below the largest requests: those are rejected alone, the
    rest still run, never beyond the budget."""
    out = _run(sim, 300, 5.0, 8 << 30, 3)
    assert out["rejected"] > 0
    assert out["rounds"] > 0 and out["p50_s"] <= out["p99_s"]


def test_policy_with_one_lane_and_saturation(sim):
    out = _run(sim, 200, 1000.0, 64 << 30, 1)
    assert out["multi_request_rounds"] > 0 and out["rejected"] == 0


HEAVY_ROUND_SRC = r"""
#include <cstdio>
#include <deque>
#include <vector>
#include "te_sched.h"
struct R { long long id; int n, m; };
int main() {
  // heavy queue: sizes alternate between about 1e8 and 1e7 entries (a factor
  // 10 apart); a light request arrived last
  std::vector<R> rs = {{1, 10000, 10000}, {2, 3000, 3000}, {3, 9000, 9000}, {4, 3200, 3200},
                       {5, 9500, 9500}, {6, 13000, 13000}, {7, 100, 100}};
  std::deque<R *> light, heavy;
  for (int k = 0; k < 6; k++) heavy.push_back(&rs[k]);
  light.push_back(&rs[6]);
  auto need = [](const std::vector<R *> &v) {
    size_t b = 0;
    for (const R *r : v) b += (size_t)r->n * r->m;   // one byte per entry
    return b;
  };
  std::vector<R *> round;
  size_t bytes = 0;
  const unsigned long long budget = 400000000ull;    // room for 1, 3, 5 but not also 6
  int rc = te::sched_next(light, heavy, budget, 0, need, round, bytes);
  std::printf("%d", rc);
  for (R *r : round) std::printf(" %lld", r->id);
  std::printf(" |");
  for (R *r : heavy) std::printf(" %lld", r->id);
  std::printf(" | %zu\n", bytes);
  return 0;
}
"""


def test_heavy_round_passes_over_incompatible_requests(tmp_path):
    """A heavy round takes every queued heavy request within the size spread of
    its head that fits the budget, in queue order; the others keep their
    places (and their order) for the next round."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "hr.cpp"
    src.write_text(HEAVY_ROUND_SRC)
    exe = str(tmp_path / "hr")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I", CSRC, "-o", exe, str(src)])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout.split("|")
    rc_round = out[0].split()
    assert rc_round[0] == "1"
    assert [int(x) for x in rc_round[1:]] == [1, 3, 5]        # 6 is compatible but over budget
    assert [int(x) for x in out[1].split()] == [2, 4, 6]        # passed over, order kept
    assert int(out[2]) == 10000 ** 2 + 9000 ** 2 + 9500 ** 2
