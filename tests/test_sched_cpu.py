"""Host-only test of the serving engine's admission policy (te_sched.h, the
header the server itself uses) with a virtual clock and a fake executor
(tests/sched_sim.cpp): budget never exceeded, one class per round, FIFO
within each class, the oldest waiting request choosing the class, heavy
rounds within the size spread, oversize requests rejected alone, every
other request served; latency percentiles reported.  The simulation is built
with AddressSanitizer and UndefinedBehaviorSanitizer."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1209_1910_amd", "csrc")
# host code only, built with g++: AddressSanitizer and UndefinedBehaviorSanitizer
SAN = ["-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module")
def sim():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    tmp = tempfile.mkdtemp()
    exe = os.path.join(tmp, "sched_sim")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-Wall", *SAN, "-I", CSRC, "-o", exe,
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
