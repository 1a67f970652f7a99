"""CPU checks of the benchmark's own arithmetic and contract: the algorithmic
byte and flop counts the roofline and the CPU baseline rest on, against
brute-force sums of their per-step definitions; the extrapolated CPU baseline
against a full oracle run of a small case; and the one-GPU contract."""
from __future__ import annotations

import os
import subprocess
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _bytes_brute(n, M, iters=3):
    # per compact-WY step of member c (c = 1..M-1): Y_c^T v reads the
    # trapezoid (column l has rows l..n-1), the Yhat passes (n - c) c, Y_{c+1}
    # x'' the trapezoid of c + 1 columns, T_c^T x and T_c [s r] the triangle
    # of order c each (c (c + 1) / 2 entries twice); writes: the new y column
    # (n - c), the new T column (c + 1) and q (n)
    tot = 0
    for c in range(1, M):
        trap_c = sum(n - l for l in range(c))
        trap_c1 = sum(n - l for l in range(c + 1))
        tot += trap_c + (n - c) * c + trap_c1 + c * (c + 1) + (n - c) + (c + 1) + n
    return 8.0 * iters * tot


@pytest.mark.parametrize("n,M", [(10, 5), (37, 37), (200, 64)])
def test_chain_alg_bytes_matches_its_definition(n, M):
    assert bench.chain_alg_bytes(n, M) == pytest.approx(_bytes_brute(n, M), rel=1e-12)


def test_chain_alg_bytes_of_the_headline_workload():
    assert bench.chain_alg_bytes(16000, 16000) == pytest.approx(1.1470e14, rel=1e-3)


def test_chain_flops_matches_the_step_count():
    n, k = 300, 40
    brute = 3 * sum(8 * n * c - 3 * c * c for c in range(1, k))
    assert bench._chain_flops(n, k) == pytest.approx(brute, rel=1e-12)


def test_cpu_baseline_extrapolates_a_full_run():
    """The fitted model, evaluated at k = n, against the oracle timed on the
    whole problem (n = 700: a single cluster of 700 members); timing on a
    shared CPU, so a loose bound."""
    pytest.importorskip("scipy")
    import oracle
    from paper_1209_1910_amd import inputs
    n = 700
    out = bench.cpu_baseline(n, ks=(120, 170, 220))
    d, e = inputs.workload_laplacian(n)
    t0 = time.perf_counter()
    oracle.eigvecs(d, e)
    t_full = time.perf_counter() - t0
    assert out["fit"]["t_full_s"] == pytest.approx(t_full, rel=1.0)
    assert out["value"] == pytest.approx(n / out["fit"]["t_full_s"])
    assert out["cores"] == 1 and out["kind"] == "oracle" and out["nproc"] >= 1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
