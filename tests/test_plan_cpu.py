"""Host-only test of the chain-to-kernel rule (te_plan.h, the header the
library itself uses): large chains go to the cooperative kernel; mid-size
chains join them when the call has at most as many chains as that kernel has
workgroups and no cooperative chain costs more than kPromoteRatio times the
largest mid-size one; MGS chains always run one per workgroup.  The driver
is built with AddressSanitizer and UndefinedBehaviorSanitizer."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1209_1910_amd", "csrc")
# host code only, built with g++: AddressSanitizer and UndefinedBehaviorSanitizer
SAN = ["-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "te_plan.h"
// stdin: coop_wgs mgs K, then K pairs (n size); stdout: one kernel code per chain
int main() {
  size_t wgs; int mgs, K;
  if (std::scanf("%zu %d %d", &wgs, &mgs, &K) != 3) return 1;
  std::vector<int> n(K), s(K);
  for (int k = 0; k < K; k++)
    if (std::scanf("%d %d", &n[k], &s[k]) != 2) return 1;
  for (char c : te::chain_kernels(n, s, wgs, mgs != 0)) std::printf("%d ", (int)c);
  std::printf("\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def drv(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("plan")
    src = d / "plan.cpp"
    src.write_text(DRIVER)
    exe = str(d / "plan")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-Wall", *SAN, "-I", CSRC, "-o", exe, str(src)])
    return exe


def _kernels(exe, chains, wgs=256, mgs=False):
    inp = f"{wgs} {int(mgs)} {len(chains)}\n" + "\n".join(f"{n} {s}" for n, s in chains)
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0
    return [int(x) for x in r.stdout.split()]


ONE_WG, COOP, PROMOTED = 0, 1, 2


def test_single_large_cluster(drv):
    assert _kernels(drv, [(16000, 16000)]) == [COOP]


def test_mid_size_chains_alone_are_promoted(drv):
    # 2100 x 200 = 420,000 entries: below the cooperative size, above the
    # promotion size; 2100 x 20 stays one per workgroup
    assert _kernels(drv, [(2100, 200)] * 10 + [(2100, 20)] * 3) == [PROMOTED] * 10 + [ONE_WG] * 3


def test_mid_size_chains_join_comparable_large_ones(drv):
    # clusters of 400 (cooperative) and 200 members at n = 4200: cost ratio 4
    out = _kernels(drv, [(4200, 400)] * 10 + [(4200, 200)] * 10)
    assert out == [COOP] * 10 + [PROMOTED] * 10


def test_mid_size_chains_stay_beside_a_much_costlier_chain(drv):
    # a few huge clusters and many of tens of members at n = 9527
    chains = [(9527, 3086), (9527, 2970), (9527, 1958), (9527, 564), (9527, 110)]
    chains += [(9527, 20)] * 40
    out = _kernels(drv, chains)
    assert out[:4] == [COOP] * 4 and out[4:] == [ONE_WG] * 41


def test_no_promotion_beyond_the_workgroup_count(drv):
    out = _kernels(drv, [(2100, 200)] * 300)
    assert out == [ONE_WG] * 300
    out = _kernels(drv, [(2100, 200)] * 256)
    assert out == [PROMOTED] * 256


def test_mgs_chains_run_one_per_workgroup(drv):
    assert _kernels(drv, [(16000, 16000), (2100, 200)], mgs=True) == [ONE_WG, ONE_WG]
