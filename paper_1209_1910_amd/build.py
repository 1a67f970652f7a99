"""Build the HIP C-ABI library in-tree (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtridiag_eigvecs.so")
SOURCES = [os.path.join(CSRC, "te_kernels.hip"), os.path.join(CSRC, "te_api.hip"),
           os.path.join(CSRC, "te_server.hip")]
HEADERS = [os.path.join(CSRC, "te_internal.h"), os.path.join(CSRC, "te_host.h"),
           os.path.join(CSRC, "te_sched.h"), os.path.join(CSRC, "te_plan.h"),
           os.path.join(ROOT, "include", "tridiag_eigvecs.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # FP64 results depend on the rounding of every operation: no contraction
    # into FMA unless the source writes fma(), no fast-math.
    "-ffp-contract=off",
    "-fno-fast-math",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every source into libtridiag_eigvecs.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
