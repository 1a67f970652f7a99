"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs every exported routine on small inputs and edge
cases (oracle/sanitize_driver.c); any memory error, leak or undefined
behaviour fails the run."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan():
    tmp = tempfile.mkdtemp()
    try:
        exe = os.path.join(tmp, "drv")
        subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-o", exe, os.path.join(ORACLE, "oracle.c"),
                               os.path.join(ORACLE, "sanitize_driver.c"), "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ok" in r.stdout
    finally:
        shutil.rmtree(tmp)
