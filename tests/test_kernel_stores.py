"""Guard for the cross-workgroup visibility rule of the chain kernels: data
that other workgroups read after a group barrier is written with st_dev
(write-through device-scope stores); a plain store to such data passes a
single run and fails now and then when several groups share the device.
This test reads the chain section of te_kernels.hip and checks that every
plain subscript store goes to a register array, LDS, or one of the listed
global stores that are released by other means (the back sweep's solution
rows, published with a release fence, and the sweep's carries, read only by
the same workgroup)."""
from __future__ import annotations

import os
import re

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1209_1910_amd", "csrc", "te_kernels.hip")

# plain global stores that do not need st_dev, with the reason
ALLOWED = {
    "xb": "back sweep rows; the sweep releases them with a fence when it publishes progress",
    "v": "back sweep rows of the partial last block; released by the same fence",
    "carry_glb": "chunk carries of the solve, read back only by the sweeping workgroup",
}


def _chain_section(text):
    a = text.index("struct Ctx {")
    b = text.index("__global__ void __launch_bounds__(256) k_finalize")
    return text[a:b]


def test_shared_chain_data_is_stored_with_st_dev():
    text = open(SRC).read()
    sec = _chain_section(text)
    code = re.sub(r"//[^\n]*", "", sec)
    local = set()
    # register arrays: every declarator of a declaration statement, e.g.
    # "double a0[R], a1[R];", and array-reference parameters "(&out)[R]"
    for m in re.finditer(r"\b(?:const\s+)?(?:double|int|float|unsigned|bool|SRow|d2v|ldrp|char|"
                         r"size_t)\s+([^;()]*\[[^;()]*);", code):
        local |= set(re.findall(r"([A-Za-z_]\w*)\s*\[", m.group(1)))
    local |= set(re.findall(r"\(\s*&\s*([A-Za-z_]\w*)\s*\)\s*\[", code))
    local |= set(re.findall(r"__shared__\s+[^;]*?\b([A-Za-z_]\w*)\s*\[", code))
    local |= {"ring", "carry_lds", "s_ring", "s_p", "s_red", "s_carry"}
    targets = set()
    for m in re.finditer(r"(?<![\w.>])([A-Za-z_][\w.]*)\s*(\[[^\]\n]+\])+\s*=(?!=)", code):
        name = m.group(1)
        base = name.split(".")[0]
        if name in local or base in local or name.startswith("s_ring"):
            continue
        targets.add(name)
    bad = sorted(t for t in targets if t not in ALLOWED)
    assert not bad, ("plain stores to possibly shared global data in the chain kernels "
                     f"(use st_dev, or add the store to ALLOWED with its reason): {bad}")
    assert targets <= set(ALLOWED)


def test_the_guard_catches_a_plain_store(tmp_path, monkeypatch):
    """A plain store to the chain scratch (here the Y^T v result x) planted in
    a copy of the source is reported."""
    import sys

    import pytest
    text = open(SRC).read()
    bad = text.replace("st_dev(&S.x[l0 + r * cx.nw], acc[r]);", "S.x[l0 + r * cx.nw] = acc[r];", 1)
    assert bad != text
    f = tmp_path / "te_kernels.hip"
    f.write_text(bad)
    monkeypatch.setattr(sys.modules[__name__], "SRC", str(f))
    with pytest.raises(AssertionError, match=r"S\.x"):
        test_shared_chain_data_is_stored_with_st_dev()
