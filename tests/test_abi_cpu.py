"""CPU checks of the C-ABI library: it loads, exports every entry point the
public header declares, and rejects invalid arguments on the host (these
calls return before any HIP runtime call, so no GPU is needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1209_1910_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tridiag_eigvecs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|size_t|void|te_server|te_batch_graph)\s+\**\s*(\w+)\s*\(", src,
                       flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = _declared()
    assert len(names) >= 8
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(binding.SYMBOLS)


NULL = ctypes.c_void_p(0)
P = ctypes.c_void_p(256)   # never dereferenced: validation fails first


@pytest.mark.parametrize("args,expect", [
    ((NULL, P, 10, 1, 10, P, P, 10, NULL), -1),
    ((P, NULL, 10, 1, 10, P, P, 10, NULL), -2),
    ((P, P, 0, 1, 1, P, P, 10, NULL), -3),
    ((P, P, 10, 0, 10, P, P, 10, NULL), -4),
    ((P, P, 10, 5, 4, P, P, 10, NULL), -5),
    ((P, P, 10, 1, 11, P, P, 10, NULL), -5),
    ((P, P, 10, 1, 10, NULL, P, 10, NULL), -6),
    ((P, P, 10, 1, 10, P, NULL, 10, NULL), -7),
    ((P, P, 10, 1, 10, P, P, 9, NULL), -8),
])
def test_tridiag_eigvecs_argument_errors(args, expect):
    assert binding.lib().tridiag_eigvecs(*args) == expect


def test_other_entry_points_argument_errors():
    L = binding.lib()
    assert L.tridiag_eigvecs_given_w(P, P, 10, 11, P, P, 10, NULL) == -4
    assert L.tridiag_eigvecs_given_w(P, P, 10, 3, NULL, P, 10, NULL) == -5
    assert L.tridiag_eigvecs_given_w(P, P, 10, 3, P, P, 5, NULL) == -7
    assert L.tridiag_eigvals(P, P, 10, 3, 2, P, NULL) == -5
    assert L.tridiag_clusters(P, 0, 1.0, P, P, P, NULL) == -2
    assert L.tridiag_clusters(P, 4, -1.0, P, P, P, NULL) == -3
    assert L.tridiag_eigvecs_workspace_bytes(10, 4, 3) == 0
    assert L.tridiag_eigvecs_workspace_bytes(0, 1, 1) == 0
    o = binding.te_opts()
    o.iters = -1
    assert L.tridiag_eigvecs_ex(P, P, 10, 1, 10, NULL, P, P, 10, ctypes.byref(o), P, 1 << 40,
                                NULL, NULL) == -10
    o.iters = 3
    assert L.tridiag_eigvecs_ex(P, P, 10, 1, 10, NULL, P, P, 10, ctypes.byref(o), NULL, 1 << 40,
                                NULL, NULL) == -11
    assert L.tridiag_eigvecs_noalloc(NULL, P, 10, 1, 10, NULL, P, P, 10, None, NULL, NULL) == -1
    assert L.tridiag_eigvecs_noalloc(P, P, 10, 1, 11, NULL, P, P, 10, None, NULL, NULL) == -5
    assert L.tridiag_eigvecs_noalloc(P, P, 10, 1, 10, NULL, NULL, P, 10, None, NULL, NULL) == -7
    assert L.tridiag_eigvecs_noalloc(P, P, 10, 1, 10, NULL, P, P, 9, None, NULL, NULL) == -9
    o.iters = -1
    assert L.tridiag_eigvecs_noalloc(P, P, 10, 1, 10, NULL, P, P, 10, ctypes.byref(o), NULL,
                                     NULL) == -10
    assert L.tridiag_eigvecs_noalloc_bytes(10, 4, 3) == 0
    assert L.bidiag_svd(NULL, P, 10, 1, 10, P, P, 10, P, 10, None, NULL, NULL) == -1
    assert L.bidiag_svd(P, P, 10, 1, 11, P, P, 10, P, 10, None, NULL, NULL) == -5
    assert L.bidiag_svd(P, P, 10, 1, 10, P, P, 10, P, 9, None, NULL, NULL) == -10
    assert L.tridiag_eigvecs_split(NULL, P, 10, 1, 10, P, P, 10, None, NULL, None, NULL) == -1
    assert L.tridiag_eigvecs_split(P, P, 10, 2, 1, P, P, 10, None, NULL, None, NULL) == -5
    assert L.tridiag_eigvecs_split(P, P, 10, 1, 10, P, P, 9, None, NULL, None, NULL) == -8
    assert L.tridiag_eigvecs_split(P, P, 10, 1, 10, P, P, 10, ctypes.byref(o), NULL, None,
                                   NULL) == -9


def test_server_argument_errors():
    L = binding.lib()
    rid = ctypes.c_int64(0)
    i64 = ctypes.byref(rid)
    # server handle checked first; then the request arguments in order
    assert L.te_server_submit(NULL, P, P, 10, 1, 10, P, P, 10, i64) == -1
    assert L.te_server_submit(P, NULL, P, 10, 1, 10, P, P, 10, i64) == -2
    assert L.te_server_submit(P, P, NULL, 10, 1, 10, P, P, 10, i64) == -3
    assert L.te_server_submit(P, P, P, 0, 1, 1, P, P, 10, i64) == -4
    assert L.te_server_submit(P, P, P, 10, 0, 10, P, P, 10, i64) == -5
    assert L.te_server_submit(P, P, P, 10, 3, 2, P, P, 10, i64) == -6
    assert L.te_server_submit(P, P, P, 10, 1, 10, NULL, P, 10, i64) == -7
    assert L.te_server_submit(P, P, P, 10, 1, 10, P, NULL, 10, i64) == -8
    assert L.te_server_submit(P, P, P, 10, 1, 10, P, P, 9, i64) == -9
    assert L.te_server_submit(P, P, P, 10, 1, 10, P, P, 10, None) == -10
    assert L.te_server_poll(NULL, 1, None) == -1
    assert L.te_server_wait(NULL, 1, None) == -1
    assert L.te_server_times(NULL, 1, None, None, None) == -1
    assert L.te_server_release(NULL, 1) == -1
    assert not L.te_server_create(0, -1, None)
    assert not L.te_server_create(0, 65, None)
    o = binding.te_opts()
    o.coop_wgs = -2
    assert not L.te_server_create(0, 1, ctypes.byref(o))
    L.te_server_destroy(NULL)


def test_batch_graph_and_autotune_argument_errors():
    """The graph path checks the batched arguments on the host, in the
    positions of tridiag_eigvecs_batched, before any HIP call; a forced chain
    configuration is checked next (argument 12)."""
    import numpy as np
    L = binding.lib()
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    off = np.array([0, 10, 16], dtype=np.int64)
    il = np.array([1, 1], dtype=np.int32)
    iu = np.array([10, 6], dtype=np.int32)
    woff = np.array([0, 10], dtype=np.int64)
    zoff = np.array([0, 100], dtype=np.int64)
    A = (off.ctypes.data_as(i64p), il.ctypes.data_as(ip), iu.ctypes.data_as(ip))
    W = woff.ctypes.data_as(i64p)
    Zo = zoff.ctypes.data_as(i64p)
    rc = ctypes.c_int(0)
    g = L.te_batch_graph_create(NULL, P, *A, P, W, P, Zo, 2, None, None, ctypes.byref(rc))
    assert not g and rc.value == -1
    g = L.te_batch_graph_create(P, P, *A, P, W, P, Zo, 0, None, None, ctypes.byref(rc))
    assert not g and rc.value == -10
    bad_iu = np.array([11, 6], dtype=np.int32)
    g = L.te_batch_graph_create(P, P, off.ctypes.data_as(i64p), il.ctypes.data_as(ip),
                                bad_iu.ctypes.data_as(ip), P, W, P, Zo, 2, None, None,
                                ctypes.byref(rc))
    assert not g and rc.value == -5
    o = binding.te_opts()
    o.iters = -1
    g = L.te_batch_graph_create(P, P, *A, P, W, P, Zo, 2, ctypes.byref(o), None, ctypes.byref(rc))
    assert not g and rc.value == -11
    assert L.te_batch_autotune(P, P, *A, NULL, W, P, Zo, 2, None, None, None, None, 0,
                               None) == -6
    assert L.te_batch_autotune(P, P, *A, P, W, P, None, 2, None, None, None, None, 0,
                               None) == -9
    assert L.te_batch_graph_launch(NULL, NULL) == -1
    assert L.te_batch_graph_info(NULL, None, None, None) == -1
    L.te_batch_graph_destroy(NULL)


def test_stop_option_is_checked_on_the_host():
    L = binding.lib()
    o = binding.te_opts()
    o.stop = 7
    assert L.tridiag_eigvecs_ex(P, P, 10, 1, 10, NULL, P, P, 10, ctypes.byref(o), P, 1 << 40,
                                NULL, NULL) == -10
    assert not L.te_server_create(0, 1, ctypes.byref(o))


def test_orth_option_is_checked_on_the_host():
    """te_opts.orth other than TE_ORTH_CWY / TE_ORTH_MGS is an invalid options
    argument (position 10 of tridiag_eigvecs_ex, 11 of the batched call)."""
    import numpy as np
    L = binding.lib()
    o = binding.te_opts()
    o.orth = 7
    assert L.tridiag_eigvecs_ex(P, P, 10, 1, 10, NULL, P, P, 10, ctypes.byref(o), P, 1 << 40,
                                NULL, NULL) == -10
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    off = np.array([0, 10], dtype=np.int64)
    il = np.array([1], dtype=np.int32)
    iu = np.array([10], dtype=np.int32)
    z = np.array([0], dtype=np.int64)
    assert L.tridiag_eigvecs_batched(P, P, off.ctypes.data_as(i64p), il.ctypes.data_as(ip),
                                     iu.ctypes.data_as(ip), P, z.ctypes.data_as(i64p), P,
                                     z.ctypes.data_as(i64p), 1, ctypes.byref(o), NULL) == -11
    o.orth = binding.TE_ORTH_MGS
    assert binding._opts(orth="mgs").orth == binding.TE_ORTH_MGS
    assert binding._opts().orth == binding.TE_ORTH_CWY


def test_graph_path_mgs_checks_on_the_host():
    """The graph path takes MGS options for problems of order up to
    TE_MGS_MAX_N (the call then goes on to the device: TE_ERR_NO_DEVICE
    here); a larger problem fails with TE_ERR_UNSUPPORTED, and the autotuner,
    which tunes the compact-WY chain only, rejects MGS options; all before
    any HIP call."""
    import numpy as np
    L = binding.lib()
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    z = np.array([0], dtype=np.int64)
    il = np.array([1], dtype=np.int32)
    o = binding.te_opts()
    o.orth = binding.TE_ORTH_MGS
    rc = ctypes.c_int(0)
    for n, expect in ((10, binding.TE_ERR_NO_DEVICE),
                      (binding.TE_MGS_MAX_N + 1, binding.TE_ERR_UNSUPPORTED)):
        off = np.array([0, n], dtype=np.int64)
        iu = np.array([n], dtype=np.int32)
        A = (off.ctypes.data_as(i64p), il.ctypes.data_as(ip), iu.ctypes.data_as(ip), P,
             z.ctypes.data_as(i64p), P, z.ctypes.data_as(i64p), 1)
        g = L.te_batch_graph_create(P, P, *A, ctypes.byref(o), None, ctypes.byref(rc))
        assert not g and rc.value == expect, (n, rc.value)
        assert L.te_batch_autotune(P, P, *A, ctypes.byref(o), None, None, None, 0,
                                   None) == binding.TE_ERR_UNSUPPORTED


def test_batched_ex_argument_errors():
    """tridiag_eigvecs_batched_ex checks arguments 1-11 as the batched call
    does, then info_all (12) and ioff (13): null, negative or overlapping
    status regions are rejected on the host."""
    import numpy as np
    L = binding.lib()
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    off = np.array([0, 10, 16], dtype=np.int64)
    il = np.array([1, 2], dtype=np.int32)
    iu = np.array([10, 6], dtype=np.int32)
    woff = np.array([0, 10], dtype=np.int64)
    zoff = np.array([0, 100], dtype=np.int64)
    A = (off.ctypes.data_as(i64p), il.ctypes.data_as(ip), iu.ctypes.data_as(ip), P,
         woff.ctypes.data_as(i64p), P, zoff.ctypes.data_as(i64p), 2)

    def call(*tail, d=P):
        return L.tridiag_eigvecs_batched_ex(d, P, *A, None, *tail, NULL)

    assert call(P, np.array([0, 11], dtype=np.int64).ctypes.data_as(i64p), d=NULL) == -1
    assert call(NULL, np.array([0, 11], dtype=np.int64).ctypes.data_as(i64p)) == -12
    assert call(P, None) == -13
    assert call(P, np.array([0, -1], dtype=np.int64).ctypes.data_as(i64p)) == -13
    # problem 0 needs 11 ints [0, 11): a region starting at 10 overlaps it
    assert call(P, np.array([0, 10], dtype=np.int64).ctypes.data_as(i64p)) == -13
    # problem 1 needs 6 ints [0, 6): problem 0 at 5 overlaps it, at 6 it does not
    assert call(P, np.array([5, 0], dtype=np.int64).ctypes.data_as(i64p)) == -13
    assert call(P, np.array([6, 0], dtype=np.int64).ctypes.data_as(i64p)) == binding.TE_ERR_NO_DEVICE


def test_binding_constants_match_the_header():
    """Every integer #define of the public header has the same value in the
    Python binding."""
    src = open(HEADER).read()
    found = 0
    for name, val in re.findall(r"^#define\s+(TE_\w+)\s+(.+?)(?:\s*/\*.*)?$", src, flags=re.M):
        v = val.strip()
        m = re.fullmatch(r"\(?(-?(?:0x[0-9A-Fa-f]+|\d+))(?:ULL)?\)?", v)
        if m:
            expect = int(m.group(1), 0)
        else:
            m = re.fullmatch(r"\(\(size_t\)(\d+)\s*<<\s*(\d+)\)", v)
            assert m, (name, v)
            expect = int(m.group(1)) << int(m.group(2))
        assert getattr(binding, name) == expect, name
        found += 1
    assert found >= 17
