"""ctypes wrapper around the CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here.

The oracle follows Ishigami, Kimura and Nakamura, arXiv:1209.1910: Sturm
bisection for the eigenvalues (the experiments of section 5.1 take them from
bisection), Peters-Wilkinson clustering (section 2.1), inverse iteration
(Eq. (1), Alg. 1 and Alg. 4) with re-orthogonalization by the new compact-WY
implementation (section 3.3.2), the ordinary one (section 3.3.1), Householder
(Alg. 2) or modified Gram-Schmidt (Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CWY_NEW, CWY_ORDINARY, HOUSEHOLDER, MGS = 0, 1, 2, 3
# per-vector status bits of eigvecs(..., with_status=True)
ST_NONFINITE, ST_BREAKDOWN, ST_PIVOT, ST_NOCONV = 1, 2, 4, 8
# iters = STOP_GROWTH selects the growth stop rule instead of a fixed count
STOP_GROWTH = -1
DEFAULT_SEED = 0x1209_1910

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("norm1", ctypes.c_double), ("tol", ctypes.c_double),
                ("pivmin", ctypes.c_double), ("pivthr", ctypes.c_double),
                ("gl", ctypes.c_double), ("gu", ctypes.c_double),
                ("tnorm", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.or_setup.argtypes = [ctypes.c_int, _dp, _dp, ctypes.POINTER(_Params)]
        L.or_sturm_count.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double]
        L.or_sturm_count.restype = ctypes.c_int
        L.or_bisect.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.or_clusters.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _ip, _ip]
        L.or_clusters.restype = ctypes.c_int
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_start_vector.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, _dp]
        L.or_lu.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                            _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_ubyte)]
        L.or_lu.restype = ctypes.c_int
        L.or_lu_solve.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp,
                                  ctypes.POINTER(ctypes.c_ubyte), _dp, _dp]
        L.or_orthogonalize.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp,
                                       ctypes.c_int, _dp, _dp, ctypes.c_int, _ip]
        L.or_eigvecs.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _dp, _dp,
                                 ctypes.c_int, _ip]
        L.or_eigvecs.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Params:
    norm1: float
    tol: float
    pivmin: float
    pivthr: float
    gl: float
    gu: float
    tnorm: float


def setup(d, e) -> Params:
    d, e = _f64(d), _f64(e)
    p = _Params()
    rc = lib().or_setup(len(d), _p(d), _p(e) if len(e) else _p(np.zeros(1)), ctypes.byref(p))
    if rc:
        raise ValueError(f"or_setup failed: {rc}")
    return Params(p.norm1, p.tol, p.pivmin, p.pivthr, p.gl, p.gu, p.tnorm)


def sturm_count(d, e, sigma: float, pivmin: float | None = None) -> int:
    d, e = _f64(d), _f64(e)
    e2 = _f64(e * e) if len(e) else np.zeros(1)
    if pivmin is None:
        pivmin = setup(d, e).pivmin
    return int(lib().or_sturm_count(len(d), _p(d), _p(e2), float(pivmin), float(sigma)))


def bisect(d, e, il: int = 1, iu: int | None = None) -> np.ndarray:
    d, e = _f64(d), _f64(e)
    n = len(d)
    iu = n if iu is None else iu
    W = np.empty(iu - il + 1)
    rc = lib().or_bisect(n, _p(d), _p(e) if len(e) else _p(np.zeros(1)), il, iu, _p(W))
    if rc:
        raise ValueError(f"or_bisect failed: {rc}")
    return W


def clusters(W, tol: float):
    W = _f64(W)
    m = len(W)
    st = np.zeros(max(m, 1), dtype=np.int32)
    sz = np.zeros(max(m, 1), dtype=np.int32)
    ncl = lib().or_clusters(m, _p(W), float(tol), st.ctypes.data_as(_ip), sz.ctypes.data_as(_ip))
    return st[:ncl].copy(), sz[:ncl].copy()


def splitmix64(seed: int, index: int) -> int:
    return int(lib().or_splitmix64(seed & (2**64 - 1), index & (2**64 - 1)))


def start_vector(seed: int, kglob: int, n: int) -> np.ndarray:
    v = np.empty(n)
    lib().or_start_vector(seed & (2**64 - 1), kglob, n, _p(v))
    return v


def lu(d, e, sigma: float, pivthr: float, with_count: bool = False):
    """Factors (u1, u2, u3, l, swap) of T - sigma I; with_count also returns
    how many pivots were replaced by +-pivthr."""
    d, e = _f64(d), _f64(e)
    n = len(d)
    u1, u2, u3, l = (np.empty(n) for _ in range(4))
    swp = np.empty(n, dtype=np.uint8)
    cnt = lib().or_lu(n, _p(d), _p(e) if len(e) else _p(np.zeros(1)), float(sigma),
                      float(pivthr), _p(u1), _p(u2), _p(u3), _p(l),
                      swp.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    f = (u1, u2, u3, l, swp)
    return (f, int(cnt)) if with_count else f


def lu_solve(factors, b) -> np.ndarray:
    u1, u2, u3, l, swp = factors
    x = _f64(b).copy()
    y = np.empty_like(x)
    lib().or_lu_solve(len(x), _p(u1), _p(u2), _p(u3), _p(l),
                      swp.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _p(x), _p(y))
    return x


def orthogonalize(V, variant: int = CWY_NEW, with_breakdown: bool = False):
    """Incremental orthogonalization of the columns of V; returns (Q, Y, T),
    and with with_breakdown the per-column reflector breakdown flags."""
    V = np.asfortranarray(V, dtype=np.float64)
    n, m = V.shape
    Q = np.zeros((n, m), order="F")
    Y = np.zeros((n, m), order="F")
    T = np.zeros((m, m), order="F")
    brk = np.zeros(m, dtype=np.int32)
    rc = lib().or_orthogonalize(n, m, _p(V), n, _p(Q), n, _p(Y), _p(T), variant,
                                brk.ctypes.data_as(_ip))
    if rc:
        raise ValueError(f"or_orthogonalize failed: {rc}")
    return (Q, Y, T, brk) if with_breakdown else (Q, Y, T)


def eigvecs(d, e, il: int = 1, iu: int | None = None, W=None, orth: int = CWY_NEW,
            iters: int = 3, seed: int = DEFAULT_SEED, with_status: bool = False):
    """Eigenvectors by inverse iteration; returns (W, Z, nclusters), and with
    with_status the per-vector ST_* bits.

    With ``W`` given (ascending) the eigenvalues are taken as input and
    ``il`` is the base of the start-vector key (eigenvalue j uses il + j).
    """
    d, e = _f64(d), _f64(e)
    n = len(d)
    if W is None:
        iu = n if iu is None else iu
        win = None
    else:
        win = _f64(W)
        iu = il + len(win) - 1
    m = iu - il + 1
    Wout = np.empty(m)
    Z = np.zeros((n, m), order="F")
    st = np.zeros(m, dtype=np.int32)
    ncl = lib().or_eigvecs(n, _p(d), _p(e) if len(e) else _p(np.zeros(1)), il, iu,
                           _p(win) if win is not None else None, orth, iters,
                           seed & (2**64 - 1), _p(Wout), _p(Z), n, st.ctypes.data_as(_ip))
    if ncl < 0:
        raise ValueError(f"or_eigvecs failed: {ncl}")
    return (Wout, Z, ncl, st) if with_status else (Wout, Z, ncl)


def split_points(d, e) -> np.ndarray:
    """Block starts of the split matrix (block b is rows bs[b]..bs[b+1]-1)."""
    d, e = _f64(d), _f64(e)
    n = len(d)
    L = lib()
    L.or_split_points.argtypes = [ctypes.c_int, _dp, _dp, _ip]
    L.or_split_points.restype = ctypes.c_int
    bs = np.zeros(n + 1, dtype=np.int32)
    nb = L.or_split_points(n, _p(d), _p(e) if len(e) else _p(np.zeros(1)), bs.ctypes.data_as(_ip))
    return bs[:nb + 1].copy()


def eigvecs_split(d, e, il: int = 1, iu: int | None = None, orth: int = CWY_NEW,
                  iters: int = 3, seed: int = DEFAULT_SEED):
    """Eigenpairs il..iu of the matrix split into unreduced blocks; returns
    (W, Z, nblocks, status, block of each column)."""
    d, e = _f64(d), _f64(e)
    n = len(d)
    iu = n if iu is None else iu
    m = iu - il + 1
    L = lib()
    L.or_eigvecs_split.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _dp, _dp,
                                   ctypes.c_int, _ip, _ip]
    L.or_eigvecs_split.restype = ctypes.c_int
    W = np.empty(m)
    Z = np.zeros((n, m), order="F")
    st = np.zeros(m, dtype=np.int32)
    blk = np.zeros(m, dtype=np.int32)
    nb = L.or_eigvecs_split(n, _p(d), _p(e) if len(e) else _p(np.zeros(1)), il, iu, orth, iters,
                            seed & (2**64 - 1), _p(W), _p(Z), n, st.ctypes.data_as(_ip),
                            blk.ctypes.data_as(_ip))
    if nb < 0:
        raise ValueError(f"or_eigvecs_split failed: {nb}")
    return W, Z, nb, st, blk


def bidiag_svd(a, b, il: int = 1, iu: int | None = None, orth: int = CWY_NEW, iters: int = 3,
               seed: int = DEFAULT_SEED):
    """Singular values (ascending) il..iu of the upper bidiagonal matrix with
    diagonal a and superdiagonal b, and their left (U) and right (V) singular
    vectors as columns; returns (S, U, V, status)."""
    a, b = _f64(a), _f64(b)
    n = len(a)
    iu = n if iu is None else iu
    m = iu - il + 1
    L = lib()
    L.or_bidiag_svd.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _dp, _dp,
                                ctypes.c_int, _dp, ctypes.c_int, _ip]
    L.or_bidiag_svd.restype = ctypes.c_int
    S = np.empty(m)
    U = np.zeros((n, m), order="F")
    V = np.zeros((n, m), order="F")
    st = np.zeros(m, dtype=np.int32)
    rc = L.or_bidiag_svd(n, _p(a), _p(b) if len(b) else _p(np.zeros(1)), il, iu, orth, iters,
                         seed & (2**64 - 1), _p(S), _p(U), n, _p(V), n, st.ctypes.data_as(_ip))
    if rc < 0:
        raise ValueError(f"or_bidiag_svd failed: {rc}")
    return S, U, V, st
