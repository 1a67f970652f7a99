"""ctypes binding of the HIP C-ABI library (argument marshalling only).

Every function here forwards to the entry point of the same name in
``libtridiag_eigvecs.so``; PyTorch provides device memory and the stream.
There is no fallback: if the library is not built, or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtridiag_eigvecs.so")

TE_DEFAULT_SEED = 0x12091910
TE_DEFAULT_ITERS = 3
TE_ORTH_CWY, TE_ORTH_MGS = 0, 1        # te_opts.orth: compact WY (Alg. 4) or MGS (Alg. 1)
TE_MGS_MAX_N = 8192
TE_ERR_HIP, TE_ERR_NO_DEVICE, TE_ERR_WORKSPACE, TE_ERR_KERNEL = -1000, -1001, -1002, -1003
TE_ERR_UNSUPPORTED = -1004
TE_INFO_NONFINITE, TE_INFO_BREAKDOWN, TE_INFO_PIVOT, TE_INFO_NOCONV = 1, 2, 4, 8  # info bits
TE_STOP_FIXED, TE_STOP_GROWTH = 0, 1    # te_opts.stop
SYMBOLS = ("tridiag_eigvecs", "tridiag_eigvecs_given_w", "tridiag_eigvecs_workspace_bytes",
           "tridiag_eigvecs_ex", "tridiag_eigvecs_batched", "tridiag_eigvals", "tridiag_clusters",
           "te_server_create", "te_server_submit", "te_server_poll", "te_server_wait",
           "te_server_times", "te_server_destroy", "te_server_release",
           "te_batch_graph_create", "te_batch_graph_launch", "te_batch_graph_info",
           "te_batch_graph_destroy", "te_batch_autotune",
           "te_timing_enable", "te_timing_reset", "te_timing_read", "te_last_hip_error",
           "tridiag_eigvecs_noalloc", "tridiag_eigvecs_noalloc_bytes", "tridiag_eigvecs_split", "bidiag_svd",
           "tridiag_eigvecs_batched_ex")
PHASES = ("setup", "bisect", "clusters", "first_solves", "transpose", "chain_small",
          "chain_coop", "finalize")


class TeError(RuntimeError):
    def __init__(self, fn, rc, hip=0):
        super().__init__(f"{fn} returned {rc}" + (f" (hip error {hip})" if hip else ""))
        self.rc = rc
        self.hip = hip


class te_opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("orth", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("cluster_rtol", ctypes.c_double),
                ("coop_wgs", ctypes.c_int), ("stop", ctypes.c_int),
                ("ws_budget", ctypes.c_uint64)]


class te_graph_cfg(ctypes.Structure):
    _fields_ = [("chain_threads", ctypes.c_int), ("chains_per_cu", ctypes.c_int)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        i, sz, i64p = ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        L.tridiag_eigvecs.argtypes = [_vp, _vp, i, i, i, _vp, _vp, i, _vp]
        L.tridiag_eigvecs_given_w.argtypes = [_vp, _vp, i, i, _vp, _vp, i, _vp]
        L.tridiag_eigvecs_workspace_bytes.argtypes = [i, i, i]
        L.tridiag_eigvecs_workspace_bytes.restype = sz
        L.tridiag_eigvecs_ex.argtypes = [_vp, _vp, i, i, i, _vp, _vp, _vp, i,
                                         ctypes.POINTER(te_opts), _vp, sz, _vp, _vp]
        L.tridiag_eigvecs_noalloc.argtypes = [_vp, _vp, i, i, i, _vp, _vp, _vp, i,
                                              ctypes.POINTER(te_opts), _vp, _vp]
        L.tridiag_eigvecs_split.argtypes = [_vp, _vp, i, i, i, _vp, _vp, i,
                                            ctypes.POINTER(te_opts), _vp, ip, _vp]
        L.bidiag_svd.argtypes = [_vp, _vp, i, i, i, _vp, _vp, i, _vp, i, ctypes.POINTER(te_opts),
                                 _vp, _vp]
        L.tridiag_eigvecs_noalloc_bytes.argtypes = [i, i, i]
        L.tridiag_eigvecs_noalloc_bytes.restype = sz
        L.tridiag_eigvecs_batched.argtypes = [_vp, _vp, i64p, ip, ip, _vp, i64p, _vp, i64p, i,
                                              ctypes.POINTER(te_opts), _vp]
        L.tridiag_eigvecs_batched_ex.argtypes = [_vp, _vp, i64p, ip, ip, _vp, i64p, _vp, i64p,
                                                 i, ctypes.POINTER(te_opts), _vp, i64p, _vp]
        L.tridiag_eigvals.argtypes = [_vp, _vp, i, i, i, _vp, _vp]
        L.tridiag_clusters.argtypes = [_vp, i, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.te_server_create.argtypes = [ctypes.c_uint64, i, ctypes.POINTER(te_opts)]
        L.te_server_create.restype = _vp
        L.te_server_submit.argtypes = [_vp, _vp, _vp, i, i, i, _vp, _vp, i, i64p]
        L.te_server_poll.argtypes = [_vp, ctypes.c_int64, ip]
        L.te_server_wait.argtypes = [_vp, ctypes.c_int64, ip]
        dp = ctypes.POINTER(ctypes.c_double)
        L.te_server_times.argtypes = [_vp, ctypes.c_int64, dp, dp, dp]
        L.te_server_release.argtypes = [_vp, ctypes.c_int64]
        L.te_server_destroy.argtypes = [_vp]
        L.te_server_destroy.restype = None
        L.te_timing_enable.argtypes = [i]
        L.te_timing_enable.restype = None
        L.te_timing_reset.restype = None
        L.te_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_longlong), i]
        L.te_last_hip_error.restype = i
        cfgp = ctypes.POINTER(te_graph_cfg)
        batch = [_vp, _vp, i64p, ip, ip, _vp, i64p, _vp, i64p, i, ctypes.POINTER(te_opts)]
        L.te_batch_graph_create.argtypes = batch + [cfgp, ip]
        L.te_batch_graph_create.restype = _vp
        L.te_batch_graph_launch.argtypes = [_vp, _vp]
        L.te_batch_graph_info.argtypes = [_vp, cfgp, ip, ctypes.POINTER(ctypes.c_uint64)]
        L.te_batch_graph_destroy.argtypes = [_vp]
        L.te_batch_graph_destroy.restype = None
        L.te_batch_autotune.argtypes = batch + [cfgp, cfgp, ctypes.POINTER(ctypes.c_double), i,
                                                ip]
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(x, device):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    x = x.to(device=device, dtype=torch.float64).contiguous()
    return x


def _host_f64(x):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        return x.detach().to("cpu", torch.float64).numpy()
    return np.asarray(x, dtype=np.float64)


def _check(fn, rc):
    if rc != 0:
        raise TeError(fn, rc, lib().te_last_hip_error())


def _opts(iters=None, seed=None, cluster_rtol=None, coop_wgs=None, ws_budget=None, orth=None,
          stop=None):
    o = te_opts()
    o.iters = int(iters or 0)
    o.stop = {None: TE_STOP_FIXED, "fixed": TE_STOP_FIXED, "growth": TE_STOP_GROWTH}.get(stop, stop)
    o.orth = {None: TE_ORTH_CWY, "cwy": TE_ORTH_CWY, "mgs": TE_ORTH_MGS}.get(orth, orth)
    o.seed = int(seed or 0)
    o.cluster_rtol = float(cluster_rtol or 0.0)
    o.coop_wgs = int(coop_wgs or 0)
    o.ws_budget = int(ws_budget or 0)
    return o


def tridiag_eigvecs(d, e, il=1, iu=None, stream=None, device="cuda"):
    """Eigenpairs il..iu (1-based, inclusive) of tridiag(e, d, e).

    Returns (W, Z): float64 device tensors, W of shape (m,), Z of shape (m, n)
    whose row j is the eigenvector of W[j] (column j of the column-major
    n x m result the library writes).
    """
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    n = d.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    W = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    Z = torch.empty((max(m, 1), n), dtype=torch.float64, device=d.device)
    rc = lib().tridiag_eigvecs(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0), n, il, iu,
                               _vp(W.data_ptr()), _vp(Z.data_ptr()), n, _stream_ptr(stream))
    _check("tridiag_eigvecs", rc)
    return W[:m], Z[:m]


def tridiag_eigvecs_given_w(d, e, W, stream=None, device="cuda"):
    """Eigenvectors for given ascending eigenvalue approximations W (m,).
    Returns Z of shape (m, n) (row j = eigenvector of W[j])."""
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    W = _dev_f64(W, device)
    n, m = d.numel(), W.numel()
    Z = torch.empty((m, n), dtype=torch.float64, device=d.device)
    rc = lib().tridiag_eigvecs_given_w(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0), n,
                                       m, _vp(W.data_ptr()), _vp(Z.data_ptr()), n,
                                       _stream_ptr(stream))
    _check("tridiag_eigvecs_given_w", rc)
    return Z


def tridiag_eigvals(d, e, il=1, iu=None, stream=None, device="cuda"):
    """Eigenvalues il..iu by Sturm bisection; returns a float64 device tensor."""
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    n = d.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    W = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    rc = lib().tridiag_eigvals(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0), n, il, iu,
                               _vp(W.data_ptr()), _stream_ptr(stream))
    _check("tridiag_eigvals", rc)
    return W[:m]


def tridiag_clusters(W, tol, stream=None, device="cuda"):
    """Cluster starts and sizes of ascending W under the gap rule; returns
    (start, size) int32 device tensors of length ncl."""
    torch = _torch()
    W = _dev_f64(W, device)
    m = W.numel()
    start = torch.empty(max(m, 1), dtype=torch.int32, device=W.device)
    size = torch.empty(max(m, 1), dtype=torch.int32, device=W.device)
    ncl = torch.zeros(1, dtype=torch.int32, device=W.device)
    rc = lib().tridiag_clusters(_vp(W.data_ptr()), m, float(tol), _vp(start.data_ptr()),
                                _vp(size.data_ptr()), _vp(ncl.data_ptr()), _stream_ptr(stream))
    _check("tridiag_clusters", rc)
    k = int(ncl.item())
    return start[:k], size[:k]


def te_timing_enable(on=True):
    lib().te_timing_enable(1 if on else 0)


def te_timing_reset():
    lib().te_timing_reset()


def te_timing_read():
    """Per-phase device milliseconds and launch counts since the last reset."""
    ms = (ctypes.c_double * 8)()
    cnt = (ctypes.c_longlong * 8)()
    k = lib().te_timing_read(ms, cnt, 8)
    return {PHASES[p]: (ms[p], cnt[p]) for p in range(min(k, 8))}


def tridiag_eigvecs_workspace_bytes(n, il, iu):
    return int(lib().tridiag_eigvecs_workspace_bytes(n, il, iu))


def tridiag_eigvecs_ex(d, e, il=1, iu=None, W_given=None, ws=None, info=None, stream=None,
                       device="cuda", **opts):
    """_ex entry point.  ws: uint8 device tensor (allocated here if None).
    Returns (W, Z, info)."""
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    n = d.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    W = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    Z = torch.empty((max(m, 1), n), dtype=torch.float64, device=d.device)
    wg = _dev_f64(W_given, device) if W_given is not None else None
    need = tridiag_eigvecs_workspace_bytes(n, il, iu)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=d.device)
    base = ws.data_ptr()
    pad = (-base) % 256
    if info is None:
        info = torch.zeros(m + 1, dtype=torch.int32, device=d.device)
    o = _opts(**opts)
    rc = lib().tridiag_eigvecs_ex(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0), n, il,
                                  iu, _vp(wg.data_ptr() if wg is not None else 0),
                                  _vp(W.data_ptr()), _vp(Z.data_ptr()), n, ctypes.byref(o),
                                  _vp(base + pad), ws.numel() - pad, _vp(info.data_ptr()),
                                  _stream_ptr(stream))
    _check("tridiag_eigvecs_ex", rc)
    return W[:m], Z[:m], info


def tridiag_eigvecs_split(d, e, il=1, iu=None, stream=None, device="cuda", **opts):
    """Eigenpairs il..iu of tridiag(e, d, e) split into unreduced blocks.
    Returns (W, Z, info, nblocks); row j of Z is the vector of W[j]."""
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    n = d.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    W = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    Z = torch.empty((max(m, 1), n), dtype=torch.float64, device=d.device)
    info = torch.zeros(m + 1, dtype=torch.int32, device=d.device)
    nb = ctypes.c_int(0)
    o = _opts(**opts)
    rc = lib().tridiag_eigvecs_split(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0), n,
                                     il, iu, _vp(W.data_ptr()), _vp(Z.data_ptr()), n,
                                     ctypes.byref(o), _vp(info.data_ptr()), ctypes.byref(nb),
                                     _stream_ptr(stream))
    _check("tridiag_eigvecs_split", rc)
    return W[:m], Z[:m], info, nb.value


def bidiag_svd(a, b, il=1, iu=None, stream=None, device="cuda", **opts):
    """Singular values (ascending) il..iu of the upper bidiagonal matrix with
    diagonal a and superdiagonal b, with left and right singular vectors.
    Returns (S, U, V, info): row j of U and of V is the pair of S[j]."""
    torch = _torch()
    a = _dev_f64(a, device)
    b = _dev_f64(b, device)
    n = a.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    S = torch.empty(max(m, 1), dtype=torch.float64, device=a.device)
    U = torch.empty((max(m, 1), n), dtype=torch.float64, device=a.device)
    V = torch.empty((max(m, 1), n), dtype=torch.float64, device=a.device)
    info = torch.zeros(m + 1, dtype=torch.int32, device=a.device)
    o = _opts(**opts)
    rc = lib().bidiag_svd(_vp(a.data_ptr()), _vp(b.data_ptr() if b.numel() else 0), n, il, iu,
                          _vp(S.data_ptr()), _vp(U.data_ptr()), n, _vp(V.data_ptr()), n,
                          ctypes.byref(o), _vp(info.data_ptr()), _stream_ptr(stream))
    _check("bidiag_svd", rc)
    return S[:m], U[:m], V[:m], info


TE_NOALLOC_SCRATCH_BYTES = 256 << 20


def tridiag_eigvecs_noalloc_bytes(n, il=1, iu=None):
    return int(lib().tridiag_eigvecs_noalloc_bytes(n, il, n if iu is None else iu))


def tridiag_eigvecs_noalloc(d, e, il=1, iu=None, W_given=None, W=None, Z=None, info=None,
                            stream=None, device="cuda", **opts):
    """The entry point that allocates no device memory (its workspace is the
    library's fixed per-device array).  W (m), Z (m x n, row j the vector of
    W[j]) and info (m + 1 int32) may be passed in preallocated.
    Returns (W, Z, info)."""
    torch = _torch()
    d = _dev_f64(d, device)
    e = _dev_f64(e, device)
    n = d.numel()
    iu = n if iu is None else iu
    m = iu - il + 1
    if W is None:
        W = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    if Z is None:
        Z = torch.empty((max(m, 1), n), dtype=torch.float64, device=d.device)
    if info is None:
        info = torch.zeros(m + 1, dtype=torch.int32, device=d.device)
    wg = _dev_f64(W_given, device) if W_given is not None else None
    o = _opts(**opts)
    rc = lib().tridiag_eigvecs_noalloc(_vp(d.data_ptr()), _vp(e.data_ptr() if e.numel() else 0),
                                       n, il, iu, _vp(wg.data_ptr() if wg is not None else 0),
                                       _vp(W.data_ptr()), _vp(Z.data_ptr()), n, ctypes.byref(o),
                                       _vp(info.data_ptr()), _stream_ptr(stream))
    _check("tridiag_eigvecs_noalloc", rc)
    return W[:m], Z[:m], info


class BatchLayout:
    """Problems packed as the batched entry points expect: d_all, e_all on the
    device; off, il, iu, woff, zoff on the host; W_all and Z_all device outputs."""

    def __init__(self, problems, device="cuda"):
        torch = _torch()
        B = len(problems)
        ns, ils, ius, ds, es = [], [], [], [], []
        for p in problems:
            d, e = p[0], p[1]
            n = len(d)
            il, iu = (p[2], p[3]) if len(p) >= 4 else (1, n)
            ns.append(n)
            ils.append(il)
            ius.append(iu)
            ds.append(_host_f64(d))
            es.append(_host_f64(e))
        self.B = B
        self.ns = ns
        self.off = np.zeros(B + 1, dtype=np.int64)
        self.off[1:] = np.cumsum(ns)
        self.ms = np.array([iu - il + 1 for il, iu in zip(ils, ius)], dtype=np.int64)
        self.woff = np.zeros(B, dtype=np.int64)
        self.woff[1:] = np.cumsum(self.ms)[:-1]
        zsz = self.ms * np.array(ns, dtype=np.int64)
        self.zoff = np.zeros(B, dtype=np.int64)
        self.zoff[1:] = np.cumsum(zsz)[:-1]
        self.d_all = _dev_f64(np.concatenate(ds), device)
        e_cat = (np.concatenate([x for x in es if len(x)]) if any(len(x) for x in es)
                 else np.zeros(1))
        self.e_all = _dev_f64(e_cat, device)
        self.W_all = torch.empty(int(self.ms.sum()), dtype=torch.float64, device=self.d_all.device)
        self.Z_all = torch.empty(int(zsz.sum()), dtype=torch.float64, device=self.d_all.device)
        self.il = np.asarray(ils, dtype=np.int32)
        self.iu = np.asarray(ius, dtype=np.int32)

    def args(self):
        """The first ten C-ABI arguments of the batched entry points."""
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        return (_vp(self.d_all.data_ptr()), _vp(self.e_all.data_ptr()),
                self.off.ctypes.data_as(i64p), self.il.ctypes.data_as(ip),
                self.iu.ctypes.data_as(ip), _vp(self.W_all.data_ptr()),
                self.woff.ctypes.data_as(i64p), _vp(self.Z_all.data_ptr()),
                self.zoff.ctypes.data_as(i64p), self.B)

    def results(self):
        """List of (W, Z) views per problem (Z row j = eigenvector of W[j])."""
        out = []
        for b in range(self.B):
            m, n = int(self.ms[b]), self.ns[b]
            W = self.W_all[self.woff[b]: self.woff[b] + m]
            Z = self.Z_all[self.zoff[b]: self.zoff[b] + m * n].view(m, n)
            out.append((W, Z))
        return out


def tridiag_eigvecs_batched(problems, stream=None, device="cuda", **opts):
    """problems: list of (d, e) or (d, e, il, iu) (numpy or tensors).
    Returns a list of (W, Z) per problem (Z row j = eigenvector of W[j])."""
    lay = problems if isinstance(problems, BatchLayout) else BatchLayout(problems, device)
    o = _opts(**opts)
    rc = lib().tridiag_eigvecs_batched(*lay.args(), ctypes.byref(o), _stream_ptr(stream))
    _check("tridiag_eigvecs_batched", rc)
    return lay.results()


def tridiag_eigvecs_batched_ex(problems, stream=None, device="cuda", **opts):
    """tridiag_eigvecs_batched with status words: returns a list of
    (W, Z, info) per problem, info (1 + m int32) laid out as for
    tridiag_eigvecs_ex."""
    torch = _torch()
    lay = problems if isinstance(problems, BatchLayout) else BatchLayout(problems, device)
    ioff = np.zeros(lay.B, dtype=np.int64)
    ioff[1:] = np.cumsum(lay.ms + 1)[:-1]
    info = torch.empty(int((lay.ms + 1).sum()), dtype=torch.int32, device=lay.d_all.device)
    o = _opts(**opts)
    rc = lib().tridiag_eigvecs_batched_ex(*lay.args(), ctypes.byref(o), _vp(info.data_ptr()),
                                          ioff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          _stream_ptr(stream))
    _check("tridiag_eigvecs_batched_ex", rc)
    return [(W, Z, info[ioff[b]: ioff[b] + 1 + int(lay.ms[b])])
            for b, (W, Z) in enumerate(lay.results())]


class BatchGraph:
    """Graph-captured batched path (te_batch_graph_*).  The graph binds the
    layout's device buffers: ``launch`` recomputes every problem from the
    inputs d_all, e_all hold at that time into W_all, Z_all."""

    def __init__(self, layout, chain_threads=None, chains_per_cu=None, **opts):
        self.layout = layout
        self._o = _opts(**opts)
        cfg = None
        if chain_threads is not None or chains_per_cu is not None:
            cfg = te_graph_cfg(int(chain_threads or 256), int(chains_per_cu or 1))
        rc = ctypes.c_int(0)
        h = lib().te_batch_graph_create(*layout.args(), ctypes.byref(self._o),
                                        ctypes.byref(cfg) if cfg is not None else None,
                                        ctypes.byref(rc))
        if not h:
            raise TeError("te_batch_graph_create", rc.value, lib().te_last_hip_error())
        self._h = ctypes.c_void_p(h)

    def launch(self, stream=None):
        _check("te_batch_graph_launch", lib().te_batch_graph_launch(self._h, _stream_ptr(stream)))
        return self.layout.results()

    def info(self):
        """{'chain_threads', 'chains_per_cu', 'segments', 'device_bytes'}"""
        c = te_graph_cfg()
        seg = ctypes.c_int(0)
        nb = ctypes.c_uint64(0)
        _check("te_batch_graph_info",
               lib().te_batch_graph_info(self._h, ctypes.byref(c), ctypes.byref(seg),
                                         ctypes.byref(nb)))
        return {"chain_threads": c.chain_threads, "chains_per_cu": c.chains_per_cu,
                "segments": seg.value, "device_bytes": nb.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().te_batch_graph_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_autotune(layout, **opts):
    """te_batch_autotune on a BatchLayout.  Returns (best, [(cfg, ms), ...])
    with cfg = (chain_threads, chains_per_cu)."""
    o = _opts(**opts)
    cap = 32
    best = te_graph_cfg()
    tried = (te_graph_cfg * cap)()
    ms = (ctypes.c_double * cap)()
    nt = ctypes.c_int(0)
    rc = lib().te_batch_autotune(*layout.args(), ctypes.byref(o), ctypes.byref(best), tried, ms,
                                 cap, ctypes.byref(nt))
    _check("te_batch_autotune", rc)
    res = [((tried[k].chain_threads, tried[k].chains_per_cu), ms[k])
           for k in range(min(nt.value, cap))]
    return (best.chain_threads, best.chains_per_cu), res


class Server:
    """Serving engine (te_server_*): submit host problems, collect host results.

    ``submit`` copies d and e and allocates the host outputs W (m,) and Z (m, n)
    (row j of Z is the eigenvector of W[j]); they are filled when the request
    completes.  Use as a context manager, or call ``close``.
    """

    def __init__(self, hbm_budget=0, lanes=0, iters=None, seed=None, cluster_rtol=None,
                 coop_wgs=None):
        self._o = _opts(iters, seed, cluster_rtol, coop_wgs)
        h = lib().te_server_create(int(hbm_budget), int(lanes), ctypes.byref(self._o))
        if not h:
            raise TeError("te_server_create", -1)
        self._h = ctypes.c_void_p(h)
        self._out = {}

    def submit(self, d, e, il=1, iu=None):
        d = np.ascontiguousarray(_host_f64(d))
        e = np.ascontiguousarray(_host_f64(e))
        n = int(d.shape[0])
        iu = n if iu is None else int(iu)
        m = iu - int(il) + 1
        W = np.empty(max(m, 0), dtype=np.float64)
        Z = np.empty((max(m, 0), n), dtype=np.float64)
        rid = ctypes.c_int64(0)
        rc = lib().te_server_submit(self._h, d.ctypes.data, e.ctypes.data if e.size else None, n,
                                    int(il), iu, W.ctypes.data, Z.ctypes.data, n,
                                    ctypes.byref(rid))
        _check("te_server_submit", rc)
        self._out[rid.value] = (W, Z)
        return rid.value

    def poll(self, rid):
        """True once request rid has completed (raises if it failed)."""
        rc = ctypes.c_int(0)
        r = lib().te_server_poll(self._h, int(rid), ctypes.byref(rc))
        if r < 0:
            raise TeError("te_server_poll", r)
        if r == 1:
            _check("te_server request", rc.value)
        return r == 1

    def wait(self, rid):
        """Block until request rid completes; returns (W, Z) (host arrays),
        which the server object then no longer holds."""
        rc = ctypes.c_int(0)
        r = lib().te_server_wait(self._h, int(rid), ctypes.byref(rc))
        if r < 0:
            raise TeError("te_server_wait", r)
        out = self._out.pop(int(rid), None)
        _check("te_server request", rc.value)
        return out

    def release(self, rid):
        """Free the server's record of completed request rid (its status and
        times); True if released, False if it has not completed yet."""
        r = lib().te_server_release(self._h, int(rid))
        if r < 0:
            raise TeError("te_server_release", r)
        if r == 1:
            self._out.pop(int(rid), None)
        return r == 1

    def held(self):
        """Requests whose host outputs the server object still holds."""
        return len(self._out)

    def result_code(self, rid):
        rc = ctypes.c_int(0)
        r = lib().te_server_wait(self._h, int(rid), ctypes.byref(rc))
        if r < 0:
            raise TeError("te_server_wait", r)
        return rc.value

    def times(self, rid):
        """(t_submit, t_start, t_done) in seconds since the server started."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        r = lib().te_server_times(self._h, int(rid), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(c))
        if r < 0:
            raise TeError("te_server_times", r)
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            lib().te_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
