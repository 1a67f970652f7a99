"""Seeded synthetic inputs for the symmetric tridiagonal eigenvector workloads.

This module only draws and assembles matrices and request traces; it holds
none of the method's arithmetic, so both the HIP path and the CPU oracle can be
fed from it without sharing any computation.

Matrix families follow the experiment section (section 5.1) of Ishigami,
Kimura and Nakamura, arXiv:1209.1910:

* random tridiagonal matrices (the paper's Type 1 draws entries from [0, 1);
  the benchmark workloads here draw them from U(-1, 1));
* tridiag(1, 1, 1) (Type 2) and the closely related tridiag(-1, 2, -1), which
  has the same eigenvectors and a textbook closed form;
* glued Wilkinson matrices W_g^+ (Type 3): g copies of W_21^+ (diagonal
  |10 - i|, i = 0..20, off-diagonal 1) joined by coupling off-diagonals delta.

Every generator returns float64 numpy arrays ``(d, e)`` with ``len(e) ==
len(d) - 1``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "uniform_tridiag",
    "type1_tridiag",
    "type2_tridiag",
    "laplacian_tridiag",
    "wilkinson_w21",
    "glued_wilkinson",
    "workload_small",
    "workload_glued",
    "workload_laplacian",
    "batched_problems",
    "serving_trace",
    "ServingRequest",
]


def uniform_tridiag(n: int, seed: int, low: float = -1.0, high: float = 1.0):
    """d then e drawn i.i.d. from U(low, high) with numpy's PCG64 ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(low, high, n)
    e = rng.uniform(low, high, max(n - 1, 0))
    return d.astype(np.float64), e.astype(np.float64)


def type1_tridiag(n: int, seed: int):
    """The paper's Type 1 matrix: entries uniform in [0, 1)."""
    return uniform_tridiag(n, seed, 0.0, 1.0)


def type2_tridiag(n: int):
    """The paper's Type 2 matrix tridiag(1, 1, 1)."""
    return np.ones(n, dtype=np.float64), np.ones(max(n - 1, 0), dtype=np.float64)


def laplacian_tridiag(n: int):
    """tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(k pi / (n + 1))."""
    return np.full(n, 2.0, dtype=np.float64), np.full(max(n - 1, 0), -1.0, dtype=np.float64)


def wilkinson_w21():
    """W_21^+: diagonal |10 - i| for i = 0..20, off-diagonal 1."""
    d = np.abs(10.0 - np.arange(21, dtype=np.float64))
    e = np.ones(20, dtype=np.float64)
    return d, e


def glued_wilkinson(g: int, delta: float):
    """g copies of W_21^+ on the diagonal, consecutive copies coupled by ``delta``.

    The coupling sits at off-diagonal positions 21 c + 20 for c = 0..g-2.
    """
    if g < 1:
        raise ValueError("g must be >= 1")
    wd, we = wilkinson_w21()
    d = np.tile(wd, g)
    e = np.empty(21 * g - 1, dtype=np.float64)
    for c in range(g):
        e[21 * c: 21 * c + 20] = we
        if c < g - 1:
            e[21 * c + 20] = delta
    return d, e


# --- the named workloads -----------------------------------------------------

def workload_small():
    """n = 1000, d then e from U(-1, 1) with seed 0 (all 1000 eigenvectors)."""
    return uniform_tridiag(1000, 0)


def workload_glued():
    """380 copies of W_21^+ coupled by 1e-8: n = 7980."""
    return glued_wilkinson(380, 1e-8)


def workload_laplacian(n: int = 16000):
    """tridiag(-1, 2, -1) at n = 16000 (the closed-form scale test)."""
    return laplacian_tridiag(n)


def batched_problems(count: int = 4096, seed: int = 1, n_lo: int = 64, n_hi: int = 2048,
                     glued_frac: float = 0.25, delta: float = 1e-8):
    """Independent problems with n log-uniform in [n_lo, n_hi].

    Draw order (one ``default_rng(seed)`` stream): ``count`` log-uniform sizes,
    then ``count`` glued flags (U < glued_frac), then per problem its entries in
    order.  A glued problem uses g = max(1, round(n / 21)) copies of W_21^+
    coupled by ``delta``, so its order is 21 g; the others draw d then e from
    U(-1, 1).  Returns a list of ``(d, e, glued)``.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    glued = rng.uniform(0.0, 1.0, count) < glued_frac
    out = []
    for b in range(count):
        n = int(sizes[b])
        if glued[b]:
            g = max(1, int(round(n / 21)))
            d, e = glued_wilkinson(g, delta)
        else:
            d = rng.uniform(-1.0, 1.0, n)
            e = rng.uniform(-1.0, 1.0, n - 1)
        out.append((d.astype(np.float64), e.astype(np.float64), bool(glued[b])))
    return out


@dataclass
class ServingRequest:
    arrival_s: float      # arrival time from the start of the trace
    d: np.ndarray
    e: np.ndarray
    il: int               # 1-based first requested eigenvalue index
    iu: int               # 1-based last requested index (inclusive)
    glued: bool


def serving_trace(count: int = 200, qps: float = 1.0, seed: int = 2, n_lo: int = 256,
                  n_hi: int = 16384, glued_frac: float = 0.3, full_frac: float = 0.5,
                  range_frac: float = 0.1, delta: float = 1e-8):
    """Poisson request stream at a fixed rate.

    Per request (one ``default_rng(seed)`` stream, in this order): exponential
    inter-arrival with mean 1/qps, log-uniform n in [n_lo, n_hi], glued flag
    (U < glued_frac), full-spectrum flag (U < full_frac), a uniform offset for a
    contiguous index range of round(range_frac * n) indices, then the entries.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += rng.exponential(1.0 / qps)
        n = int(np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        glued = bool(rng.uniform() < glued_frac)
        full = bool(rng.uniform() < full_frac)
        off_u = rng.uniform()
        if glued:
            g = max(1, int(round(n / 21)))
            d, e = glued_wilkinson(g, delta)
            n = 21 * g
        else:
            d = rng.uniform(-1.0, 1.0, n)
            e = rng.uniform(-1.0, 1.0, n - 1)
        if full:
            il, iu = 1, n
        else:
            cnt = max(1, int(round(range_frac * n)))
            off = min(int(off_u * (n - cnt + 1)), n - cnt)
            il, iu = off + 1, off + cnt
        reqs.append(ServingRequest(t, d.astype(np.float64), e.astype(np.float64), il, iu, glued))
    return reqs
