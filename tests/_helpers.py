"""Test-side helpers: independent brute force and comparison metrics.

Nothing here implements the method under test.  ``jacobi_eigh`` is the
textbook cyclic Jacobi eigenvalue algorithm for dense symmetric matrices
(Golub and Van Loan, Matrix Computations, section 8.5), used as brute force on
tiny inputs.
"""
from __future__ import annotations

import math

import numpy as np


def dense(d, e):
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def jacobi_eigh(A, sweeps: int = 40):
    """Cyclic-by-row Jacobi: returns (eigenvalues ascending, eigenvectors).

    Each rotation zeroes a_pq exactly and updates the diagonal by -+ t a_pq
    (Rutishauser's form), which keeps the eigenvalues accurate to a few ulps
    of ||A||.
    """
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    V = np.eye(n)
    for _ in range(sweeps):
        off = float(np.sum(np.abs(np.triu(A, 1))))
        if off == 0.0:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                if abs(apq) <= 1e-30 * max(abs(A[p, p]), abs(A[q, q])):
                    A[p, q] = A[q, p] = 0.0
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                app, aqq = A[p, p], A[q, q]
                ap = A[:, p].copy()
                aq = A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                A[p, :] = A[:, p]
                A[q, :] = A[:, q]
                A[p, p] = app - t * apq
                A[q, q] = aqq + t * apq
                A[p, q] = A[q, p] = 0.0
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def mp_eigh(A, dps: int = 40):
    """High-precision brute force (mpmath, dps decimal digits); returns float64
    (eigenvalues ascending, eigenvectors)."""
    import mpmath
    with mpmath.workdps(dps):
        M = mpmath.matrix(np.asarray(A, dtype=np.float64).tolist())
        E, Q = mpmath.eigsy(M)
        w = np.array([float(x) for x in E])
        V = np.array([[float(Q[i, j]) for j in range(Q.cols)] for i in range(Q.rows)])
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def laplacian_eigs(n: int):
    k = np.arange(1, n + 1, dtype=np.float64)
    return 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))


def laplacian_vectors(n: int, cols=None):
    """Unit eigenvectors of tridiag(-1, 2, -1): sqrt(2/(n+1)) sin(i k pi/(n+1)).

    The product i*k is reduced modulo 2(n+1) in exact integer arithmetic before
    scaling so that large n keeps full accuracy.
    """
    ks = np.arange(1, n + 1) if cols is None else np.asarray(cols) + 1
    i = np.arange(1, n + 1, dtype=np.int64)[:, None]
    ik = (i * ks[None, :].astype(np.int64)) % (2 * (n + 1))
    return math.sqrt(2.0 / (n + 1)) * np.sin(ik.astype(np.float64) * np.pi / (n + 1))


def align_signs(Z, Zref):
    s = np.sign(np.sum(Z * Zref, axis=0))
    s[s == 0] = 1.0
    return Zref * s


def sin_angles(Z, Zref):
    """Per-column sin of the angle between vectors, ||z - (z.r) r|| / ||z|| with r
    the normalized reference (accurate for tiny angles, unlike sqrt(1 - cos^2))."""
    Z = np.asarray(Z, dtype=np.float64)
    R = np.asarray(Zref, dtype=np.float64)
    R = R / np.linalg.norm(R, axis=0)
    Zn = Z / np.linalg.norm(Z, axis=0)
    P = Zn - R * np.sum(Zn * R, axis=0)
    return np.linalg.norm(P, axis=0)


def subspace_sin(A, B):
    """Largest principal-angle sine between span(A) and span(B) (orthonormal bases)."""
    if A.shape[1] == 0:
        return 0.0
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    # sin of the largest angle = ||(I - qb qb^T) qa||_2
    r = qa - qb @ (qb.T @ qa)
    return float(np.linalg.norm(r, 2))


def residual(d, e, W, Z):
    """max_j ||T z_j - w_j z_j||_2 / ||T||_1, computed with the tridiagonal product."""
    d = np.asarray(d)
    e = np.asarray(e)
    TZ = d[:, None] * Z
    if len(e):
        TZ[:-1] += e[:, None] * Z[1:]
        TZ[1:] += e[:, None] * Z[:-1]
    R = TZ - Z * W[None, :]
    norm1 = np.max(np.abs(d) + np.concatenate([[0.0], np.abs(e)]) + np.concatenate([np.abs(e), [0.0]]))
    return float(np.max(np.linalg.norm(R, axis=0)) / norm1)


def orthogonality(Z):
    m = Z.shape[1]
    return float(np.max(np.abs(Z.T @ Z - np.eye(m))))


def clusters_from(W, tol):
    """Chain clustering of ascending values by gap > tol (test-side restatement)."""
    starts = [0]
    for j in range(1, len(W)):
        if W[j] - W[j - 1] > tol:
            starts.append(j)
    starts.append(len(W))
    return [(starts[a], starts[a + 1] - starts[a]) for a in range(len(starts) - 1)]
