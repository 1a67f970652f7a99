"""GPU parity of the bidiagonal singular vectors (bidiag_svd, through the
Golub-Kahan tridiagonal) against the oracle: singular values bit-exact,
left and right singular vectors per cluster within 1e-9 (subspaces), the
closed form of the all-ones bidiagonal, B V = U S and orthonormality."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from tests._helpers import orthogonality, sin_angles, subspace_sin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1209_1910_amd import binding as B  # noqa: E402


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _bidiag(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(2.0, 3.0, n), rng.uniform(-1.0, 1.0, n - 1)


def _gk(a, b):
    n = len(a)
    e = np.empty(2 * n - 1)
    e[0::2] = a
    e[1::2] = b
    return np.zeros(2 * n), e


def _run(a, b, il=1, iu=None):
    S, U, V, info = B.bidiag_svd(a, b, il, iu)
    torch.cuda.synchronize()
    return (S.cpu().numpy(), U.cpu().numpy().T.copy(), V.cpu().numpy().T.copy(),
            info.cpu().numpy())


@pytest.mark.parametrize("n,seed,il,iu", [(1, 0, 1, 1), (2, 1, 1, 2), (300, 2, 1, 300),
                                          (1000, 3, 1, 1000), (777, 4, 101, 600)])
def test_bidiag_vs_oracle(n, seed, il, iu):
    a, b = _bidiag(n, seed)
    _say(f"bidiag n={n} {il}..{iu}")
    S, U, V, info = _run(a, b, il, iu)
    So, Uo, Vo, st = O.bidiag_svd(a, b, il, iu, seed=B.TE_DEFAULT_SEED)
    assert np.array_equal(S, So)
    dg, eg = _gk(a, b)
    cst, csz = O.clusters(So, O.setup(dg, eg).tol)
    worst = 0.0
    for s, c in zip(cst, csz):
        worst = max(worst, subspace_sin(U[:, s:s + c], Uo[:, s:s + c]),
                    subspace_sin(V[:, s:s + c], Vo[:, s:s + c]))
    assert worst <= 1e-9, worst
    Bm = np.diag(a) + np.diag(b, 1)
    scale = np.max(np.abs(a)) + np.max(np.abs(b), initial=0.0)
    assert np.max(np.abs(Bm @ V - U * S)) <= 1e-12 * scale
    assert np.max(np.abs(Bm.T @ U - V * S)) <= 1e-12 * scale
    assert orthogonality(U) <= 1e-11 and orthogonality(V) <= 1e-11
    assert np.array_equal(info[1:], st) and info[0] == np.count_nonzero(st)


def test_bidiag_all_ones_closed_form():
    """sigma_k = 2 cos(k pi / (2n + 1)); the vectors interleave in the
    eigenvectors sin(i k pi / (2n + 1)) of tridiag(1, 0, 1) of order 2n."""
    n = 500
    _say(f"bidiag all ones n={n}")
    S, U, V, _ = _run(np.ones(n), np.ones(n - 1))
    k = np.arange(n, 0, -1)
    assert np.max(np.abs(S - 2.0 * np.cos(k * np.pi / (2 * n + 1)))) <= 8 * np.finfo(float).eps * 2
    i = np.arange(1, 2 * n + 1)
    Z = np.sin(np.outer(i, k) * np.pi / (2 * n + 1))
    Vc = Z[0::2] / np.linalg.norm(Z[0::2], axis=0)
    Uc = Z[1::2] / np.linalg.norm(Z[1::2], axis=0)
    assert np.max(sin_angles(V, Vc)) <= 1e-9 and np.max(sin_angles(U, Uc)) <= 1e-9
    # U and V are one sign apart in each column, as the interleaved vector dictates
    sv = np.sign(np.sum(V * Vc, axis=0))
    su = np.sign(np.sum(U * Uc, axis=0))
    assert np.array_equal(sv, su)
