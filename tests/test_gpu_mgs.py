"""GPU parity of the modified Gram-Schmidt variant (te_opts.orth =
TE_ORTH_MGS, the paper's Alg. 1) against the oracle's MGS path, through the
C-ABI, and its agreement with the compact-WY path.

Bars as for the compact-WY path: eigenvalues bit-exact; cluster subspaces
(largest principal-angle sine) and singleton vectors within 1e-9 of the
oracle; residual max ||T z - w z|| / ||T||_1 <= 1e-12; orthogonality
max |Z^T Z - I| <= 1e-11.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1209_1910_amd import inputs as G
from tests._helpers import orthogonality, residual, sin_angles, subspace_sin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1209_1910_amd import binding as B  # noqa: E402

SEED = B.TE_DEFAULT_SEED


def _say(msg):
    print(f"[gpu-mgs] {msg}", flush=True)


def _gpu(d, e, il=1, iu=None, orth="mgs"):
    W, Z, _ = B.tridiag_eigvecs_ex(d, e, il, iu, orth=orth)
    torch.cuda.synchronize()
    return W.cpu().numpy(), Z.cpu().numpy().T.copy()


def _compare(d, e, Wg, Zg, Wo, Zo):
    p = O.setup(d, e)
    assert np.array_equal(Wg, Wo), "eigenvalues not bit-identical"
    st, sz = O.clusters(Wo, p.tol)
    worst = 0.0
    for s, c in zip(st, sz):
        if c == 1:
            worst = max(worst, float(sin_angles(Zg[:, s:s + 1], Zo[:, s:s + 1])[0]))
        else:
            worst = max(worst, subspace_sin(Zg[:, s:s + c], Zo[:, s:s + c]))
    assert worst <= 1e-9, worst
    assert residual(d, e, Wg, Zg) <= 1e-12
    assert orthogonality(Zg) <= 1e-11
    return worst


CASES = {
    "n2": lambda: (np.array([0.3, -1.1]), np.array([0.7])),
    "ragged333": lambda: G.uniform_tridiag(333, 17),
    "small1000": G.workload_small,
    "laplacian500": lambda: G.laplacian_tridiag(500),
    "glued24": lambda: G.glued_wilkinson(24, 1e-8),
    "glued60": lambda: G.glued_wilkinson(60, 1e-8),
    "type1_700": lambda: G.type1_tridiag(700, 5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_mgs_vs_oracle_mgs(name):
    d, e = CASES[name]()
    _say(f"mgs {name} n={len(d)}")
    Wg, Zg = _gpu(d, e)
    Wo, Zo, _ = O.eigvecs(d, e, orth=O.MGS, seed=SEED)
    _compare(d, e, Wg, Zg, Wo, Zo)


def test_mgs_and_cwy_span_the_same_cluster_subspaces():
    d, e = G.glued_wilkinson(40, 1e-8)
    _say("mgs vs cwy, glued 40")
    Wm, Zm = _gpu(d, e, orth="mgs")
    Wc, Zc = _gpu(d, e, orth="cwy")
    assert np.array_equal(Wm, Wc)
    st, sz = O.clusters(Wm, O.setup(d, e).tol)
    for s, c in zip(st, sz):
        assert subspace_sin(Zm[:, s:s + c], Zc[:, s:s + c]) <= 1e-9, s


def test_mgs_range_batched_and_repeat():
    """Ranges follow the oracle's MGS range run; a batch gives each problem the
    bits of its own call; a repeat gives the same bits."""
    d, e = G.uniform_tridiag(600, 23)
    for il, iu in [(101, 250), (37, 38)]:
        _say(f"mgs range {il}..{iu}")
        Wg, Zg = _gpu(d, e, il, iu)
        Wr, Zr, _ = O.eigvecs(d, e, il=il, iu=iu, orth=O.MGS, seed=SEED)
        _compare(d, e, Wg, Zg, Wr, Zr)
    probs = [(dd, ee) for dd, ee, _ in G.batched_problems(count=16, seed=7, n_lo=32, n_hi=500)]
    _say("mgs batched 16")
    out = B.tridiag_eigvecs_batched(probs, orth="mgs")
    torch.cuda.synchronize()
    for (dd, ee), (W, Z) in zip(probs, out):
        W1, Z1 = _gpu(dd, ee)
        assert np.array_equal(W.cpu().numpy(), W1)
        assert np.array_equal(Z.cpu().numpy().T, Z1)
    W2, Z2 = _gpu(d, e, 101, 250)
    W3, Z3 = _gpu(d, e, 101, 250)
    assert np.array_equal(W2, W3) and np.array_equal(Z2, Z3)


def test_mgs_limits():
    """n above TE_MGS_MAX_N reports TE_ERR_UNSUPPORTED before any work is
    enqueued, in the plain and in the graph path (there for any problem of
    the batch); the autotuner takes compact-WY options only."""
    d, e = G.uniform_tridiag(B.TE_MGS_MAX_N + 1, 3)
    with pytest.raises(B.TeError) as err:
        B.tridiag_eigvecs_ex(d, e, 1, 4, orth="mgs")
    assert err.value.rc == B.TE_ERR_UNSUPPORTED
    lay = B.BatchLayout([G.uniform_tridiag(64, 1), (d, e, 1, 4)])
    with pytest.raises(B.TeError) as err:
        B.BatchGraph(lay, orth="mgs")
    assert err.value.rc == B.TE_ERR_UNSUPPORTED
    lay = B.BatchLayout([G.uniform_tridiag(64, 1)])
    with pytest.raises(B.TeError) as err:
        B.batch_autotune(lay, orth="mgs")
    assert err.value.rc == B.TE_ERR_UNSUPPORTED
