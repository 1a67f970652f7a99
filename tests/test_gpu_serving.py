"""Serving engine on the GPU, through the C-ABI (te_server_*).

Each result must be the same whether its request ran alone or in a mix of
requests admitted together and overlapping on the device.  The method runs
problem by problem, and the cluster chains give the same bits for any number
of workgroups, so the bar is bit-identical W and Z (also against the plain
one-problem entry point).  The mixed results also meet the accuracy
bars (residual <= 1e-12 ||T||_1, orthogonality <= 1e-11) and, for a small
case, the oracle to the subspace bar 1e-9.  The HBM budget is exercised with
a budget that admits one request at a time and one that a request exceeds.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1209_1910_amd import inputs as G
from tests._helpers import orthogonality, residual, subspace_sin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1209_1910_amd import binding as B  # noqa: E402

TE_ERR_WORKSPACE = -1002


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _requests():
    """A mix of sizes and kinds: a range request, glued Wilkinson, cluster
    chains on both chain kernels (the Laplacian is one cluster for n >= 1571,
    and at n = 1600 and 2100 that cluster goes to the cooperative kernel),
    light and heavy classes (n * m >= 2^22 is heavy)."""
    reqs = []
    d, e = G.uniform_tridiag(300, 41)
    reqs.append((d, e, 1, 300))
    d, e = G.uniform_tridiag(700, 42)
    reqs.append((d, e, 100, 170))
    d, e = G.glued_wilkinson(10, 1e-8)
    reqs.append((d, e, 1, len(d)))
    d, e = G.laplacian_tridiag(1600)
    reqs.append((d, e, 1, 1600))
    d, e = G.laplacian_tridiag(2100)          # heavy class
    reqs.append((d, e, 1, 2100))
    d, e = G.type1_tridiag(500, 44)
    reqs.append((d, e, 1, 500))
    d, e = np.array([0.25]), np.array([])
    reqs.append((d, e, 1, 1))
    return reqs


def _io_bytes(n, m):
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    return al(8 * n) + al(8 * max(n - 1, 1)) + al(8 * m) + al(8 * n * m)


def _need(n, il, iu):
    return B.lib().tridiag_eigvecs_workspace_bytes(n, il, iu) + _io_bytes(n, iu - il + 1)


def _alone(reqs):
    out = []
    for k, (d, e, il, iu) in enumerate(reqs):
        _say(f"alone {k}: n={len(d)} il={il} iu={iu}")
        with B.Server(lanes=1) as s:
            rid = s.submit(d, e, il, iu)
            W, Z = s.wait(rid)
            out.append((W.copy(), Z.copy()))
    return out


@pytest.fixture(scope="module")
def alone():
    reqs = _requests()
    return reqs, _alone(reqs)


def test_mix_equals_alone(alone):
    reqs, ref = alone
    _say("mix: all requests at once, 3 lanes")
    with B.Server(lanes=3) as s:
        ids = [s.submit(d, e, il, iu) for (d, e, il, iu) in reqs]
        got = [s.wait(r) for r in ids]
        times = [s.times(r) for r in ids]
    for k, ((W, Z), (Wr, Zr)) in enumerate(zip(got, ref)):
        assert np.array_equal(W, Wr), k
        assert np.array_equal(Z, Zr), k
    for t_sub, t_start, t_done in times:
        assert 0.0 <= t_sub <= t_start <= t_done
    for (d, e, il, iu), (W, Z) in zip(reqs, got):
        assert residual(d, e, W, Z.T.copy()) <= 1e-12
        assert orthogonality(Z.T.copy()) <= 1e-11


def test_mix_equals_plain_entry_point(alone):
    reqs, ref = alone
    for k, (d, e, il, iu) in enumerate(reqs):
        _say(f"plain {k}")
        W, Z = B.tridiag_eigvecs(d, e, il, iu)
        torch.cuda.synchronize()
        assert np.array_equal(W.cpu().numpy(), ref[k][0]), k
        assert np.array_equal(Z.cpu().numpy(), ref[k][1]), k


def test_served_small_case_matches_oracle(alone):
    reqs, ref = alone
    d, e, il, iu = reqs[0]
    Wo, Zo, _ = O.eigvecs(d, e, il, iu)
    W, Z = ref[0]
    assert np.array_equal(W, Wo)
    p = O.setup(d, e)
    st, sz = O.clusters(Wo, p.tol)
    worst = max(subspace_sin(Z.T[:, s:s + c], Zo[:, s:s + c]) for s, c in zip(st, sz))
    assert worst <= 1e-9


def test_budget_one_at_a_time_and_too_large(alone):
    reqs, ref = alone
    needs = [_need(len(d), il, iu) for (d, e, il, iu) in reqs]
    budget = max(needs) + 4096
    big_d, big_e = G.uniform_tridiag(3000, 43)
    assert _need(3000, 1, 3000) > budget
    _say(f"budget {budget} bytes")
    with B.Server(hbm_budget=budget, lanes=2) as s:
        ids = [s.submit(d, e, il, iu) for (d, e, il, iu) in reqs]
        big = s.submit(big_d, big_e, 1, 3000)
        got = [s.wait(r) for r in ids]
        assert s.result_code(big) == TE_ERR_WORKSPACE
        assert s.poll(ids[0])
    for k, ((W, Z), (Wr, Zr)) in enumerate(zip(got, ref)):
        assert np.array_equal(W, Wr), k
        assert np.array_equal(Z, Zr), k


def test_requests_keep_arriving_while_busy(alone):
    """Continuous batching: requests submitted while earlier rounds run are
    admitted into later rounds; every result is still the alone result."""
    reqs, ref = alone
    order = [4, 0, 1, 3, 2, 5, 6, 0, 2]
    with B.Server(lanes=2) as s:
        ids = []
        for k in order:
            d, e, il, iu = reqs[k]
            ids.append(s.submit(d, e, il, iu))
            s.poll(ids[0])
        for k, rid in zip(order, ids):
            W, Z = s.wait(rid)
            assert np.array_equal(W, ref[k][0]), k
            assert np.array_equal(Z, ref[k][1]), k


def test_concurrent_submitters(alone):
    """Several host threads submit to one server at once (the entry points
    are thread-safe); every result is still the alone result."""
    import threading
    reqs, ref = alone
    errors = []
    with B.Server(lanes=3) as s:
        def worker(t):
            try:
                for k in range(t, len(reqs), 3):
                    d, e, il, iu = reqs[k]
                    W, Z = s.wait(s.submit(d, e, il, iu))
                    if not (np.array_equal(W, ref[k][0]) and np.array_equal(Z, ref[k][1])):
                        errors.append(k)
            except Exception as exc:  # surfaced below
                errors.append(repr(exc))
        threads = [threading.Thread(target=worker, args=(t,)) for t in range(3)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
    assert not errors, errors


def test_released_requests_are_forgotten():
    """A long request stream does not grow the server: each completed request
    is released once read (its id is then unknown), and wait hands the host
    outputs to the caller, so neither side keeps per-request state."""
    d, e = G.uniform_tridiag(64, 3)
    W0, Z0 = B.tridiag_eigvecs(d, e)
    torch.cuda.synchronize()
    W0, Z0 = W0.cpu().numpy(), Z0.cpu().numpy()
    _say("release: 200 requests")
    with B.Server(lanes=2) as s:
        ids = [s.submit(d, e) for _ in range(200)]
        for rid in ids:
            W, Z = s.wait(rid)
            assert np.array_equal(W, W0) and np.array_equal(Z, Z0)
            assert s.release(rid)
            with pytest.raises(B.TeError):
                s.poll(rid)
        assert s.held() == 0
