"""GPU tests of the graph-captured batched path (te_batch_graph_*) and its
autotuner, through the C-ABI.

The graph runs every step on the device (the chain plan included) and must
give the same bits as the host-planned batched call, which the parity tests
tie to the oracle; a few problems are also checked against the oracle here.
Each graph is replayed several times, with eager work and synchronizations
between the replays, and every replay is compared with the eager result.
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

SEED = B.TE_DEFAULT_SEED


def _say(msg):
    print(f"[gpu-graph] {msg}", flush=True)


def _mixed(count, seed, n_lo, n_hi, ranges=False):
    probs = [(d, e) for d, e, _ in G.batched_problems(count=count, seed=seed, n_lo=n_lo,
                                                      n_hi=n_hi)]
    if ranges:  # every third problem asks for a contiguous index range
        out = []
        for k, (d, e) in enumerate(probs):
            n = len(d)
            if k % 3 == 1 and n >= 10:
                il = 1 + n // 4
                out.append((d, e, il, il + n // 10))
            else:
                out.append((d, e))
        probs = out
    return probs


def _snapshot(lay):
    torch.cuda.synchronize()
    return lay.W_all.cpu().numpy().copy(), lay.Z_all.cpu().numpy().copy()


def _eager(probs):
    lay = B.BatchLayout(probs)
    B.tridiag_eigvecs_batched(lay)
    return _snapshot(lay)


def test_graph_replays_match_eager_batched_and_oracle():
    probs = _mixed(40, 11, 16, 600, ranges=True)
    _say("graph vs eager, 40 problems with ranges")
    W0, Z0 = _eager(probs)
    lay = B.BatchLayout(probs)
    with B.BatchGraph(lay) as g:
        info = g.info()
        assert info["segments"] == 1 and info["device_bytes"] > 0
        for rep in range(3):
            lay.W_all.fill_(float("nan"))      # eager work between the replays
            lay.Z_all.fill_(float("nan"))
            torch.cuda.synchronize()
            g.launch()
            W1, Z1 = _snapshot(lay)
            assert np.array_equal(W1, W0), rep
            assert np.array_equal(Z1, Z0), rep
    # a few problems against the oracle directly
    for k in (0, 1, 7, 20):
        p = probs[k]
        d, e = p[0], p[1]
        il, iu = (p[2], p[3]) if len(p) == 4 else (1, len(d))
        Wg = W0[lay.woff[k]: lay.woff[k] + lay.ms[k]]
        Zg = Z0[lay.zoff[k]: lay.zoff[k] + lay.ms[k] * len(d)].reshape(-1, len(d)).T
        Wo, Zo, _ = O.eigvecs(d, e, il, iu, seed=SEED)
        assert np.array_equal(Wg, Wo), k
        tol = O.setup(d, e).tol
        Wfull = O.bisect(d, e)
        st, sz = O.clusters(Wo, tol)
        for s, c in zip(st, sz):
            # a cluster that the range cuts out of a larger one (a neighbour
            # outside the range within the gap) may hold part of a numerically
            # degenerate group, whose vectors are not unique: residual and
            # orthogonality only
            lo, hi = il - 1 + s, il - 1 + s + c
            cut = (lo > 0 and Wfull[lo] - Wfull[lo - 1] <= tol) or \
                  (hi < len(d) and Wfull[hi] - Wfull[hi - 1] <= tol)
            if not cut:
                assert subspace_sin(Zg[:, s:s + c], Zo[:, s:s + c]) <= 1e-9, (k, s)
        assert residual(d, e, Wg, Zg) <= 1e-12
        assert orthogonality(Zg) <= 1e-11


def test_graph_reads_inputs_at_launch():
    """The graph binds the buffers, not their contents: new matrices of the
    same sizes written into d_all / e_all give their own eigenpairs."""
    a = _mixed(12, 3, 16, 300)
    b = []
    rng = np.random.default_rng(99)
    for d, e in a:
        b.append((rng.uniform(-1, 1, len(d)), rng.uniform(-1, 1, len(e))))
    Wb, Zb = _eager(b)
    lay = B.BatchLayout(a)
    with B.BatchGraph(lay) as g:
        g.launch()
        lay_b = B.BatchLayout(b)
        lay.d_all.copy_(lay_b.d_all)
        lay.e_all.copy_(lay_b.e_all)
        torch.cuda.synchronize()
        g.launch()
        W1, Z1 = _snapshot(lay)
    assert np.array_equal(W1, Wb) and np.array_equal(Z1, Zb)


def test_graph_configurations_and_segments_agree():
    """Every chain configuration (threads per chain workgroup, chains per CU)
    and a budget that forces several segments give identical bits."""
    probs = _mixed(30, 21, 32, 700)
    probs.append(G.glued_wilkinson(30, 1e-8))          # clusters of 30 and 60 members
    W0, Z0 = _eager(probs)
    lay = B.BatchLayout(probs)
    for nt, per in ((256, 1), (256, 2), (512, 1), (512, 2)):
        _say(f"config {nt} x {per}")
        try:
            g = B.BatchGraph(lay, chain_threads=nt, chains_per_cu=per)
        except B.TeError as err:
            assert err.rc == -12, err      # beyond this variant's occupancy limit
            continue
        with g:
            for rep in range(2):
                lay.Z_all.zero_()
                g.launch()
                W1, Z1 = _snapshot(lay)
                assert np.array_equal(W1, W0) and np.array_equal(Z1, Z0), (nt, per, rep)
    _say("segments")
    with B.BatchGraph(lay, chain_threads=256, chains_per_cu=1, ws_budget=128 << 20) as g:
        assert g.info()["segments"] > 1
        lay.Z_all.zero_()
        g.launch()
        W1, Z1 = _snapshot(lay)
        assert np.array_equal(W1, W0) and np.array_equal(Z1, Z0)


@pytest.mark.parametrize("stop", ["fixed", "growth"])
def test_graph_mgs_chains_match_eager_mgs(stop):
    """With MGS options the graph runs the MGS chain kernel: every replay is
    bit-identical to the host-planned batched call with the same options; a
    chain configuration of another workgroup size is rejected (argument 12)."""
    probs = _mixed(24, 41, 32, 600, ranges=True)
    probs.append(G.glued_wilkinson(20, 1e-8))          # clusters of 20 and 40 members
    opts = dict(orth="mgs") if stop == "fixed" else dict(orth="mgs", stop=B.TE_STOP_GROWTH)
    lay0 = B.BatchLayout(probs)
    _say(f"mgs graph ({stop}): eager")
    B.tridiag_eigvecs_batched(lay0, **opts)
    W0, Z0 = _snapshot(lay0)
    lay = B.BatchLayout(probs)
    with pytest.raises(B.TeError) as err:
        B.BatchGraph(lay, chain_threads=256, chains_per_cu=1, **opts)
    assert err.value.rc == -12
    for cfg in ({}, dict(chain_threads=512, chains_per_cu=1)):
        _say(f"mgs graph ({stop}) {cfg}")
        with B.BatchGraph(lay, **cfg, **opts) as g:
            assert g.info()["chain_threads"] == 512
            for rep in range(2):
                lay.W_all.zero_()
                lay.Z_all.fill_(float("nan"))
                torch.cuda.synchronize()
                g.launch()
                W1, Z1 = _snapshot(lay)
                assert np.array_equal(W1, W0) and np.array_equal(Z1, Z0), (cfg, rep)
    # the MGS result itself against the oracle's MGS on the glued problem
    d, e = probs[-1]
    W, Z = lay.results()[-1]
    iters = O.STOP_GROWTH if stop == "growth" else 3
    Wo, Zo, _ = O.eigvecs(d, e, orth=O.MGS, seed=SEED, iters=iters)
    assert np.array_equal(W.cpu().numpy(), Wo)
    Zg = Z.cpu().numpy().T.copy()
    st, sz = O.clusters(Wo, O.setup(d, e).tol)
    assert max(sz) >= 20
    for s0, c in zip(st, sz):   # each cluster's subspace (a singleton: its line)
        assert subspace_sin(Zg[:, s0:s0 + c], Zo[:, s0:s0 + c]) <= 1e-9, (s0, c)
    assert residual(d, e, Wo, Zg) <= 1e-12 and orthogonality(Zg) <= 1e-11


def test_autotune_records_and_uses_the_winner(tmp_path, monkeypatch):
    tf = tmp_path / "tune.txt"
    monkeypatch.setenv("TE_TUNE_FILE", str(tf))
    probs = _mixed(64, 31, 64, 900)
    W0, Z0 = _eager(probs)
    lay = B.BatchLayout(probs)
    _say("autotune")
    best, tried = B.batch_autotune(lay)
    assert len(tried) >= 2 and best in [c for c, _ in tried]
    assert all(ms > 0 for _, ms in tried)
    assert min(tried, key=lambda t: t[1])[0] == best
    line = [ln for ln in tf.read_text().splitlines() if ln and not ln.startswith("#")][-1]
    assert tuple(int(x) for x in line.split()[2:4]) == best
    with B.BatchGraph(lay) as g:          # no configuration given: the table's
        info = g.info()
        assert (info["chain_threads"], info["chains_per_cu"]) == best
        lay.Z_all.zero_()
        g.launch()
        W1, Z1 = _snapshot(lay)
    assert np.array_equal(W1, W0) and np.array_equal(Z1, Z0)


def test_graph_full_batched_workload():
    """The 4096-problem batched workload in the launch configuration the
    benchmark times: bit-identical to the host-planned batched call (compared
    on the device), and sampled problems against the oracle."""
    full = G.batched_problems()
    probs = [(d, e) for d, e, _ in full]
    lay = B.BatchLayout(probs)
    _say("full batched workload: eager")
    B.tridiag_eigvecs_batched(lay)
    torch.cuda.synchronize()
    W0, Z0 = lay.W_all.clone(), lay.Z_all.clone()
    lay.W_all.zero_()
    lay.Z_all.zero_()
    _say("full batched workload: graph")
    with B.BatchGraph(lay) as g:
        g.launch()
    torch.cuda.synchronize()
    assert torch.equal(lay.W_all, W0) and torch.equal(lay.Z_all, Z0)
    del W0, Z0
    rng = np.random.default_rng(4)
    small = [k for k in range(len(probs)) if len(probs[k][0]) <= 700]
    glued = [k for k in small if full[k][2]]
    pick = list(rng.choice(small, 4, replace=False)) + glued[:2]
    for k in pick:
        d, e = probs[k]
        n = len(d)
        Wg = lay.W_all[lay.woff[k]: lay.woff[k] + n].cpu().numpy()
        Zg = lay.Z_all[lay.zoff[k]: lay.zoff[k] + n * n].cpu().numpy().reshape(n, n).T
        Wo, Zo, _ = O.eigvecs(d, e, seed=SEED)
        assert np.array_equal(Wg, Wo), k
        st, sz = O.clusters(Wo, O.setup(d, e).tol)
        for s, c in zip(st, sz):
            assert subspace_sin(Zg[:, s:s + c], Zo[:, s:s + c]) <= 1e-9, (k, s)
        assert residual(d, e, Wg, Zg) <= 1e-12
        assert orthogonality(Zg) <= 1e-11
