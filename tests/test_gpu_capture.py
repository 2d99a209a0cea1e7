"""The entry points only enqueue work, so a caller may capture a whole call into
its own HIP graph: rf_svd (k = 300, where the Ritz eigensolver is large enough
to be replayed from the library's own graph cache when not capturing) and
rf_lowrank, captured on torch's capture stream, replayed several times with
eager work between the replays, against the eager result bit for bit."""
import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _A(m, n, seed):
    A, _ = synth.workload("poly65k", m=m, n=n, seed=seed)
    return torch.from_numpy(A.astype(np.float32)).to(DEV)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_rf_svd_captured_in_caller_graph(precision):
    A = _A(3000, 1600, 4)
    k, l, q, s, seed = 300, 600, 1, 8, 12
    p = rf.params(k, l, q, s, seed, precision)
    nws = rf.rf_workspace_size(rf.RF_OP_SVD, A, p)
    ws = torch.empty(nws, dtype=torch.uint8, device=DEV)
    out = (torch.empty((3000, k), device=DEV), torch.empty(k, dtype=torch.float64, device=DEV),
           torch.empty((k, 1600), device=DEV), torch.zeros(24, dtype=torch.uint8, device=DEV))
    # eager reference (also fills the library's eigensolver graph cache for these buffers)
    rf.rf_svd(A, k, l, q, s, seed, precision, workspace=(ws, nws), out=out)
    torch.cuda.synchronize()
    want = [t.clone() for t in out]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rf.rf_svd(A, k, l, q, s, seed, precision, workspace=(ws, nws), out=out)
    for rep in range(3):
        for t in out[:3]:
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(700, 700, device=DEV) @ torch.randn(700, 700, device=DEV)
        torch.cuda.synchronize()
        del junk
        for a, b in zip(out, want):
            assert torch.equal(a, b), rep
    # an eager call after the capture still matches
    rf.rf_svd(A, k, l, q, s, seed, precision, workspace=(ws, nws), out=out)
    torch.cuda.synchronize()
    for a, b in zip(out, want):
        assert torch.equal(a, b)


def test_rf_lowrank_captured_in_caller_graph():
    A = _A(2000, 1200, 5)
    k, l, q, s, seed = 80, 200, 2, 4, 3
    p = rf.params(k, l, q, s, seed, "mixed")
    nws = rf.rf_workspace_size(rf.RF_OP_LOWRANK, A, p)
    ws = torch.empty(nws, dtype=torch.uint8, device=DEV)
    Y0, X0, _ = rf.rf_lowrank(A, k, l, q, s, seed, "mixed", workspace=(ws, nws))
    torch.cuda.synchronize()
    holder = {}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        holder["out"] = rf.rf_lowrank(A, k, l, q, s, seed, "mixed", workspace=(ws, nws))
    Y, X, _ = holder["out"]
    for rep in range(3):
        Y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, Y0) and torch.equal(X, X0), rep


def test_eig_graph_cache_eviction_without_device_sync():
    """More distinct buffer sets than the cache holds: entries are dropped only
    once their last launch is done (event query), results stay correct."""
    rng = np.random.default_rng(0)
    outs = []
    for i in range(11):
        M = rng.standard_normal((160, 160))
        G = torch.from_numpy(M @ M.T).to(DEV)
        lam, V = rf.rf_test_eig(G, tol=1e-12)
        outs.append((G, lam, V))
    torch.cuda.synchronize()
    for G, lam, V in outs:
        ref = np.linalg.eigvalsh(G.cpu().numpy())[::-1]
        assert np.allclose(lam.cpu().numpy(), ref, rtol=1e-10, atol=1e-10 * ref[0])
