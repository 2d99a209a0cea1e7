"""Batched randomised SVD (rf_svd_batched_plan / _run) against the FP64 oracle,
problem by problem (problem i uses matrix index i in the Philox counter), and
graph replays against direct launches."""
import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
import synth
from oracle import methods as me, evaluate as ev

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problems(seed, count, mrange=(120, 1500), nrange=(60, 900), krange=(4, 64)):
    """Uneven shapes and ranks; sigma_i = i^-p with p in [0.5, 2] (no noise)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(*mrange))
        n = int(rng.integers(*nrange))
        k = int(min(rng.integers(*krange), n // 2, m // 2))
        l = min(2 * k, n, m)
        p = float(rng.uniform(0.5, 2.0))
        r = min(m, n)
        sigma = np.arange(1, r + 1, dtype=np.float64) ** -p
        A = synth.spectrum_matrix(m, n, sigma, 1000 + 17 * seed + i).astype(np.float32)
        out.append((A, k, l))
    return out


def _oracle(A, k, l, q, i, seed):
    return me.rand_svd(A.astype(np.float64), me.Params(k=k, l=l, q=q, s=4, seed=seed, b=i))


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_fp32_matches_oracle(use_graph):
    probs = _problems(1, 7)
    As = [torch.from_numpy(A).to(DEV) for A, _, _ in probs]
    plan = rf.BatchPlan(As, [k for _, k, _ in probs], [l for _, _, l in probs], q=2, seeds=42, precision="fp32",
                        use_graph=use_graph).run()
    torch.cuda.synchronize()
    info = plan.info.cpu().numpy()
    for i, (A, k, l) in enumerate(probs):
        ref = _oracle(A, k, l, 2, i, 42)
        sig = plan.sigma[i].cpu().numpy()
        U = plan.U[i].cpu().numpy().astype(np.float64)
        tol = 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]
        assert np.all(np.abs(sig - ref.sigma) <= tol), (i, np.max(np.abs(sig - ref.sigma) / tol))
        assert np.max(np.abs(U.T @ U - np.eye(k))) < 2e-5
        A64 = A.astype(np.float64)
        eg, eo = ev.frob_error(A64, U), ev.frob_error(A64, ref.U)
        assert abs(eg - eo) <= 1e-4 * eo + 1e-6 * np.linalg.norm(A64), (i, eg, eo)
        assert int.from_bytes(info[i, 0:4].tobytes(), "little") & 2 == 0


def _truncated_problem(m, n, k, p, seed, r=None):
    """U diag(sigma) V^T with sigma_i = i^-p and Haar factors of rank r (the
    spectrum law of the batched workload, truncated so that a 8192 x 4096
    instance is generated in seconds)."""
    r = min(m, n) if r is None else r
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -p
    return synth.spectrum_matrix(m, n, sigma, seed).astype(np.float32)


def test_batched_fp32_matches_oracle_at_workload_ranks():
    """Ranks of the batched workload (k up to 256, so the Cholesky/inverse runs
    2 to 4 tiles of 64 and the batched Jacobi several rounds), m up to 8192,
    n up to 4096, sketch = min(2k, n), s = 4, q = 2: each problem against the
    oracle (problem index i in the Philox counter)."""
    shapes = [(3000, 1500, 64, 1.2), (2500, 1200, 65, 0.7), (4000, 2000, 128, 1.5), (3000, 2500, 200, 0.5),
              (8192, 4096, 256, 1.0)]
    probs = []
    for i, (m, n, k, pw) in enumerate(shapes):
        A = _truncated_problem(m, n, k, pw, 300 + i, r=min(m, n, 1024))
        probs.append((A, k, min(2 * k, n)))
    As = [torch.from_numpy(A).to(DEV) for A, _, _ in probs]
    for precision in ("fp32", "mixed"):
        plan = rf.BatchPlan(As, [k for _, k, _ in probs], [l for _, _, l in probs], q=2, seeds=21,
                            precision=precision, use_graph=True).run()
        torch.cuda.synchronize()
        for i, (A, k, l) in enumerate(probs):
            ref = _oracle(A, k, l, 2, i, 21)
            A64 = A.astype(np.float64)
            U = plan.U[i].cpu().numpy().astype(np.float64)
            sig = plan.sigma[i].cpu().numpy()
            eg, eo = ev.frob_error(A64, U), ev.frob_error(A64, ref.U)
            print("%s problem %d (m %d n %d k %d): err gpu %.8e oracle %.8e rel %.2e" %
                  (precision, i, A.shape[0], A.shape[1], k, eg, eo, abs(eg - eo) / eo))
            assert np.max(np.abs(U.T @ U - np.eye(k))) < 2e-5
            if precision == "fp32":
                tol = 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]
                assert np.all(np.abs(sig - ref.sigma) <= tol), (i, np.max(np.abs(sig - ref.sigma) / tol))
                assert abs(eg - eo) <= 1e-4 * eo, i
            else:
                assert eg <= 1.02 * eo, i
        del plan


def test_batched_mixed_error_against_oracle():
    probs = _problems(2, 5)
    As = [torch.from_numpy(A).to(DEV) for A, _, _ in probs]
    plan = rf.rf_svd_batched(As, [k for _, k, _ in probs], [l for _, _, l in probs], q=2, seeds=7,
                             precision="mixed")
    torch.cuda.synchronize()
    for i, (A, k, l) in enumerate(probs):
        ref = _oracle(A, k, l, 2, i, 7)
        A64 = A.astype(np.float64)
        U = plan.U[i].cpu().numpy().astype(np.float64)
        sig = plan.sigma[i].cpu().numpy()
        assert ev.frob_error(A64, U) <= 1.02 * ev.frob_error(A64, ref.U) + 1e-6 * np.linalg.norm(A64)
        assert np.all(np.abs(sig - ref.sigma) <= 2e-2 * ref.sigma + 1e-3 * ref.sigma[0])
        assert np.max(np.abs(U.T @ U - np.eye(k))) < 2e-5


def test_batched_problem0_matches_single_call():
    """Problem 0 of a batch draws the same sketch and Omega as rf_svd (index 0)."""
    probs = _problems(3, 3)
    As = [torch.from_numpy(A).to(DEV) for A, _, _ in probs]
    plan = rf.rf_svd_batched(As, [k for _, k, _ in probs], [l for _, _, l in probs], q=1, seeds=5,
                             precision="fp32")
    A, k, l = probs[0]
    U, sig, Vt, _ = rf.rf_svd(As[0], k, l, 1, 4, seed=5)
    torch.cuda.synchronize()
    s_b, s_1 = plan.sigma[0].cpu().numpy(), sig.cpu().numpy()
    assert np.all(np.abs(s_b - s_1) <= 1e-5 * s_1 + 2e-6 * s_1[0])


def test_graph_replays_match_direct_launches():
    probs = _problems(4, 6)
    As = [torch.from_numpy(A).to(DEV) for A, _, _ in probs]
    ks, ls = [k for _, k, _ in probs], [l for _, _, l in probs]
    direct = rf.BatchPlan(As, ks, ls, q=2, seeds=11, precision="mixed", use_graph=False).run()
    torch.cuda.synchronize()
    want = [(u.clone(), s.clone(), v.clone()) for u, s, v in zip(direct.U, direct.sigma, direct.Vt)]
    graph = rf.BatchPlan(As, ks, ls, q=2, seeds=11, precision="mixed", use_graph=True)
    for rep in range(3):
        for t in graph.U + graph.Vt:
            t.fill_(float("nan"))                    # eager work between replays
        graph.run()
        torch.cuda.synchronize()
        junk = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)
        torch.cuda.synchronize()
        del junk
        for i, (u, s, v) in enumerate(want):
            assert torch.equal(graph.U[i], u), (rep, i)
            assert torch.equal(graph.sigma[i], s), (rep, i)
            assert torch.equal(graph.Vt[i], v), (rep, i)


def test_batched_tiny_and_square_problems():
    rng = np.random.default_rng(9)
    shapes = [(70, 40, 5, 10), (64, 64, 16, 32), (300, 9, 2, 8), (129, 257, 30, 60)]
    As, ks, ls, refs = [], [], [], []
    for i, (m, n, k, l) in enumerate(shapes):
        r = min(m, n)
        A = synth.spectrum_matrix(m, n, np.exp(-0.2 * np.arange(r)), 50 + i).astype(np.float32)
        As.append(torch.from_numpy(A).to(DEV)); ks.append(k); ls.append(l)
        refs.append(_oracle(A, k, l, 1, i, 3))
    plan = rf.rf_svd_batched(As, ks, ls, q=1, seeds=3, precision="fp32")
    torch.cuda.synchronize()
    for i, ref in enumerate(refs):
        sig = plan.sigma[i].cpu().numpy()
        assert np.all(np.abs(sig - ref.sigma) <= 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]), i


def test_batched_rejects_unsupported():
    A = torch.zeros((100, 60), device=DEV)
    with pytest.raises(rf.RFError) as e:
        rf.BatchPlan([A, A], [4, 4], [8, 8], q=1, nnz_per_col=8)
    assert e.value.status == 3
    with pytest.raises(rf.RFError) as e:
        rf.BatchPlan([A], [10], [8], q=1)           # sketch < k
    assert e.value.status == 1
