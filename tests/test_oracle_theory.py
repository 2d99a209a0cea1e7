"""Deterministic statements of Section 3 checked by brute force on tiny inputs.

Each theorem is conditional on measured properties of the drawn matrices
(Definition 3.1 with a given lambda and eps).  We measure those properties
exactly and, whenever the hypotheses hold, assert the conclusions.  A mistake
in the oracle's range finder (a wrong power, a transposed operand, a lost
column) breaks these bounds on some seed.
"""
import math
import numpy as np
import pytest

import synth
from oracle import sketch as sk, methods as me, theory as th


def spectrum(m, n, seed, decay=1.0):
    sig = np.arange(1, min(m, n) + 1, dtype=np.float64) ** (-decay)
    return synth.spectrum_matrix(m, n, sig, seed), sig


def test_definition_3_1_normalised_form():
    """The normalised form ||C S S^T C^T - C C^T|| (Appendix E.2) equals the
    smallest eps of Definition 3.1 computed as a generalised eigenvalue
    problem."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((8, 12))
    S = rng.standard_normal((12, 30)) / math.sqrt(30)
    lam = 0.3
    eps = th.spec_approx_eps(A, S, lam)
    M = A @ A.T + lam * np.eye(8)
    N = A @ S @ S.T @ A.T + lam * np.eye(8)
    L = np.linalg.cholesky(M)
    Li = np.linalg.inv(L)
    g = np.linalg.eigvalsh(Li @ N @ Li.T)
    assert abs(eps - max(abs(g - 1))) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_lemma_3_3(seed):
    rng = np.random.default_rng(seed)
    m, n, k, r = 30, 25, 3, 20
    A, _ = spectrum(m, n, seed, decay=1.0)
    sv = np.linalg.svd(A, compute_uv=False)
    lam = th.lam_tail(sv, k)
    Om = rng.standard_normal((n, r)) / math.sqrt(r)
    eps = th.spec_approx_eps(A, Om, lam)
    Q, _ = me.orth(A @ Om)
    if eps <= 0.5:
        err2 = np.linalg.norm(A - Q @ (Q.T @ A), 2) ** 2
        errF2 = np.linalg.norm(A - Q @ (Q.T @ A)) ** 2
        assert err2 <= 2 * lam * (1 + 1e-10)
        bound = 2 * min(l * lam + np.sum(sv[l:] ** 2) for l in range(len(sv) + 1))
        assert errF2 <= bound * (1 + 1e-10)


def theorem_3_5_case(seed, q):
    rng = np.random.default_rng(100 + seed)
    m, n, k, l, r1, s = 24, 200, 2, 4, 150, 8
    A, _ = spectrum(m, n, seed, decay=1.0)
    sv = np.linalg.svd(A, compute_uv=False)
    table = sk.sketch_table(n, s, r1, seed=seed)
    S = sk.sketch_matrix(table, r1).toarray()
    lam1 = th.lam_tail(sv, l)
    eps = th.spec_approx_eps(A, S, lam1)
    At = A @ S
    B = At.copy()
    for _ in range(q):
        B = At @ (At.T @ B)
    r2 = 24
    Om = rng.standard_normal((r1, r2)) / math.sqrt(r2)
    svB = np.linalg.svd(B, compute_uv=False)
    lam2 = th.lam_tail(svB, k)
    eps2 = th.spec_approx_eps(B, Om, lam2)
    res = me.range_finder(A, me.Params(k=r2, l=r1, q=q, s=s, seed=seed), table=table, Om=Om)
    return A, sv, res.Q, eps, lam1, eps2, lam2


@pytest.mark.parametrize("q", [0, 1, 2])
def test_theorem_3_5(q):
    held = 0
    for seed in range(8):
        A, sv, Q, eps, lam1, eps2, lam2 = theorem_3_5_case(seed, q)
        if eps > 0.5 or eps2 > 0.5:
            continue
        held += 1
        R = A - Q @ (Q.T @ A)
        spec = np.linalg.norm(R, 2) ** 2
        frob = np.linalg.norm(R) ** 2
        e = 1.0 / (2 * q + 1)
        assert spec <= (1 + 2 * eps) * ((2 * lam2) ** e + eps * lam1) * (1 + 1e-9)
        fb = min(8 * r * (lam2 ** e + lam1) + np.sum(sv[r:] ** 2) for r in range(len(sv) + 1))
        assert frob <= fb * (1 + 1e-9)
    assert held >= 2, "hypotheses of Theorem 3.5 held on too few seeds to test it"


@pytest.mark.parametrize("seed", range(4))
def test_lemma_e1(seed):
    """Lemma E.1: for q >= log(2 m_hat)/(2 eps),
    (2/k sum_{i>k} sigma_i(AS)^{2(2q+1)})^{1/(2q+1)} <= (1+4eps) sigma_{k+1}^2 + 2 lam1 eps."""
    m, n, k, l, r1, s = 20, 300, 1, 3, 250, 8
    A, _ = spectrum(m, n, seed, decay=1.0)
    sv = np.linalg.svd(A, compute_uv=False)
    S = sk.sketch_matrix(sk.sketch_table(n, s, r1, seed=seed + 50), r1).toarray()
    lam1 = th.lam_tail(sv, l)
    eps = th.spec_approx_eps(A, S, lam1)
    assert 0 < eps <= 0.5, "hypothesis of Lemma E.1 not met; enlarge the sketch"
    sa = np.linalg.svd(A @ S, compute_uv=False)
    mhat = int(np.sum(sa > 1e-12 * sa[0]))
    q = int(math.ceil(math.log(2 * mhat) / (2 * eps)))
    p = 2 * q + 1
    # scale out sigma_{k+1} before taking the high power to stay in range
    c = sv[k]
    lhs = c ** 2 * ((2.0 / k) * np.sum((sa[k:] / c) ** (2 * p))) ** (1.0 / p)
    rhs = (1 + 4 * eps) * sv[k] ** 2 + 2 * lam1 * eps
    assert lhs <= rhs * (1 + 1e-9)
