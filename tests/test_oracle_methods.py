"""Pins for oracle/methods.py against facts the paper and linear algebra fix.

Every check compares the oracle with something other than itself: brute-force
loops, closed forms (Eckart-Young), special cases that reduce to textbook
routines (S = I gives the classical range finder, Section 2; S2 = I gives the
orthogonal projection), or exact identities from the proofs (Theorem 2.5).
"""
import math
import numpy as np
import pytest

import synth
from oracle import sketch as sk, methods as me, evaluate as ev


def identity_table(n):
    return np.arange(n, dtype=np.int32).reshape(n, 1)


def small(m=120, n=80, seed=1, decay=1.0, noise=0.0):
    sig = (np.arange(1, min(m, n) + 1, dtype=np.float64)) ** (-decay)
    return synth.lowrank_noise(m, n, sig, noise, seed)


def proj(Q):
    return Q @ Q.T


# ---- sketch application -------------------------------------------------------
@pytest.mark.parametrize("m,n,s,r1", [(5, 9, 3, 7), (4, 13, 1, 5), (6, 10, 4, 4)])
def test_sketch_right_bruteforce_integer(m, n, s, r1):
    """A S with integer A: the sums are exact, compare with a plain loop."""
    rng = np.random.default_rng(m * 100 + n)
    A = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
    t = sk.sketch_table(n, s, r1, seed=11)
    raw = [[0] * r1 for _ in range(m)]
    for i in range(m):
        for j in range(n):
            for tt in range(s):
                e = int(t[j, tt]) & 0xFFFFFFFF
                b, neg = e & 0x7FFFFFFF, e >> 31
                raw[i][b] += (-1 if neg else 1) * int(A[i, j])
    expect = np.array(raw, dtype=np.float64) / math.sqrt(s)
    got = me.sketch_right(A, t, r1)
    assert np.array_equal(got * math.sqrt(s), expect * math.sqrt(s)) or np.allclose(got, expect, rtol=0, atol=1e-12)


def test_sketch_left_bruteforce_integer():
    rng = np.random.default_rng(3)
    m, n, s, r1 = 11, 4, 2, 6
    A = rng.integers(-5, 6, size=(m, n)).astype(np.float64)
    t = sk.sketch_table(m, s, r1, seed=4, stream=sk.STREAM_S2)
    out = np.zeros((r1, n))
    bucket, sign = sk.decode_table(t)
    for i in range(m):
        for tt in range(s):
            out[bucket[i, tt]] += sign[i, tt] * A[i]
    assert np.allclose(me.sketch_left(A, t, r1), out / math.sqrt(s), atol=1e-12)


# ---- orth ---------------------------------------------------------------------------
def test_orth_properties():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((50, 12)) @ np.diag(np.logspace(0, -6, 12))
    Q, rank = me.orth(Y)
    assert rank == 12
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-13)
    R = Q.T @ Y
    assert np.allclose(np.tril(R, -1), 0, atol=1e-12)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(Q @ R, Y, atol=1e-13)
    # uniqueness: Q from the Cholesky factor of Y^T Y is the same matrix
    L = np.linalg.cholesky(Y.T @ Y)
    Qc = Y @ np.linalg.inv(L.T)
    assert np.allclose(Qc, Q, atol=1e-6)


def test_orth_rank_deficient_contains_range():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 8))
    Q, rank = me.orth(Y)
    assert rank == 3
    assert np.allclose(Q.T @ Q, np.eye(8), atol=1e-12)
    assert np.linalg.norm(Y - proj(Q) @ Y) < 1e-12 * np.linalg.norm(Y)


# ---- Algorithm 1 ------------------------------------------------------------------------
@pytest.mark.parametrize("q", [0, 1, 3])
def test_eckart_young_lower_bound(q):
    A = small(150, 90, seed=3, decay=0.7, noise=1e-3)
    sv = np.linalg.svd(A, compute_uv=False)
    k = 10
    res = me.range_finder(A, me.Params(k=k, l=40, q=q, s=4, seed=5))
    assert np.allclose(res.Q.T @ res.Q, np.eye(k), atol=1e-13)
    assert ev.frob_error(A, res.Q) >= ev.opt_frob(sv, k) * (1 - 1e-12)
    assert ev.spectral_error(A, res.Q) >= sv[k] * (1 - 1e-6)


@pytest.mark.parametrize("q", [0, 2])
def test_exact_recovery_rank_le_k(q):
    rng = np.random.default_rng(8)
    m, n, r, k = 100, 70, 6, 10
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    res = me.range_finder(A, me.Params(k=k, l=30, q=q, s=3, seed=2))
    assert ev.frob_error_explicit(A, res.Q) <= 1e-12 * np.linalg.norm(A)


def test_q0_span_is_A_S_Omega():
    A = small(60, 50, seed=4)
    p = me.Params(k=7, l=20, q=0, s=2, seed=3)
    res = me.range_finder(A, p)
    Y = A @ sk.sketch_matrix(res.extras["table"], p.l).toarray() @ res.extras["Omega"]
    Qy, _ = np.linalg.qr(Y)
    assert np.allclose(proj(res.Q), proj(Qy), atol=1e-10)


@pytest.mark.parametrize("q", [1, 2])
def test_power_schedule_matches_unorthonormalised_formula(q):
    """Re-orthonormalisation leaves span((At At^T)^q At Omega) unchanged
    (remark after Algorithm 1); check against the formula evaluated directly on
    a well-conditioned tiny case."""
    A = small(40, 30, seed=6, decay=0.3)
    p = me.Params(k=4, l=12, q=q, s=2, seed=8)
    res = me.range_finder(A, p)
    At = res.At
    Y = At @ res.extras["Omega"]
    for _ in range(q):
        Y = At @ (At.T @ Y)
    Qy, _ = np.linalg.qr(Y)
    assert np.allclose(proj(res.Q), proj(Qy), atol=1e-8)


def tan_max_angle(Uk, Q):
    c = np.linalg.svd(Uk.T @ Q, compute_uv=False).min()
    sin = np.linalg.norm(Uk - Q @ (Q.T @ Uk), 2)       # accurate for small angles
    return sin / c


def gapped(m, n, k, seed):
    sig = np.concatenate([np.linspace(10, 6, k), 0.5 * np.linspace(1, 0.1, n - k)])
    return synth.spectrum_matrix(m, n, sig, seed)


def test_classical_reduction_converges_to_truncated_svd():
    """S = I is the classical range finder (Section 2).  Subspace iteration
    obeys tan theta(U_k, Q_q) <= (sigma_{k+1}/sigma_k)^(2q) tan theta(U_k, Q_0)
    (textbook bound), and the Ritz values converge to sigma_1..sigma_k."""
    rng = np.random.default_rng(10)
    m, n, k = 80, 60, 5
    A = gapped(m, n, k, 12)
    U, sv, _ = np.linalg.svd(A, full_matrices=False)
    Uk = U[:, :k]
    Om = rng.standard_normal((n, k))
    tans = []
    for q in range(0, 5):
        res = me.range_finder(A, me.Params(k=k, l=n, q=q, s=1, seed=0), table=identity_table(n), Om=Om)
        tans.append(tan_max_angle(Uk, res.Q))
    rho = (sv[k] / sv[k - 1]) ** 2
    for q in range(1, 5):
        assert tans[q] <= rho ** q * tans[0] * (1 + 1e-6) + 1e-13
    assert tans[-1] < 1e-6
    res = me.rand_svd(A, me.Params(k=k, l=n, q=8, s=1, seed=0), table=identity_table(n), Om=Om)
    assert np.allclose(res.sigma, sv[:k], rtol=1e-10)


def test_classical_form_equals_identity_sketch():
    """classical=True (At = A, Omega n x k) is Algorithm 1 with S = I_n: the
    identity table with r1 = n, s = 1 gives At = A exactly in FP64, so the two
    paths agree to rounding, for the range finder, RandSVD and Algorithm 2
    with S1 = I."""
    A = small(70, 40, seed=21, decay=0.8)
    n = A.shape[1]
    for q in (0, 2):
        p_cl = me.Params(k=6, l=12, q=q, s=3, seed=9)
        cl = me.range_finder(A, p_cl, classical=True)
        Om = sk.omega(n, 6, 9)
        via = me.range_finder(A, me.Params(k=6, l=n, q=q, s=1, seed=9), table=identity_table(n), Om=Om)
        assert np.array_equal(cl.extras["Omega"], Om)
        assert np.allclose(cl.Q, via.Q, atol=1e-12)
        sv = me.rand_svd(A, p_cl, classical=True)
        assert np.allclose(sv.sigma, np.linalg.svd(via.Q.T @ A, compute_uv=False), rtol=1e-12)
    lr = me.lowrank(A, me.Params(k=6, l=12, q=1, s=3, seed=9), classical=True)
    P, T = lr.extras["P"], lr.extras["T"]
    assert P.shape == (12, 6) and T.shape == (12, n)
    assert np.allclose(P.T @ (P @ lr.X - T), 0, atol=1e-10)


def test_sketched_converges_to_top_subspace_of_At():
    """With a sparse S the iteration converges to the top-k left singular
    subspace of At = A S, not of A (proof sketch of Theorem 3.5, Section 3.1;
    the error plateau of Section 4)."""
    A = gapped(90, 70, 5, 13)
    p = me.Params(k=5, l=20, q=40, s=2, seed=14)
    res = me.range_finder(A, p)
    Ua, sa, _ = np.linalg.svd(res.At, full_matrices=False)
    assert sa[5] / sa[4] < 0.5
    assert tan_max_angle(Ua[:, :5], res.Q) < 1e-10
    Uk = np.linalg.svd(A, full_matrices=False)[0][:, :5]
    assert tan_max_angle(Uk, res.Q) > 1e-6          # ... and not to that of A


def test_scale_invariance():
    A = small(70, 50, seed=15, noise=1e-3)
    p = me.Params(k=6, l=20, q=2, s=3, seed=16)
    r1 = me.rand_svd(A, p)
    r2 = me.rand_svd(1000.0 * A, p)
    assert np.allclose(r1.Q, r2.Q, atol=1e-10)
    assert np.allclose(1000.0 * r1.sigma, r2.sigma, rtol=1e-10)


# ---- randomised SVD ---------------------------------------------------------------------------
def test_rand_svd_identities():
    A = small(100, 60, seed=17, decay=0.8, noise=1e-2)
    p = me.Params(k=8, l=30, q=1, s=4, seed=18)
    r = me.rand_svd(A, p)
    assert np.allclose((r.U * r.sigma) @ r.Vt, proj(r.Q) @ A, atol=1e-12)
    assert np.allclose(r.U.T @ r.U, np.eye(8), atol=1e-12)
    assert np.allclose(r.Vt @ r.Vt.T, np.eye(8), atol=1e-12)
    assert np.all(np.diff(r.sigma) <= 0)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.all(r.sigma <= sv[:8] * (1 + 1e-12))             # interlacing of Q^T A
    assert np.allclose(r.sigma, np.linalg.svd(r.Q.T @ A, compute_uv=False), rtol=1e-12)
    big = np.argmax(np.abs(r.U), axis=0)
    assert np.all(r.U[big, np.arange(8)] > 0)


# ---- Algorithm 2 -------------------------------------------------------------------------
def test_lowrank_s2_identity_is_projection():
    A = small(50, 40, seed=19, noise=1e-3)
    p = me.Params(k=6, l=50, q=1, s=1, seed=20)
    t1 = sk.sketch_table(40, 1, 50, seed=20)
    r = me.lowrank(A, p, table1=t1, table2=identity_table(50))
    assert np.allclose(r.Q @ r.X, proj(r.Q) @ A, atol=1e-12)


def test_lowrank_normal_equations():
    A = small(90, 60, seed=21, noise=1e-3)
    p = me.Params(k=6, l=24, q=2, s=3, seed=22)
    r = me.lowrank(A, p)
    P, T = r.extras["P"], r.extras["T"]
    assert np.allclose(P.T @ (P @ r.X - T), 0, atol=1e-10)
    # and it is at least as good as the optimum and not absurdly worse
    sv = np.linalg.svd(A, compute_uv=False)
    err = np.linalg.norm(A - r.Q @ r.X)
    assert err >= ev.opt_frob(sv, 6) * (1 - 1e-12)


# ---- Algorithm 3 -------------------------------------------------------------------------
@pytest.mark.parametrize("q", [0, 1, 3])
def test_nystrom_identity_theorem_2_5(q):
    """C W^+ C^T = A^{1/2} Q Q^T A^{1/2}, Q = Algorithm 1 on A^{1/2} with the
    same S and Omega (proof of Theorem 2.5)."""
    n = 40
    lam = np.concatenate([np.logspace(0, -3, 20), np.zeros(n - 20)])
    A = synth.psd_from_spectrum(n, lam, 23)
    w, V = np.linalg.eigh(A)
    Ah = (V * np.sqrt(np.maximum(w, 0))[None, :]) @ V.T
    p = me.Params(k=5, l=15, q=q, s=2, seed=24)
    nys = me.nystrom(A, p)
    rf = me.range_finder(Ah, p, table=nys.extras["table"], Om=nys.extras["Omega"])
    Ahat = nys.F @ nys.F.T
    assert np.allclose(Ahat, Ah @ proj(rf.Q) @ Ah, atol=1e-10)
    ev_ = np.linalg.eigvalsh(A - Ahat)
    assert ev_.min() > -1e-10                    # A - Ahat >= 0
    assert np.linalg.eigvalsh(Ahat).min() > -1e-12
    # ||A - Ahat|| = ||(I - Q Q^T) A^{1/2}||^2
    lhs = np.linalg.norm(A - Ahat, 2)
    rhs = np.linalg.norm(Ah - proj(rf.Q) @ Ah, 2) ** 2
    assert abs(lhs - rhs) < 1e-10


@pytest.mark.parametrize("family", ["rademacher", "gaussian", "srht"])
def test_dense_families_algorithm_1(family):
    """Algorithm 1 with the dense sketches of Lemma 3.2 (items 1 and 3): exact
    recovery for rank(A) <= k, the q = 0 span is that of A S Omega, and the
    Eckart-Young lower bound holds."""
    rng = np.random.default_rng(4)
    m, n, r, k, l = 90, 70, 5, 8, 20
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    p = me.Params(k=k, l=l, q=1, s=1, seed=6)
    res = me.range_finder(A, p, family=family)
    assert ev.frob_error_explicit(A, res.Q) <= 1e-10 * np.linalg.norm(A)
    B = small(60, 50, seed=3, decay=0.7)
    p0 = me.Params(k=6, l=16, q=0, s=1, seed=2)
    res0 = me.range_finder(B, p0, family=family)
    S = me.sketch_dense_family(50, p0, family)
    Y = B @ S @ res0.extras["Omega"]
    assert np.allclose(proj(res0.Q), proj(np.linalg.qr(Y)[0]), atol=1e-10)
    sv = np.linalg.svd(B, compute_uv=False)
    assert ev.frob_error(B, res0.Q) >= ev.opt_frob(sv, 6) * (1 - 1e-12)
