"""Error measures for low-rank approximations (float64).

* frob_error(A, Q): ||A - Q Q^T A||_F computed as ||A||_F^2 - 2 ||B||_F^2 +
  <B, G B> with B = Q^T A, G = Q^T Q (exact algebra, valid when Q is not
  exactly orthonormal).  The metric of the benchmark divides it by opt_F.
* opt_frob(sv, k): Eckart-Young optimum (sum_{i>k} sigma_i^2)^{1/2}.
* spectral_error(A, Q): ||(I - Q Q^T) A||_2 by power iteration on the residual
  operator (the error plotted in Section 4 is ||A - U Sigma V^T|| / sigma_{k+1} - 1,
  and with r2 = k, U Sigma V^T = Q Q^T A).

Pinned by tests/test_oracle_evaluate.py: the explicit residual for any Q
(orthonormal or not), LAPACK's 2-norm, and the Eckart-Young closed forms
(the truncated SVD leaves the spectrum tail in the Frobenius norm and
sigma_{k+1} in the spectral norm) on matrices of known spectrum.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
import numpy as np


def frob_error(A, Q):
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    B = Q.T @ A
    G = Q.T @ Q
    val = np.sum(A * A) - 2.0 * np.sum(B * B) + np.sum(B * (G @ B))
    return float(np.sqrt(max(val, 0.0)))


def frob_error_explicit(A, Q):
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(A - Q @ (Q.T @ A)))


def opt_frob(sv, k):
    sv = np.sort(np.asarray(sv, dtype=np.float64))[::-1]
    return float(np.sqrt(np.sum(sv[k:] ** 2)))


def spectral_error(A, Q, iters=200, seed=0):
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.shape[1])

    def res(v):
        y = A @ v
        return y - Q @ (Q.T @ y)

    def res_t(y):
        y = y - Q @ (Q.T @ y)
        return A.T @ y

    lam = 0.0
    for _ in range(iters):
        x = res_t(res(x))
        nrm = np.linalg.norm(x)
        if nrm == 0:
            return 0.0
        x /= nrm
        lam = np.linalg.norm(res(x))
    return float(lam)


def orth_error(Q):
    Q = np.asarray(Q, dtype=np.float64)
    G = Q.T @ Q - np.eye(Q.shape[1])
    return float(np.max(np.abs(np.linalg.eigvalsh(G)))) if G.size else 0.0
