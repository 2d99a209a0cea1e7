"""Brute-force measurement of the quantities in Section 3, for tiny inputs.

* spec_approx_eps(A, S, lam): smallest eps with
  (1-eps)(A A^T + lam I) <= A S S^T A^T + lam I <= (1+eps)(A A^T + lam I)
  (Definition 3.1), computed as || C S S^T C^T - C C^T ||_2 with
  C = (A A^T + lam I)^{-1/2} A (the normalised form used in the proof of
  Lemma 3.2, Appendix E.2).
* lam_tail(sv, k) = (1/k) sum_{i>k} sigma_i^2  (eq. defining lambda in Lemma 3.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
import numpy as np


def lam_tail(sv, k):
    sv = np.sort(np.asarray(sv, dtype=np.float64))[::-1]
    return float(np.sum(sv[k:] ** 2) / k)


def spec_approx_eps(A, S, lam):
    A = np.asarray(A, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    M = A @ A.T + lam * np.eye(A.shape[0])
    w, V = np.linalg.eigh(M)
    if np.min(w) <= 0:
        raise ValueError("A A^T + lam I must be positive definite (lam > 0 or full row rank)")
    Mih = V @ np.diag(w ** -0.5) @ V.T
    C = Mih @ A
    D = C @ S @ S.T @ C.T - C @ C.T
    return float(np.max(np.abs(np.linalg.eigvalsh(0.5 * (D + D.T)))))
