"""The paper's algorithms, written out plainly in float64.

* range_finder  -- Algorithm 1 (Sketch-Powered Range Finder), Section 2:
                   Q = orth((At At^T)^q At Omega), At = A S.
* rand_svd      -- the randomised SVD finisher of Section 2 ("Sketch-Powered
                   Low-Rank Factorization" paragraph): B = Q^T A = Ub Sigma V^T,
                   U = Q Ub; used in Section 4 with r1 = l, r2 = k.
* lowrank       -- Algorithm 2 (Sketch-Powered Low-Rank Factorization):
                   X = (S2^T Y)^+ (S2^T A).
* nystrom       -- Algorithm 3 (Sketch-Powered Nystrom Approximation):
                   Ct = A S, Wt = S^T A S, Y = Wt^q Omega, C = Ct Y, W = Y^T Wt Y.

Readings (also in the design doc):
* re-orthonormalisation: the paper omits it from Algorithm 1 "for simplicity"
  and notes it leaves the output unchanged in exact arithmetic (remark after
  Algorithm 1).  The oracle uses subspace iteration: Q0 = orth(At Omega), then
  for each power step Z = orth(At^T Q), Q = orth(At Z).  Algorithm 3 likewise
  uses Y_j = orth(Wt Y_{j-1}).
* orth(Y) is the Q factor of the Householder QR of Y with the signs fixed so
  that diag(R) >= 0.  For full-rank Y this Q is unique, so any correct QR
  (CholeskyQR on the GPU) gives the same matrix up to rounding; for
  rank-deficient Y it is still an orthonormal basis containing range(Y)
  (definition of orth in the Notation paragraph, Section 1).
* Algorithm 2 returns Q = orth(Y) instead of Y (Y X is unchanged under Y -> Y M
  for invertible M) and solves the least-squares problem by LAPACK lstsq.
* Algorithm 3: W^+ by eigh with eigenvalues <= r2 * eps * lambda_max dropped;
  F = C V_+ Lambda_+^{-1/2} so that C W^+ C^T = F F^T.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from dataclasses import dataclass, field
import numpy as np

from . import sketch as sk

EPS64 = np.finfo(np.float64).eps


@dataclass
class Params:
    k: int              # target rank r2
    l: int              # sketch size r1
    q: int = 0          # power steps
    s: int = 8          # nonzeros per row of S
    seed: int = 0
    b: int = 0          # matrix index inside a batch


@dataclass
class Result:
    Q: np.ndarray = None
    U: np.ndarray = None
    sigma: np.ndarray = None
    Vt: np.ndarray = None
    X: np.ndarray = None
    C: np.ndarray = None
    W: np.ndarray = None
    F: np.ndarray = None
    At: np.ndarray = None
    rank_found: int = 0
    extras: dict = field(default_factory=dict)


def orth(Y):
    """Orthonormal basis of range(Y) with the sign convention diag(R) >= 0.

    Returns (Q, rank) where rank counts singular values of Y above
    r2 * eps * sigma_1 (informational; Q always has Y.shape[1] columns)."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d[None, :]
    sv = np.linalg.svd(Y, compute_uv=False)
    rank = int(np.sum(sv > Y.shape[1] * EPS64 * (sv[0] if sv.size else 0.0))) if sv.size and sv[0] > 0 else 0
    return Q, rank


def sketch_right(A, table, r1):
    """At = A S (Algorithm 1, line 1): one pass over A with the sparse S."""
    S = sk.sketch_matrix(table, r1)
    return np.asarray((S.T @ A.T).T)


def sketch_left(A, table, r1):
    """S2^T A for an m x r1 sketch S2 given by its (m x s) table (Algorithm 2)."""
    S2 = sk.sketch_matrix(table, r1)
    return np.asarray(S2.T @ A)


def draws(shape_n, p: Params, table=None, Om=None):
    table = sk.sketch_table(shape_n, p.s, p.l, p.seed, sk.STREAM_S1, p.b) if table is None else table
    Om = sk.omega(p.l, p.k, p.seed, p.b) if Om is None else Om
    return table, Om


def power_loop(At, Om, q):
    """Subspace iteration for orth((At At^T)^q At Om)."""
    Q, rank = orth(At @ Om)
    for _ in range(q):
        Z, _ = orth(At.T @ Q)
        Q, rank = orth(At @ Z)
    return Q, rank


def sketch_dense_family(n, p: Params, family):
    """S of a dense family of Lemma 3.2 (item 1: "rademacher" / "gaussian";
    item 3: "srht") as an n x r1 matrix, drawn from p.seed."""
    if family in ("rademacher", "gaussian"):
        return sk.dense_sketch(n, p.l, p.seed, family, p.b)
    if family == "srht":
        return sk.srht_matrix(n, p.l, p.seed, p.b)
    raise ValueError(family)


def range_finder(A, p: Params, table=None, Om=None, classical=False, family="sparse"):
    """Algorithm 1.  Pinned by: Eckart-Young lower bound, exact recovery for
    rank(A) <= k, q = 0 span identity, S = I reduction to the classical range
    finder and its convergence to the truncated SVD, convergence to the top-k
    left singular subspace of At for sketched S, Lemma 3.3 / Theorem 3.5
    on tiny inputs (tests/test_oracle_methods.py, tests/test_oracle_theory.py).

    classical=True takes S = I (Section 2, "Comparison with Classical Range
    Finder"): At = A and Omega is n x k (drawn from the Omega stream with n rows
    unless given); p.l is then unused here."""
    A = np.asarray(A, dtype=np.float64)
    if classical:
        Om = sk.omega(A.shape[1], p.k, p.seed, p.b) if Om is None else Om
        Q, rank = power_loop(A, Om, p.q)
        return Result(Q=Q, At=A, rank_found=rank, extras={"table": None, "Omega": Om})
    if family != "sparse":
        # Lemma 3.2 items 1 and 3: the same Algorithm 1 with a dense S
        Om = sk.omega(p.l, p.k, p.seed, p.b) if Om is None else Om
        At = A @ sketch_dense_family(A.shape[1], p, family)
        Q, rank = power_loop(At, Om, p.q)
        return Result(Q=Q, At=At, rank_found=rank, extras={"table": None, "Omega": Om})
    table, Om = draws(A.shape[1], p, table, Om)
    At = sketch_right(A, table, p.l)
    Q, rank = power_loop(At, Om, p.q)
    return Result(Q=Q, At=At, rank_found=rank, extras={"table": table, "Omega": Om})


def svd_sign_fix(U, Vt):
    """R9 convention: flip (u_i, v_i) so that the entry of largest |.| of u_i is
    positive (lowest index on ties)."""
    idx = np.argmax(np.abs(U), axis=0)
    sgn = np.sign(U[idx, np.arange(U.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn[None, :], Vt * sgn[:, None]


def rand_svd(A, p: Params, table=None, Om=None, classical=False, family="sparse"):
    """Randomised SVD on top of Algorithm 1 (Section 2; Section 4 protocol).
    Pinned by: U Sigma V^T = Q Q^T A, sigma_i(B) <= sigma_i(A) (interlacing),
    orthonormality of U and V."""
    A = np.asarray(A, dtype=np.float64)
    res = range_finder(A, p, table, Om, classical, family)
    B = res.Q.T @ A
    Ub, sig, Vt = np.linalg.svd(B, full_matrices=False)
    U = res.Q @ Ub
    U, Vt = svd_sign_fix(U, Vt)
    res.U, res.sigma, res.Vt = U, sig, Vt
    res.extras["B"] = B
    return res


def lowrank(A, p: Params, table1=None, Om=None, table2=None, classical=False, family="sparse"):
    """Algorithm 2.  Pinned by: S2 = I reduces Y X to Q Q^T A; the normal
    equations (S2^T Q)^T (S2^T Q X - S2^T A) = 0.  classical=True runs it with
    S1 = I (the baseline of the additional experiments); S2 keeps p.l rows."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    res = range_finder(A, p, table1, Om, classical, family)
    if table2 is None:
        table2 = sk.sketch_table(m, p.s, p.l, p.seed, sk.STREAM_S2, p.b)
    P = sketch_left(res.Q, table2, p.l)
    T = sketch_left(A, table2, p.l)
    X, *_ = np.linalg.lstsq(P, T, rcond=None)
    res.X = X
    res.extras.update({"table2": table2, "P": P, "T": T})
    return res


def nystrom(A, p: Params, table=None, Om=None):
    """Algorithm 3 for a PSD A (n x n).  Pinned by the identity used in the
    proof of Theorem 2.5: C W^+ C^T = A^{1/2} Q Q^T A^{1/2} with Q from
    Algorithm 1 run on A^{1/2} with the same S and Omega, and by
    0 <= C W^+ C^T <= A."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    table, Om = draws(n, p, table, Om)
    Ct = sketch_right(A, table, p.l)                    # A S
    S = sk.sketch_matrix(table, p.l)
    Wt = np.asarray(S.T @ Ct)                           # S^T A S
    Wt = 0.5 * (Wt + Wt.T)
    Y = Om.copy()
    for _ in range(p.q):
        Y, _ = orth(Wt @ Y)
    C = Ct @ Y
    W = Y.T @ Wt @ Y
    W = 0.5 * (W + W.T)
    lam, V = np.linalg.eigh(W)
    keep = lam > W.shape[0] * EPS64 * max(lam.max(), 0.0)
    F = C @ (V[:, keep] / np.sqrt(lam[keep])[None, :]) if np.any(keep) else np.zeros((n, 0))
    return Result(C=C, W=W, F=F, At=Ct, rank_found=int(keep.sum()),
                  extras={"table": table, "Omega": Om, "Wt": Wt, "Y": Y})
