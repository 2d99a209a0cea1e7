"""Pins for oracle/evaluate.py, the error measures every parity test and the
benchmark ratio go through.

Each measure is checked against a computation that shares none of its algebra
(the explicit residual, LAPACK's SVD-based 2-norm) and against closed forms
fixed by the Eckart-Young theorem (the error of the truncated SVD is the tail
of the spectrum, in the Frobenius and the spectral norm).  The matrices are
built with a known spectrum, so the expected values come from the generator's
sigma, not from the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import evaluate as ev


def known_spectrum(m, n, sigma, seed):
    """A = U diag(sigma) V^T with Haar U, V and its exact factors."""
    rng = np.random.default_rng(seed)
    r = len(sigma)
    U = synth.haar(m, r, rng)
    V = synth.haar(n, r, rng)
    return (U * sigma[None, :]) @ V.T, U, V


SIG = 2.0 ** -np.arange(40, dtype=np.float64)          # strong gaps: power iteration converges fast
SIG_POLY = np.arange(1, 41, dtype=np.float64) ** -1.0


@pytest.mark.parametrize("k", [1, 5, 17])
def test_frob_error_truncated_svd_is_spectrum_tail(k):
    """Eckart-Young: ||A - U_k U_k^T A||_F = (sum_{i>k} sigma_i^2)^{1/2}."""
    A, U, _ = known_spectrum(90, 60, SIG_POLY, 3)
    want = np.sqrt(np.sum(SIG_POLY[k:] ** 2))
    assert ev.frob_error(A, U[:, :k]) == pytest.approx(want, rel=1e-10)
    assert ev.frob_error_explicit(A, U[:, :k]) == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("kind", ["orthonormal", "scaled", "perturbed", "rank_deficient"])
def test_frob_error_equals_explicit_residual(kind):
    """The expanded form ||A||^2 - 2||B||^2 + <B, G B> equals the explicit
    residual ||A - Q Q^T A||_F for any Q, orthonormal or not (a dropped term,
    a wrong sign or factor, or G = I assumed would break the non-orthonormal
    cases)."""
    rng = np.random.default_rng(7)
    A, _, _ = known_spectrum(80, 50, SIG_POLY, 11)
    Q = synth.haar(80, 9, rng)
    if kind == "scaled":
        Q = Q * np.linspace(0.3, 1.7, 9)[None, :]
    elif kind == "perturbed":
        Q = Q + 0.05 * rng.standard_normal(Q.shape)
    elif kind == "rank_deficient":
        Q[:, 4] = Q[:, 2]
    got, want = ev.frob_error(A, Q), ev.frob_error_explicit(A, Q)
    assert got == pytest.approx(want, rel=1e-10)
    # an explicit loop over entries for the residual of the first case family
    R = A - Q @ (Q.T @ A)
    brute = np.sqrt(sum(R[i, j] ** 2 for i in range(R.shape[0]) for j in range(R.shape[1])))
    assert got == pytest.approx(brute, rel=1e-10)


def test_frob_error_of_full_basis_and_empty_basis():
    A, _, _ = known_spectrum(30, 20, SIG_POLY[:20], 5)
    rng = np.random.default_rng(1)
    full = synth.haar(30, 30, rng)
    assert ev.frob_error(A, full) <= 1e-12 * np.linalg.norm(A)
    assert ev.frob_error(A, np.zeros((30, 3))) == pytest.approx(np.sqrt(np.sum(SIG_POLY[:20] ** 2)), rel=1e-12)


@pytest.mark.parametrize("k", [0, 3, 25])
def test_opt_frob_matches_known_spectrum(k):
    A, _, _ = known_spectrum(70, 45, SIG_POLY, 2)
    sv = np.linalg.svd(A, compute_uv=False)
    want = np.sqrt(np.sum(SIG_POLY[k:] ** 2))
    assert ev.opt_frob(sv, k) == pytest.approx(want, rel=1e-10)
    # input order does not matter (the function sorts)
    assert ev.opt_frob(sv[::-1].copy(), k) == pytest.approx(want, rel=1e-10)
    assert ev.opt_frob(np.random.default_rng(0).permutation(sv), k) == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("k", [1, 4, 10])
def test_spectral_error_truncated_svd_is_next_singular_value(k):
    """Eckart-Young in the spectral norm: ||A - U_k U_k^T A||_2 = sigma_{k+1}."""
    A, U, _ = known_spectrum(60, 40, SIG, 4)
    assert ev.spectral_error(A, U[:, :k]) == pytest.approx(SIG[k], rel=1e-8)


def test_spectral_error_matches_lapack_two_norm_for_random_basis():
    rng = np.random.default_rng(12)
    A, _, _ = known_spectrum(70, 50, SIG, 9)
    Q = synth.haar(70, 6, rng)
    want = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    assert ev.spectral_error(A, Q, iters=400) == pytest.approx(want, rel=1e-8)
    # no basis at all: the error is ||A||_2 = sigma_1
    assert ev.spectral_error(A, np.zeros((70, 2))) == pytest.approx(SIG[0], rel=1e-8)


def test_orth_error_matches_two_norm_and_closed_forms():
    rng = np.random.default_rng(5)
    Q = synth.haar(40, 7, rng)
    P = Q + 1e-3 * rng.standard_normal(Q.shape)
    assert ev.orth_error(P) == pytest.approx(np.linalg.norm(P.T @ P - np.eye(7), 2), rel=1e-9)
    # c Q with orthonormal Q: Q^T Q - I = (c^2 - 1) I
    assert ev.orth_error(1.25 * Q) == pytest.approx(1.25 ** 2 - 1.0, rel=1e-12)
    assert ev.orth_error(Q) <= 1e-14
    # two unit vectors at angle theta: the eigenvalues of Q^T Q - I are +-cos(theta)
    th = 0.3
    two = np.array([[1.0, np.cos(th)], [0.0, np.sin(th)], [0.0, 0.0]])
    assert ev.orth_error(two) == pytest.approx(np.cos(th), rel=1e-12)
