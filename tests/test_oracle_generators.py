"""Pins for the oracle's random draws (sketch S and Gaussian Omega).

The paper fixes the distribution of S -- s nonzeros +-1/sqrt(s) per row at
random positions (Lemma 3.2, item 2) -- and that Omega is Gaussian (Algorithm 1,
Theorem 2.1); it fixes no generator.  So the pins here are the distributional
properties: structure, uniformity, sign balance, isotropy E[S S^T] = I, normal
moments and a Kolmogorov-Smirnov test, and independence across streams.
The exact Philox bit stream is "parity unpinned" against an external vector.
"""
import math
import numpy as np
import pytest
from scipy import stats

from oracle import sketch as sk


@pytest.mark.parametrize("n,s,r1", [(1, 1, 1), (7, 3, 10), (500, 8, 2000), (1000, 1, 37), (300, 4, 4)])
def test_table_structure(n, s, r1):
    t = sk.sketch_table(n, s, r1, seed=123)
    assert t.shape == (n, s) and t.dtype == np.int32
    bucket, sign = sk.decode_table(t)
    lo = sk.block_bounds(r1, s)
    for tt in range(s):
        assert np.all(bucket[:, tt] >= lo[tt]) and np.all(bucket[:, tt] < lo[tt + 1])
    # s distinct buckets per row (one per block)
    assert all(len(set(row)) == s for row in bucket.tolist())
    assert set(np.unique(sign)) <= {-1.0, 1.0}
    S = sk.sketch_matrix(t, r1).toarray()
    assert np.allclose(np.sum(S != 0, axis=1), s)
    assert np.allclose(np.abs(S[S != 0]), 1.0 / math.sqrt(s))


def test_table_deterministic_and_stream_dependent():
    a = sk.sketch_table(4096, 8, 2000, seed=9)
    b = sk.sketch_table(4096, 8, 2000, seed=9)
    assert np.array_equal(a, b)
    for other in (sk.sketch_table(4096, 8, 2000, seed=10),
                  sk.sketch_table(4096, 8, 2000, seed=9, stream=2),
                  sk.sketch_table(4096, 8, 2000, seed=9, b=1),
                  sk.sketch_table(4096, 8, 2000, seed=9 + (1 << 32))):
        # independent draws agree on a bucket only with probability ~ 1/w
        frac = np.mean((a & 0x7FFFFFFF) == (other & 0x7FFFFFFF))
        assert frac < 0.02


def test_bucket_uniformity_chi2_and_sign_balance():
    n, s, r1 = 200_000, 4, 400
    t = sk.sketch_table(n, s, r1, seed=2024)
    bucket, sign = sk.decode_table(t)
    lo = sk.block_bounds(r1, s)
    for tt in range(s):
        w = lo[tt + 1] - lo[tt]
        counts = np.bincount(bucket[:, tt] - lo[tt], minlength=w)
        chi2 = np.sum((counts - n / w) ** 2 / (n / w))
        p = stats.chi2.sf(chi2, w - 1)
        assert p > 1e-4, (tt, chi2, p)
    frac_neg = np.mean(sign < 0)
    assert abs(frac_neg - 0.5) < 5 * 0.5 / math.sqrt(sign.size)


def test_sketch_isotropy():
    """E[S S^T] = I_n for a CountSketch-type S (each row has unit norm; distinct
    rows have independent random signs)."""
    n, s, r1, T = 12, 3, 9, 4000
    acc = np.zeros((n, n))
    for seed in range(T):
        S = sk.sketch_matrix(sk.sketch_table(n, s, r1, seed=seed), r1).toarray()
        acc += S @ S.T
    acc /= T
    assert np.allclose(np.diag(acc), 1.0)
    off = acc - np.diag(np.diag(acc))
    assert np.max(np.abs(off)) < 5.0 / math.sqrt(T)


def test_gaussian_moments_and_ks():
    z = sk.gaussian(500, 401, seed=77).ravel()          # odd count: ragged last counter
    assert z.size == 500 * 401
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-4
    z2 = sk.gaussian(500, 401, seed=77, stream=3).ravel()
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 / math.sqrt(z.size)
    # pairs from one Box-Muller draw are uncorrelated
    zz = sk.gaussian(1, 400_000, seed=5).ravel()
    assert abs(np.corrcoef(zz[0::2], zz[1::2])[0, 1]) < 0.01


def test_gaussian_prefix_consistency():
    """Entry e depends only on (seed, stream, b, e): a larger matrix with the
    same column count extends a smaller one."""
    a = sk.gaussian(10, 7, seed=3)
    b = sk.gaussian(20, 7, seed=3)
    assert np.array_equal(a, b[:10])


# ---- Lemma 3.2 items 1 and 3: dense sub-Gaussian sketches and the SRHT ----------
def _fwht_recursive(x):
    """Walsh-Hadamard transform by the textbook recursion H_2n = [[H, H], [H, -H]]
    (written out independently of scipy's hadamard)."""
    x = list(x)
    if len(x) == 1:
        return x
    h = len(x) // 2
    a, b = _fwht_recursive(x[:h]), _fwht_recursive(x[h:])
    return [u + v for u, v in zip(a, b)] + [u - v for u, v in zip(a, b)]


def test_dense_rademacher_structure():
    n, r1 = 300, 40
    S = sk.dense_sketch(n, r1, 7, "rademacher")
    assert np.all(np.abs(np.abs(S) - 1 / np.sqrt(r1)) < 1e-15)
    # every row has squared norm exactly 1 (diag of S S^T), the signs balance
    assert np.allclose(np.sum(S * S, axis=1), 1.0, atol=1e-12)
    assert abs(np.mean(np.sign(S))) < 4 / np.sqrt(n * r1)
    # independent of the sparse sketch's stream and of other seeds
    assert not np.array_equal(S, sk.dense_sketch(n, r1, 8, "rademacher"))
    off = (S @ S.T)[~np.eye(n, dtype=bool)]
    assert abs(off.mean()) < 3 / np.sqrt(r1 * n) and 0.5 / r1 < off.var() < 2 / r1


def test_dense_gaussian_moments():
    from scipy import stats
    n, r1 = 400, 50
    S = sk.dense_sketch(n, r1, 3, "gaussian") * np.sqrt(r1)
    assert abs(S.mean()) < 4 / np.sqrt(S.size) and abs(S.var() - 1) < 0.05
    assert stats.kstest(S.ravel(), "norm").pvalue > 1e-3


@pytest.mark.parametrize("n", [1, 2, 8, 64])
def test_hadamard_matches_recursive_walsh_hadamard(n):
    """x^T H (the oracle's H) equals the recursive transform of x."""
    import scipy.linalg as sla
    x = np.random.default_rng(n).standard_normal(n)
    assert np.allclose(x @ sla.hadamard(n), _fwht_recursive(x), atol=1e-12)


@pytest.mark.parametrize("bits", [2, 4, 6])
def test_feistel_is_a_permutation(bits):
    v = sk._feistel(np.arange(1 << bits, dtype=np.uint64), bits, 11, 0)
    assert sorted(v.tolist()) == list(range(1 << bits))


@pytest.mark.parametrize("n,r1", [(100, 20), (128, 128), (1000, 300), (5, 3)])
def test_srht_draws_structure(n, r1):
    d, picks = sk.srht_draws(n, r1, 5)
    n2 = sk.srht_size(n)
    assert n2 >= n and n2 & (n2 - 1) == 0 and n2 < 2 * max(n, 1)
    assert len(d) == n2 and set(np.unique(d)) <= {-1.0, 1.0}
    assert len(picks) == r1 and len(set(picks.tolist())) == r1
    assert np.all(np.diff(picks) > 0) and picks[0] >= 0 and picks[-1] < n2


def test_srht_columns_orthogonal():
    """S^T S = (n'/r1) I exactly when n = n' (H H^T = n' I, D^2 = I)."""
    S = sk.srht_matrix(256, 40, 3)
    assert np.allclose(S.T @ S, (256 / 40) * np.eye(40), atol=1e-12)
    # and S is isotropic: S S^T has expectation I (its trace is exactly n' * r1 / r1 ... = 256)
    assert np.isclose(np.trace(S @ S.T), 256.0)


def test_srht_subset_is_uniform():
    """Each index of [0, n') is picked with probability r1/n' (chi-squared over seeds)."""
    n, r1, trials = 64, 16, 400
    cnt = np.zeros(n)
    for sd in range(trials):
        cnt[sk.srht_draws(n, r1, 1000 + sd)[1]] += 1
    exp = trials * r1 / n
    chi2 = np.sum((cnt - exp) ** 2 / exp)
    assert chi2 < n + 5 * np.sqrt(2 * n)
