"""Parity at the benchmark's full size and launch configuration: A 65536 x 16384
FP32, k = 1000, sketch 2000, 8 nonzeros per column, q = 1, seed 42 (the call
`bench.py` times).  The oracle runs once on the host in FP64 (about a minute).

The instance follows the benchmark's law (sigma_i = i^-1.5, Haar factors, Gaussian
noise of spectral size 1e-4 sigma_1) with the low-rank part truncated at rank 1200,
so that it is generated in seconds; the noise keeps A full rank.

Checked: sampled rows of A S and sampled columns of S2^T A element by element; the Ritz singular values (1e-5
relative plus the 2e-6 sigma_1 floor of FP32 B = Q^T A); the Frobenius error
||A - U U^T A||_F against the oracle's (1e-4 relative in the FP32 form, 2 % in the
mixed form); orthonormality of U."""
import math

import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
from oracle import methods as me, sketch as sk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24
M, N, K, L, S, Q, SEED = 65536, 16384, 1000, 2000, 8, 1, 42


@pytest.fixture(scope="module")
def instance():
    g = torch.Generator(device=DEV)
    g.manual_seed(2024)
    r = 1200
    sig = torch.arange(1, r + 1, device=DEV, dtype=torch.float64) ** -1.5
    U, R = torch.linalg.qr(torch.randn(M, r, generator=g, device=DEV, dtype=torch.float64))
    U *= torch.sign(torch.diagonal(R)).unsqueeze(0)
    V, R = torch.linalg.qr(torch.randn(N, r, generator=g, device=DEV, dtype=torch.float64))
    V *= torch.sign(torch.diagonal(R)).unsqueeze(0)
    A64 = (U * sig.unsqueeze(0)) @ V.t()
    del U, V, R
    A64 += (1e-4 / (math.sqrt(M) + math.sqrt(N))) * torch.randn(M, N, generator=g, device=DEV, dtype=torch.float64)
    A32 = A64.to(torch.float32)
    A64 = A32.double()            # the stored FP32 matrix is the problem instance
    torch.cuda.synchronize()
    ref = me.rand_svd(A64.cpu().numpy(), me.Params(k=K, l=L, q=Q, s=S, seed=SEED))
    return A32, A64, ref


def test_fullsize_sketch_left_columns(instance):
    """Sampled columns of S2^T A (Algorithm 2's second pass over A) at full size, in
    the launch configuration rf_lowrank uses; bound as for the small cases: the
    column's fixed-point grid (cnt_b c max_i |a_ij| 2^-29 / sqrt(s)) plus FP32
    rounding of the conversion, scale and row-split partials."""
    A32, A64, _ = instance
    got = rf.rf_sketch_apply_left(A32, L, S, SEED)
    cols = np.concatenate([np.random.default_rng(2).choice(N, 30, replace=False), [0, N - 1]])
    got = got[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    Ac = A64[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    table = sk.sketch_table(M, S, L, SEED, sk.STREAM_S2)
    S2 = sk.sketch_matrix(table, L)
    ref = me.sketch_left(Ac, table, L)
    mag = np.asarray(np.abs(S2.T) @ np.abs(Ac))
    cnt = np.bincount((table.astype(np.int64) & 0x7FFFFFFF).ravel(), minlength=L).astype(np.float64)
    tol = (cnt[:, None] * cnt.max() * np.max(np.abs(Ac), axis=0)[None, :] * 2.0 ** -29 / math.sqrt(S)
           + 72 * U32 * mag + 1e-30)
    err = np.abs(got - ref)
    print("left sketch columns: max err/tol %.3f" % np.max(err / tol))
    assert np.all(err <= tol)


def _frob_err(A64, Ud):
    """||A - U U^T A||_F in FP64 on the GPU (valid for non-orthonormal U)."""
    B = Ud.t() @ A64
    G = Ud.t() @ Ud
    val = float((A64 * A64).sum()) - 2.0 * float((B * B).sum()) + float((B * (G @ B)).sum())
    return math.sqrt(max(val, 0.0))


def test_fullsize_sketch_rows(instance):
    A32, A64, _ = instance
    got = rf.rf_sketch_apply(A32, L, S, SEED).cpu().numpy()
    rows = np.random.default_rng(1).choice(M, 96, replace=False)
    rows = np.concatenate([rows, [0, M - 1]])
    Ar = A64[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    table = sk.sketch_table(N, S, L, SEED)
    ref = me.sketch_right(Ar, table, L)
    mag = np.asarray(np.abs(Ar) @ np.abs(sk.sketch_matrix(table, L).toarray()))
    # FP32 summation bound plus the fixed-point grid of the pass: each term rounded to
    # at most c 2^-25 of its 2048-column chunk's band maximum (c = chunk occupancy,
    # band = the 8 rows sharing a workgroup); the band maximum is bounded here by the
    # largest |a| of the row's whole band
    buckets = table.astype(np.int64) & 0x7FFFFFFF
    bands = np.stack([A64[(i // 8) * 8:(i // 8) * 8 + 8].abs().cpu().numpy() for i in rows])  # (rows, 8, N)
    fx = np.zeros_like(ref)
    for c0 in range(0, N, 2048):
        cnt = np.zeros(L)
        for t in range(S):
            cnt += np.bincount(buckets[c0:c0 + 2048, t], minlength=L)
        band = bands[:, :, c0:c0 + 2048].max(axis=(1, 2))
        fx += (band * max(cnt.max(), 1.0) * 2.0 ** -25)[:, None] * cnt[None, :]
    tol = (N * S / L + 8) * 4 * U32 * mag + fx / math.sqrt(S) + 1e-30
    err = np.abs(got[rows] - ref)
    print("sketch rows: max err/tol %.3f" % np.max(err / tol))
    assert np.all(err <= tol)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_fullsize_svd(instance, precision):
    A32, A64, ref = instance
    U, sig, Vt, info = rf.rf_svd(A32, K, L, Q, S, SEED, precision)
    torch.cuda.synchronize()
    d = rf.info_dict(info)
    assert d["status"] == 0 and d["rank_found"] == K and d["nonfinite"] == 0
    sig = sig.cpu().numpy()
    Ud = U.double()
    e_gpu = _frob_err(A64, Ud)
    e_ref = _frob_err(A64, torch.from_numpy(ref.U).to(DEV))
    print("%s: ||A - UU^TA||_F gpu %.8e oracle %.8e (rel diff %.2e)" % (precision, e_gpu, e_ref,
                                                                          abs(e_gpu - e_ref) / e_ref))
    orth = float(torch.max(torch.abs(Ud.t() @ Ud - torch.eye(K, device=DEV, dtype=torch.float64))))
    assert orth < 2e-5
    assert np.all(np.diff(sig) <= 0)
    if precision == "fp32":
        tol = 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]
        print("max |dsigma|/tol = %.3f" % np.max(np.abs(sig - ref.sigma) / tol))
        assert np.all(np.abs(sig - ref.sigma) <= tol)
        assert abs(e_gpu - e_ref) <= 1e-4 * e_ref
    else:
        assert abs(e_gpu - e_ref) <= 2e-2 * e_ref


def test_fullsize_mixed_sigma_weyl_bound(instance):
    """Mixed form at full size: B = Q^T A is taken on BF16 MFMA with A and Q
    rounded to BF16 as they are loaded.  By Weyl's inequality its singular values
    differ from those of the exact Q^T A (FP64, the mixed form's own Q) by at
    most ||Q^T dA||_2 + ||dQ^T bf16(A)||_2 (dA, dQ the BF16 rounding errors) plus
    FP32 accumulation (~sqrt(m) u32 sigma_1); the FP64 Ritz step adds
    1e-5 sigma_i + 2e-6 sigma_1 at most, as in the FP32 form.  Q is the mixed
    range finder's output (the same kernels as inside rf_svd)."""
    A32, A64, _ = instance
    U, sig, Vt, info = rf.rf_svd(A32, K, L, Q, S, SEED, "mixed")
    Qm, _ = rf.rf_range_finder(A32, K, L, Q, S, SEED, "mixed")
    torch.cuda.synchronize()
    Qd = Qm.double()
    def svals(X):  # singular values of a wide k x n matrix from the FP64 eigenvalues of X X^T
        lam = torch.linalg.eigvalsh(X @ X.t()).clamp_min(0).sqrt()
        return torch.flip(lam, [0])
    B = Qd.t() @ A64
    exact = svals(B).cpu().numpy()
    Ab = A32.to(torch.bfloat16).double()
    dQ = Qd - Qm.to(torch.bfloat16).double()
    e1 = float(svals(Qd.t() @ (A64 - Ab))[0])
    e2 = float(svals(dQ.t() @ Ab)[0])
    acc = math.sqrt(M) * U32 * exact[0]
    sig = sig.cpu().numpy()
    tol = e1 + e2 + acc + 1e-5 * exact + 2e-6 * exact[0]
    d = np.abs(sig - exact)
    print("mixed sigma: ||Q^T dA|| %.3e ||dQ^T A|| %.3e  max |dsigma| %.3e  max |dsigma|/tol %.3f  "
          "max rel (top 100) %.2e" % (e1, e2, d.max(), np.max(d / tol), np.max(d[:100] / exact[:100])))
    assert np.all(d <= tol)
