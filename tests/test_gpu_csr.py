"""Sparse A in CSR form (the nnz(A) costs of Theorems 2.1 and 2.5): the sketch
pass of a CSR matrix element by element against the oracle's A S on the same
matrix, and Algorithm 1 / RandSVD end to end against the FP64 oracle run on the
dense copy of the same matrix (the same linear operator)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_2605_09755_amd as rf
from oracle import methods as me, evaluate as ev, sketch as sk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24


def graded_sparse(m, n, density, seed, decay=1.0):
    """D1 R D2 with R sparse Gaussian and D1, D2 diagonal, decaying: sparse, with a
    decaying spectrum."""
    rng = np.random.default_rng(seed)
    R = sp.random(m, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    d1 = np.arange(1, m + 1) ** -(0.5 * decay)
    d2 = np.arange(1, n + 1) ** -(0.5 * decay)
    A = (sp.diags(d1) @ R @ sp.diags(d2)).tocsr()
    A.data = A.data.astype(np.float32).astype(np.float64)
    A.sort_indices()
    return A


@pytest.mark.parametrize("m,n,dens,s,r1", [(300, 900, 0.02, 8, 100), (64, 5000, 0.1, 4, 640), (500, 200, 0.005, 1, 37),
                                           (40, 3000, 0.5, 16, 2000)])
def test_sketch_csr_elementwise(m, n, dens, s, r1):
    A = graded_sparse(m, n, dens, m + n)
    t = sk.sketch_table(n, s, r1, 4)
    ref = me.sketch_right(A.toarray(), t, r1)
    got = rf.rf_sketch_apply_csr(rf.Csr.from_scipy(A, DEV), r1, s, 4).cpu().numpy()
    # exact 64-bit fixed-point sums: per term 2^-(60 - log2 nnz_row) of the row max,
    # then one FP32 rounding of the result
    nnz = np.diff(A.indptr)
    rmax = np.array([np.max(np.abs(A.data[A.indptr[i]:A.indptr[i + 1]])) if nnz[i] else 0 for i in range(m)])
    grid = rmax * 2.0 ** -(60 - np.ceil(np.log2(np.maximum(nnz, 1)))) * nnz
    tol = 2 * U32 * np.abs(ref) + grid[:, None] + 1e-37
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def test_sketch_csr_empty_nan_and_bad_index_rows():
    m, n, r1 = 6, 50, 20
    dense = np.zeros((m, n))
    dense[1, [3, 7]] = [1.0, -2.0]
    dense[2, 5] = np.nan
    dense[4, :] = np.arange(n)
    A = sp.csr_matrix(np.where(np.isnan(dense), 1.0, dense))
    A.data[A.indptr[2]] = np.nan                         # row 2 holds a NaN
    C = rf.Csr.from_scipy(A, DEV)
    got = rf.rf_sketch_apply_csr(C, r1, 4, 1).cpu().numpy()
    assert np.all(got[[0, 3, 5]] == 0)                   # empty rows
    assert np.all(np.isnan(got[2]))
    t = sk.sketch_table(n, 4, r1, 1)
    ref = me.sketch_right(np.nan_to_num(A.toarray()), t, r1)
    assert np.allclose(got[[1, 4]], ref[[1, 4]], rtol=1e-6, atol=1e-6)
    # a column index outside [0, n) is skipped and reported by rf_svd_csr
    col = C.col_idx.clone()
    col[0] = 10 ** 6
    B = rf.Csr(C.row_ptr, col, torch.nan_to_num(C.values), (m, n))
    U, sig, Vt, info = rf.rf_svd_csr(B, 2, 4, 0, 2, seed=1)
    torch.cuda.synchronize()
    assert rf.info_dict(info)["status"] & 16


@pytest.mark.parametrize("q", [0, 2])
@pytest.mark.parametrize("m,n,dens,k,l,s", [(3000, 1500, 0.01, 40, 120, 8), (2000, 4000, 0.003, 25, 80, 4)])
def test_svd_csr_parity(q, m, n, dens, k, l, s):
    A = graded_sparse(m, n, dens, 7 * m + q)
    Ad = A.toarray()
    C = rf.Csr.from_scipy(A, DEV)
    U, sig, Vt, info = rf.rf_svd_csr(C, k, l, q, s, seed=19, orth_err=True)
    ref = me.rand_svd(Ad, me.Params(k=k, l=l, q=q, s=s, seed=19))
    sig = sig.cpu().numpy()
    tol = 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]
    print("csr svd q=%d max |dsigma|/tol %.3f" % (q, np.max(np.abs(sig - ref.sigma) / tol)))
    assert np.all(np.abs(sig - ref.sigma) <= tol)
    Ug = U.cpu().numpy().astype(np.float64)
    eg, eo = ev.frob_error(Ad, Ug), ev.frob_error(Ad, ref.U)
    assert abs(eg - eo) <= 1e-4 * eo
    inf = rf.info_dict(info)
    assert inf["orth_err"] < 2e-5 and inf["status"] == 0
    # V: V^T = Sigma^-1 U^T A on the well-resolved part
    good = sig > 1e-3 * sig[0]
    Vg = Vt.cpu().numpy().astype(np.float64)[good]
    assert np.allclose(Vg, (Ug.T @ Ad)[good] / sig[good, None], atol=2e-4)
    Qm, _ = rf.rf_range_finder_csr(C, k, l, q, s, seed=19, precision="mixed")
    assert ev.frob_error(Ad, Qm.cpu().numpy().astype(np.float64)) <= 1.02 * eo


def test_csr_rejections():
    A = graded_sparse(100, 80, 0.1, 1)
    C = rf.Csr.from_scipy(A, DEV)
    p = rf.params(5, 10, 1, 2, 0, "fp32", rf.RF_FLAG_CLASSICAL)
    assert rf.lib().rf_workspace_size_csr(rf.RF_OP_SVD, C.desc(), p) == 0
    with pytest.raises(rf.RFError):
        rf.rf_svd_csr(C, 20, 10)
