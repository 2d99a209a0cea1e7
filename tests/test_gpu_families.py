"""Sketch families of Lemma 3.2 beyond the sparse sign sketch (item 1: dense
Rademacher and Gaussian S; item 3: the SRHT) through the C ABI, against the
FP64 oracle on the same draws: A S element by element with the rounding bound
of each form, and Algorithm 1 / RandSVD end to end."""
import math

import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
import synth
from oracle import methods as me, evaluate as ev, sketch as sk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24


def dev32(A):
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).to(DEV)


def _ref_S(n, r1, seed, family):
    return me.sketch_dense_family(n, me.Params(k=1, l=r1, seed=seed), family)


@pytest.mark.parametrize("family", ["rademacher", "gaussian"])
@pytest.mark.parametrize("m,n,r1", [(300, 700, 90), (77, 2048, 256), (5, 33, 7)])
def test_dense_sketch_apply_fp32(family, m, n, r1):
    """FP32 MFMA product: |dAt| <= (n + 4) u32 (|A| |S|) (recursive summation,
    plus the FP32 rounding of the N(0,1) draws and of the 1/sqrt(r1) scale)."""
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    A64 = A.astype(np.float64)
    S = _ref_S(n, r1, 5, family)
    ref = A64 @ S
    got = rf.rf_sketch_apply(dev32(A), r1, 1, 5, family=family).cpu().numpy()
    tol = (n + 4) * U32 * (np.abs(A64) @ np.abs(S)) + 1e-30
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def test_dense_sketch_apply_mixed_bf16():
    """Mixed form: A rounded to BF16 on load, S = +-1 exact in BF16: the product
    equals bf16(A) S up to FP32 accumulation."""
    rng = np.random.default_rng(1)
    m, n, r1 = 200, 1000, 128
    A = rng.standard_normal((m, n)).astype(np.float32)
    Ab = torch.from_numpy(A).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    S = _ref_S(n, r1, 9, "rademacher")
    ref = Ab @ S
    got = rf.rf_sketch_apply(dev32(A), r1, 1, 9, family="rademacher", precision="mixed").cpu().numpy()
    tol = (n + 4) * U32 * (np.abs(Ab) @ np.abs(S)) + 1e-30
    assert np.all(np.abs(got - ref) <= tol)


@pytest.mark.parametrize("m,n,r1", [(64, 1000, 100), (40, 16384, 2000), (9, 32768, 4000), (33, 50, 20),
                                    (17, 200, 128), (3, 5, 2)])
def test_srht_sketch_apply(m, n, r1):
    """FWHT in FP32 over L = log2 n' stages: |dAt| <= (L + 2) u32 ||a_i||_1 / sqrt(r1)."""
    rng = np.random.default_rng(n + r1)
    A = rng.standard_normal((m, n)).astype(np.float32)
    A64 = A.astype(np.float64)
    n2 = sk.srht_size(n)
    d, picks = sk.srht_draws(n, r1, 13)
    # the oracle's dense S for the small cases; an explicit transform for the large ones
    if n2 <= 4096:
        ref = A64 @ sk.srht_matrix(n, r1, 13)
    else:
        X = np.zeros((m, n2))
        X[:, :n] = A64 * d[None, :n]
        h = 1
        while h < n2:                                  # Walsh-Hadamard by butterflies, FP64
            X = X.reshape(m, -1, 2, h)
            X = np.concatenate([X[:, :, 0] + X[:, :, 1], X[:, :, 0] - X[:, :, 1]], axis=2).reshape(m, n2)
            h *= 2
        ref = X[:, picks] / math.sqrt(r1)
    got = rf.rf_sketch_apply(dev32(A), r1, 1, 13, family="srht").cpu().numpy()
    L = max(1, int(math.log2(n2)))
    tol = (L + 2) * U32 * np.sum(np.abs(A64), axis=1)[:, None] / math.sqrt(r1) + 1e-30
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def test_srht_bf16_and_fp8_storage():
    from tests import fp8_ref
    rng = np.random.default_rng(3)
    m, n, r1 = 150, 3000, 300
    A = rng.standard_normal((m, n)).astype(np.float32)
    Sd = sk.srht_matrix(n, r1, 2)
    L = 12
    Ab = torch.from_numpy(A).to(torch.bfloat16)
    Ab64 = Ab.to(torch.float32).numpy().astype(np.float64)
    got = rf.rf_sketch_apply(Ab.to(DEV), r1, 1, 2, family="srht").cpu().numpy()
    tol = (L + 2) * U32 * np.sum(np.abs(Ab64), axis=1)[:, None] / math.sqrt(r1)
    assert np.all(np.abs(got - Ab64 @ Sd) <= tol)
    codes, scales = fp8_ref.quantize_blocks(A.astype(np.float64))
    Aq = fp8_ref.dequantize(codes, scales)
    got = rf.rf_sketch_apply(torch.from_numpy(codes).to(DEV), r1, 1, 2, scales=torch.from_numpy(scales).to(DEV),
                             family="srht").cpu().numpy()
    tol = (L + 3) * U32 * np.sum(np.abs(Aq), axis=1)[:, None] / math.sqrt(r1)
    assert np.all(np.abs(got - Aq @ Sd) <= tol)


@pytest.mark.parametrize("family", ["rademacher", "gaussian", "srht"])
@pytest.mark.parametrize("q", [0, 2])
def test_range_finder_and_svd_per_family(family, q):
    A, _ = synth.workload("poly65k", m=1500, n=900)
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    k, l = 40, 120
    Q, info = rf.rf_range_finder(dev32(A32), k, l, q, 1, seed=31, orth_err=True, family=family)
    ref = me.range_finder(A64, me.Params(k=k, l=l, q=q, s=1, seed=31), family=family)
    eg, eo = ev.frob_error(A64, Q.cpu().numpy().astype(np.float64)), ev.frob_error(A64, ref.Q)
    print("%s q=%d err gpu %.10e oracle %.10e rel %.2e" % (family, q, eg, eo, abs(eg - eo) / eo))
    assert abs(eg - eo) <= 1e-4 * eo
    assert rf.info_dict(info)["orth_err"] < 2e-5
    U, sig, Vt, _ = rf.rf_svd(dev32(A32), k, l, q, 1, seed=31, family=family)
    rs = me.rand_svd(A64, me.Params(k=k, l=l, q=q, s=1, seed=31), family=family)
    sig = sig.cpu().numpy()
    assert np.all(np.abs(sig - rs.sigma) <= 1e-5 * rs.sigma + 2e-6 * rs.sigma[0])
    Qm, _ = rf.rf_range_finder(dev32(A32), k, l, q, 1, seed=31, precision="mixed", family=family)
    assert ev.frob_error(A64, Qm.cpu().numpy().astype(np.float64)) <= 1.02 * eo


def test_lowrank_with_srht():
    A, _ = synth.workload("poly65k", m=1200, n=700)
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    Y, X, _ = rf.rf_lowrank(dev32(A32), 30, 90, 1, 4, seed=2, family="srht")
    ref = me.lowrank(A64, me.Params(k=30, l=90, q=1, s=4, seed=2), family="srht")
    eg = np.linalg.norm(A64 - Y.cpu().numpy().astype(np.float64) @ X.cpu().numpy().astype(np.float64))
    eo = np.linalg.norm(A64 - ref.Q @ ref.X)
    assert abs(eg - eo) <= 1e-4 * eo


def test_family_rejections():
    A8 = torch.zeros((100, 60), dtype=torch.uint8, device=DEV)
    sc = torch.ones((1, 1), device=DEV)
    with pytest.raises(rf.RFError) as e:
        rf.rf_sketch_apply(A8, 10, 1, 0, scales=sc, family="rademacher")
    assert e.value.status == rf.RF_EUNSUPPORTED
    big = torch.zeros((2, 40000), device=DEV)
    with pytest.raises(rf.RFError) as e:
        rf.rf_sketch_apply(big, 16, 1, 0, family="srht")
    assert e.value.status == rf.RF_EUNSUPPORTED
    A = torch.zeros((100, 100), device=DEV)
    T = rf.rf_sketch_table(100, 1, 10, 0, 0)
    with pytest.raises(rf.RFError) as e:
        rf.rf_range_finder_ex(A, 5, 10, S_table=T, q=1, nnz_per_col=1, family="srht")
    assert e.value.status == rf.RF_EINVAL
    with pytest.raises(rf.RFError) as e:
        rf.rf_range_finder(A, 5, 10, 1, 1, classical=True, family="gaussian")
    assert e.value.status == rf.RF_EINVAL
