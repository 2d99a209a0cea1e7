"""Algorithm 1 with caller-given S and Omega (rf_range_finder_ex) and the
classical form S = I (RF_FLAG_CLASSICAL: the baseline of Section 2,
"Comparison with Classical Range Finder", and of the additional experiments,
Algorithm 2 with S1 = I), against the FP64 oracle on the same inputs."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
import synth
from oracle import methods as me, evaluate as ev, sketch as sk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev32(A):
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).to(DEV)


def _instance(name, m, n):
    A, _ = synth.workload(name, m=m, n=n)
    A32 = A.astype(np.float32)
    return A32, A32.astype(np.float64)


@pytest.mark.parametrize("q", [0, 1, 3])
@pytest.mark.parametrize("m,n,k", [(1500, 800, 30), (999, 517, 13)])
def test_classical_range_finder_parity(q, m, n, k):
    A32, A = _instance("poly65k", m, n)
    Q, info = rf.rf_range_finder(dev32(A32), k, 2 * k, q, 1, seed=17, orth_err=True, classical=True)
    Q = Q.cpu().numpy().astype(np.float64)
    ref = me.range_finder(A, me.Params(k=k, l=2 * k, q=q, s=1, seed=17), classical=True)
    eg, eo = ev.frob_error(A, Q), ev.frob_error(A, ref.Q)
    print("classical q=%d err gpu %.10e oracle %.10e rel %.2e" % (q, eg, eo, abs(eg - eo) / eo))
    assert abs(eg - eo) <= 1e-4 * eo
    assert rf.info_dict(info)["orth_err"] < 2e-5


def test_classical_svd_and_mixed():
    A32, A = _instance("polydecay", 1200, 700)
    k = 40
    U, sig, Vt, _ = rf.rf_svd(dev32(A32), k, 80, 2, 1, seed=3, classical=True)
    ref = me.rand_svd(A, me.Params(k=k, l=80, q=2, s=1, seed=3), classical=True)
    sig = sig.cpu().numpy()
    tol = 1e-5 * ref.sigma + 2e-6 * ref.sigma[0]
    assert np.all(np.abs(sig - ref.sigma) <= tol), np.max(np.abs(sig - ref.sigma) / tol)
    Qm, _ = rf.rf_range_finder(dev32(A32), k, 80, 2, 1, seed=3, precision="mixed", classical=True)
    em = ev.frob_error(A, Qm.cpu().numpy().astype(np.float64))
    eo = ev.frob_error(A, ref.Q)
    print("classical mixed err %.8e oracle %.8e" % (em, eo))
    assert em <= 1.02 * eo


def test_classical_lowrank_parity():
    """Algorithm 2 with S1 = I: S2 keeps `sketch` rows (stream 2)."""
    A32, A = _instance("polydecay", 1100, 600)
    k, l = 25, 90
    Y, X, _ = rf.rf_lowrank(dev32(A32), k, l, 1, 4, seed=8, classical=True)
    Y, X = Y.cpu().numpy().astype(np.float64), X.cpu().numpy().astype(np.float64)
    ref = me.lowrank(A, me.Params(k=k, l=l, q=1, s=4, seed=8), classical=True)
    eg, eo = np.linalg.norm(A - Y @ X), np.linalg.norm(A - ref.Q @ ref.X)
    print("classical lowrank err gpu %.10e oracle %.10e rel %.2e" % (eg, eo, abs(eg - eo) / eo))
    assert abs(eg - eo) <= 1e-4 * eo


def test_ex_with_seeded_inputs_equals_range_finder():
    """The table and Omega the library draws itself, passed back in, give the
    same bits (same kernels on the same inputs)."""
    A32, _ = _instance("poly65k", 1300, 700)
    dA = dev32(A32)
    k, l, s, seed = 40, 120, 8, 23
    Q0, _ = rf.rf_range_finder(dA, k, l, 2, s, seed=seed)
    T = rf.rf_sketch_table(700, s, l, seed, 0)
    Om = rf.rf_gaussian(l, k, seed, 1)
    Q1, info = rf.rf_range_finder_ex(dA, k, l, S_table=T, Omega=Om, q=2, nnz_per_col=s, seed=seed)
    torch.cuda.synchronize()
    assert torch.equal(Q0, Q1)
    assert rf.info_dict(info)["status"] & 8 == 0


@pytest.mark.parametrize("s", [1, 3, 8])
def test_ex_with_caller_inputs_matches_oracle(s):
    """A table and Omega that do not come from the library's generator."""
    A32, A = _instance("poly65k", 1400, 900)
    k, l = 30, 96
    rng = np.random.default_rng(5 + s)
    lo = sk.block_bounds(l, s)
    buckets = np.stack([rng.integers(lo[t], lo[t + 1], size=900) for t in range(s)], axis=1)
    neg = rng.integers(0, 2, size=(900, s))
    table = (buckets | (neg << 31)).astype(np.int64).astype(np.uint32).view(np.int32)
    Om = rng.standard_normal((l, k)).astype(np.float32)
    Q, info = rf.rf_range_finder_ex(dev32(A32), k, l, S_table=torch.from_numpy(table).to(DEV),
                                    Omega=torch.from_numpy(Om).to(DEV), q=1, nnz_per_col=s, seed=0, orth_err=True)
    ref = me.range_finder(A, me.Params(k=k, l=l, q=1, s=s, seed=0), table=table, Om=Om.astype(np.float64))
    eg, eo = ev.frob_error(A, Q.cpu().numpy().astype(np.float64)), ev.frob_error(A, ref.Q)
    print("ex s=%d err gpu %.10e oracle %.10e" % (s, eg, eo))
    assert abs(eg - eo) <= 1e-4 * eo
    inf = rf.info_dict(info)
    assert inf["status"] & 8 == 0 and inf["orth_err"] < 2e-5


def test_ex_classical_with_given_omega():
    A32, A = _instance("polydecay", 900, 500)
    k = 20
    Om = np.random.default_rng(2).standard_normal((500, k)).astype(np.float32)
    Q, _ = rf.rf_range_finder_ex(dev32(A32), k, 40, Omega=torch.from_numpy(Om).to(DEV), q=2, nnz_per_col=1,
                                 classical=True)
    ref = me.range_finder(A, me.Params(k=k, l=40, q=2, s=1, seed=0), Om=Om.astype(np.float64), classical=True)
    eg, eo = ev.frob_error(A, Q.cpu().numpy().astype(np.float64)), ev.frob_error(A, ref.Q)
    assert abs(eg - eo) <= 1e-4 * eo


def test_ex_table_outside_blocks_is_reported():
    A32, _ = _instance("poly65k", 400, 300)
    s, l, k = 4, 40, 8
    T = rf.rf_sketch_table(300, s, l, 5, 0)
    T[7, 2] = 39          # block 2 of 40/4 is [20, 30): out of block
    T[11, 0] = 1 << 30    # far out of range
    Q, info = rf.rf_range_finder_ex(dev32(A32), k, l, S_table=T, q=1, nnz_per_col=s, seed=5)
    torch.cuda.synchronize()
    assert rf.info_dict(info)["status"] & 8
    assert torch.isfinite(Q).all()


def test_classical_rejections():
    Ab = torch.zeros((100, 60), dtype=torch.bfloat16, device=DEV)
    with pytest.raises(rf.RFError) as e:
        rf.rf_range_finder(Ab, 5, 10, 1, 1, classical=True)
    assert e.value.status == rf.RF_EUNSUPPORTED
    A = torch.zeros((60, 60), device=DEV)
    p = rf.params(5, 10, 1, 2, 0, "fp32", rf.RF_FLAG_CLASSICAL)
    L = rf.lib()
    C = torch.empty((60, 5), device=DEV)
    W = torch.empty((5, 5), dtype=torch.float64, device=DEV)
    st = L.rf_nystrom(ctypes.byref(rf.matrix(A)), ctypes.byref(p), C.data_ptr(), 5, W.data_ptr(), 5, None, 5,
                      None, 0, None, None)
    assert st == rf.RF_EUNSUPPORTED
    T = rf.rf_sketch_table(60, 1, 10, 0, 0)
    with pytest.raises(rf.RFError) as e:
        rf.rf_range_finder_ex(A, 5, 10, S_table=T, q=1, nnz_per_col=1, classical=True)
    assert e.value.status == rf.RF_EINVAL
