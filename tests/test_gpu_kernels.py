"""Kernel-level parity on the GPU: every HIP kernel of the path against the
FP64 oracle (or an exact NumPy reference where the operation is a plain
definition), through the C ABI.  Integer work is compared bit for bit."""
import math

import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
from oracle import sketch as sk, methods as me
from tests import fp8_ref

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24


def bf16_round(x):
    t = torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t, t.to(torch.float32).numpy().astype(np.float64)


# ---------------------------------------------------------------- K1 sketch table
@pytest.mark.parametrize("n,s,r1,seed,stream,b", [
    (1000, 8, 100, 42, 0, 0), (777, 3, 50, 7, 2, 1), (16384, 8, 2000, 102, 0, 0),
    (5, 1, 1, 0, 0, 0), (100, 16, 64, (1 << 40) | 5, 3, 7), (4099, 4, 4096, 9, 0, 0)])
def test_sketch_table_bitexact(n, s, r1, seed, stream, b):
    g = rf.rf_sketch_table(n, s, r1, seed, stream, b, DEV)
    torch.cuda.synchronize()
    ref = sk.sketch_table(n, s, r1, seed, stream, b)
    assert np.array_equal(g.cpu().numpy(), ref)


# ---------------------------------------------------------------- K2 Gaussian
@pytest.mark.parametrize("rows,cols,seed,stream", [(31, 17, 3, 1), (2000, 100, 42, 1), (1000, 1001, 5, 3)])
def test_gaussian_within_one_ulp(rows, cols, seed, stream):
    g = rf.rf_gaussian(rows, cols, seed, stream, 0, DEV).cpu().numpy()
    ref = sk.gaussian(rows, cols, seed, stream).astype(np.float32)
    ulp = np.spacing(np.abs(ref).astype(np.float32))
    assert np.all(np.abs(g - ref) <= ulp)
    assert np.mean(g == ref) > 0.99


# ---------------------------------------------------------------- K3 A S
def _sketch_ref(A64, n, s, r1, seed):
    t = sk.sketch_table(n, s, r1, seed)
    return me.sketch_right(A64, t, r1), np.asarray(np.abs(A64) @ np.abs(sk.sketch_matrix(t, r1).toarray()))


def _fixed_point_bound(A64, table, r1, s, J=2048):
    """Rounding bound of the fixed-point scatter.  Within a column chunk of the pass
    (2048 columns, or 1024 for s = 4, inside the 2048-column chunks used here) a row's
    terms are rounded to half a grid step of at most c 2^-25 times the largest |a| of
    the chunk over the row's band of 64/s rows (c = the chunk's largest bucket
    occupancy; two bits of headroom and up to two bits kept from an earlier chunk's
    scale).  Returns, per output, that bound summed over the output's terms, times
    1/sqrt(s)."""
    m, n = A64.shape
    R = max(64 // s, 1)
    buckets = (table.astype(np.int64) & 0x7FFFFFFF)
    out = np.zeros((m, r1))
    for c0 in range(0, n, J):
        cols = slice(c0, min(n, c0 + J))
        cnt = np.zeros((r1,))
        for t in range(s):
            cnt += np.bincount(buckets[cols, t], minlength=r1)
        cmax = max(cnt.max(), 1.0)
        half_step = np.zeros((m,))
        for b0 in range(0, m, R):
            half_step[b0:b0 + R] = np.max(np.abs(A64[b0:b0 + R, cols])) * cmax * 2.0 ** -25
        out += half_step[:, None] * cnt[None, :]
    return out / math.sqrt(s)


def _sketch_tol(A64, n, s, r1, seed, mag):
    """FP32 summation bound plus the fixed-point grid of the scatter."""
    return ((n * s / r1 + 8) * 4 * U32 * mag + _fixed_point_bound(A64, sk.sketch_table(n, s, r1, seed), r1, s)
            + 1e-30)


@pytest.mark.parametrize("m,n,s,r1", [
    (64, 256, 8, 100), (77, 1000, 8, 100), (130, 513, 4, 40), (100, 300, 1, 50), (100, 300, 2, 50),
    (50, 200, 3, 20), (40, 700, 16, 64), (70, 2000, 1, 1000), (9, 5000, 8, 4000), (1, 1, 1, 1),
    (20, 3000, 4, 1500), (17, 7000, 16, 6000), (33, 6000, 8, 5000)])
def test_sketch_apply_f32(m, n, s, r1):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    A64 = A.astype(np.float64)
    ref, mag = _sketch_ref(A64, n, s, r1, 11)
    got = rf.rf_sketch_apply(torch.from_numpy(A).to(DEV), r1, s, 11).cpu().numpy()
    tol = _sketch_tol(A64, n, s, r1, 11, mag)
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


@pytest.mark.parametrize("m,n,s,r1", [(40, 3000, 4, 2800), (33, 5000, 5, 900), (64, 32768, 1, 700),
                                     (5, 20000, 2, 3000), (300, 4096, 1, 2000), (2, 1000, 7, 7)])
def test_sketch_apply_gather_form(m, n, s, r1):
    """The gather form (s without a fixed-point path, and s = 4 sketches beyond
    640 buckets per block): element-wise within the FP32 summation bound, and the
    same bits on a second call (fixed summation order, no atomics)."""
    rng = np.random.default_rng(m + n + s)
    A = (rng.standard_normal((m, n)) * np.exp(rng.standard_normal((1, n)))).astype(np.float32)
    A64 = A.astype(np.float64)
    ref, mag = _sketch_ref(A64, n, s, r1, 19)
    dA = torch.from_numpy(A).to(DEV)
    got = rf.rf_sketch_apply(dA, r1, s, 19)
    again = rf.rf_sketch_apply(dA, r1, s, 19)
    torch.cuda.synchronize()
    assert torch.equal(got, again)
    got = got.cpu().numpy()
    tol = _sketch_tol(A64, n, s, r1, 19, mag)
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def test_sketch_apply_strided_rows():
    rng = np.random.default_rng(5)
    big = rng.standard_normal((60, 1030)).astype(np.float32)
    A = torch.from_numpy(big).to(DEV)[:, 3:1003]          # ld = 1030, unaligned start
    ref, mag = _sketch_ref(big[:, 3:1003].astype(np.float64), 1000, 8, 96, 3)
    got = rf.rf_sketch_apply(A, 96, 8, 3).cpu().numpy()
    assert np.all(np.abs(got - ref) <= _sketch_tol(big[:, 3:1003].astype(np.float64), 1000, 8, 96, 3, mag))


@pytest.mark.parametrize("m,n,s,r1", [(64, 512, 8, 100), (33, 333, 4, 60), (40, 3000, 8, 3000)])
def test_sketch_apply_bf16(m, n, s, r1):
    rng = np.random.default_rng(1)
    At, A64 = bf16_round(rng.standard_normal((m, n)))
    ref, mag = _sketch_ref(A64, n, s, r1, 12)
    got = rf.rf_sketch_apply(At.to(DEV), r1, s, 12).cpu().numpy()
    assert np.all(np.abs(got - ref) <= _sketch_tol(A64, n, s, r1, 12, mag))


@pytest.mark.parametrize("m,n,s,r1", [(256, 384, 8, 64), (200, 300, 4, 40), (130, 3100, 8, 3000)])
def test_sketch_apply_fp8_block_scaled(m, n, s, r1):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((m, n)) * np.exp(rng.standard_normal((m, 1)))
    codes, scales = fp8_ref.quantize_blocks(X)
    A64 = fp8_ref.dequantize(codes, scales)
    ref, mag = _sketch_ref(A64, n, s, r1, 13)
    got = rf.rf_sketch_apply(torch.from_numpy(codes).to(DEV), r1, s, 13,
                             scales=torch.from_numpy(scales).to(DEV)).cpu().numpy()
    assert np.all(np.abs(got - ref) <= _sketch_tol(A64, n, s, r1, 13, mag))


@pytest.mark.parametrize("s,r1", [(8, 200), (4, 96), (16, 400), (8, 4000)])
def test_sketch_apply_chunk_scales(s, r1):
    """Column chunks of very different magnitude (and an all-zero chunk) over many
    chunks: every fixed-point rescale and partial fold of the pass is exercised.
    A term that is tiny next to the largest entry of its chunk is rounded on that
    entry's grid, so the bound adds the fixed-point grid to the summation bound."""
    rng = np.random.default_rng(s * 1000 + r1)
    m, n = 40, 2048 * 13 + 77
    A = rng.standard_normal((m, n))
    f = np.repeat([1.0, 1e3, 1e-3, 1.0, 0.0, 1.0, 1.0, 2.0 ** 20, 1.0, 1.0, 1.0, 1.0, 1e-6, 1.0], 2048)[:n]
    A = (A * f).astype(np.float32)
    A64 = A.astype(np.float64)
    ref, mag = _sketch_ref(A64, n, s, r1, 17)
    got = rf.rf_sketch_apply(torch.from_numpy(A).to(DEV), r1, s, 17).cpu().numpy()
    tol = _sketch_tol(A64, n, s, r1, 17, mag)
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


@pytest.mark.parametrize("s", [1, 3, 8])
def test_sketch_apply_nonfinite_rows(s):
    """A row holding NaN or Inf gives a non-finite row of AS (the FP32 sum over
    it is non-finite in the buckets it touches); every other row is unaffected."""
    rng = np.random.default_rng(21)
    m, n, r1 = 70, 900, 64
    A = rng.standard_normal((m, n)).astype(np.float32)
    A[3, 17] = np.nan
    A[40, 800] = np.inf
    A[41, 0] = -np.inf
    clean = np.ones(m, dtype=bool)
    clean[[3, 40, 41]] = False
    A64 = np.where(np.isfinite(A), A, 0.0).astype(np.float64)
    ref, mag = _sketch_ref(A64, n, s, r1, 31)
    got = rf.rf_sketch_apply(torch.from_numpy(A).to(DEV), r1, s, 31).cpu().numpy()
    tol = _sketch_tol(A64, n, s, r1, 31, mag)
    assert np.all(np.abs(got[clean] - ref[clean]) <= tol[clean])
    for i in np.flatnonzero(~clean):
        assert not np.all(np.isfinite(got[i]))


# ---------------------------------------------------------------- S2^T A (Algorithm 2)
def _left_ref(A64, s, r1, seed):
    m = A64.shape[0]
    t = sk.sketch_table(m, s, r1, seed, sk.STREAM_S2)
    S2 = sk.sketch_matrix(t, r1)
    ref = me.sketch_left(A64, t, r1)
    mag = np.asarray(np.abs(S2.T) @ np.abs(A64))
    return t, ref, mag


def _left_tol(A64, t, s, r1, mag):
    """Bound of the fixed-point left sketch.  Column j has one scale for the whole
    pass: 2^e > c max_i |a_ij| with 2^e <= 4 c max_i |a_ij| (c = the largest bucket
    occupancy over all rows), terms rounded to half of 2^(e-30), so output (b, j)
    with cnt_b terms is off by at most cnt_b c max_i|a_ij| 2^-29 / sqrt(s); plus FP32
    rounding of the conversion, the 1/sqrt(s) scale and up to 64 row-split partials
    summed in FP32 (72 units of 2^-24 of the sum of |terms|)."""
    cnt = np.bincount((t.astype(np.int64) & 0x7FFFFFFF).ravel(), minlength=r1).astype(np.float64)
    c = max(cnt.max(), 1.0)
    colmax = np.max(np.abs(A64), axis=0) if A64.shape[0] else np.zeros(A64.shape[1])
    return cnt[:, None] * c * colmax[None, :] * 2.0 ** -29 / math.sqrt(s) + 72 * U32 * mag + 1e-30


@pytest.mark.parametrize("m,n,s,r1", [
    (3000, 200, 8, 1500), (2001, 130, 8, 700), (4100, 65, 8, 100), (1, 10, 1, 1), (7, 3, 8, 8),
    (500, 300, 4, 600), (700, 90, 16, 1100), (1000, 64, 3, 50), (300, 1000, 8, 2000)])
def test_sketch_left_f32(m, n, s, r1):
    rng = np.random.default_rng(m + 3 * n + s)
    A = (rng.standard_normal((m, n)) * np.exp(rng.standard_normal((1, n)))).astype(np.float32)
    A64 = A.astype(np.float64)
    t, ref, mag = _left_ref(A64, s, r1, 23)
    got = rf.rf_sketch_apply_left(torch.from_numpy(A).to(DEV), r1, s, 23).cpu().numpy()
    tol = _left_tol(A64, t, s, r1, mag)
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def test_sketch_left_bf16_and_fp8():
    rng = np.random.default_rng(8)
    m, n, s, r1 = 2000, 130, 8, 900
    At, A64 = bf16_round(rng.standard_normal((m, n)))
    t, ref, mag = _left_ref(A64, s, r1, 29)
    got = rf.rf_sketch_apply_left(At.to(DEV), r1, s, 29).cpu().numpy()
    assert np.all(np.abs(got - ref) <= _left_tol(A64, t, s, r1, mag))
    X = rng.standard_normal((m, 300)) * np.exp(rng.standard_normal((m, 1)))
    codes, scales = fp8_ref.quantize_blocks(X)
    A64 = fp8_ref.dequantize(codes, scales)
    t, ref, mag = _left_ref(A64, s, r1, 29)
    got = rf.rf_sketch_apply_left(torch.from_numpy(codes).to(DEV), r1, s, 29,
                                  scales=torch.from_numpy(scales).to(DEV)).cpu().numpy()
    assert np.all(np.abs(got - ref) <= _left_tol(A64, t, s, r1, mag))


def test_sketch_left_nonfinite_columns():
    """A column holding NaN or Inf comes out NaN in every bucket; the others are
    unaffected (their scales never see it)."""
    rng = np.random.default_rng(9)
    m, n, s, r1 = 1500, 150, 8, 600
    A = rng.standard_normal((m, n)).astype(np.float32)
    A[10, 5] = np.nan
    A[1400, 77] = np.inf
    A64 = np.where(np.isfinite(A), A, 0.0).astype(np.float64)
    t, ref, mag = _left_ref(A64, s, r1, 37)
    got = rf.rf_sketch_apply_left(torch.from_numpy(A).to(DEV), r1, s, 37).cpu().numpy()
    clean = np.ones(n, dtype=bool)
    clean[[5, 77]] = False
    tol = _left_tol(A64, t, s, r1, mag)
    assert np.all(np.abs(got[:, clean] - ref[:, clean]) <= tol[:, clean])
    assert np.all(np.isnan(got[:, ~clean]))


# ---------------------------------------------------------------- K5/K6 GEMM
def _operands(M, N, K, a_kc, b_kc, rng, bf16):
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    if bf16:
        At, A = bf16_round(A)
        Bt, B = bf16_round(B)
    else:
        At = torch.from_numpy(A.astype(np.float32)); A = A.astype(np.float32).astype(np.float64)
        Bt = torch.from_numpy(B.astype(np.float32)); B = B.astype(np.float32).astype(np.float64)
    Astore = At if a_kc else At.t().contiguous()      # a_kc: (M, K) row-major; else (K, M)
    Bstore = Bt.t().contiguous() if b_kc else Bt      # b_kc: (N, K) row-major; else (K, N)
    return Astore.to(DEV), Bstore.to(DEV), A, B


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("a_kc,b_kc", [(1, 1), (1, 0), (0, 1), (0, 0)])
@pytest.mark.parametrize("M,N,K", [(128, 128, 32), (300, 200, 100), (1000, 70, 5000), (64, 1000, 2000), (1, 1, 1)])
def test_gemm(bf16, a_kc, b_kc, M, N, K):
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    dA, dB, A, B = _operands(M, N, K, a_kc, b_kc, rng, bf16)
    C = rf.rf_test_gemm(dA, dB, M, N, K, a_kc, b_kc).cpu().numpy()
    ref = A @ B
    mag = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(C - ref) <= (K + 2) * U32 * mag + 1e-30), np.max(np.abs(C - ref) / (mag + 1e-30))


@pytest.mark.parametrize("a_kc,b_kc", [(1, 1), (1, 0), (0, 1), (0, 0)])
@pytest.mark.parametrize("M,N,K", [(512, 512, 64), (600, 700, 300), (1030, 1000, 4100), (777, 520, 33)])
def test_gemm_bf16_large_tiles(a_kc, b_kc, M, N, K):
    """Shapes routed to the 256 x 256-tile BF16 kernel (several tiles, ragged
    edges in M, N and K, split-K)."""
    rng = np.random.default_rng(M + 5 * N + 11 * K)
    dA, dB, A, B = _operands(M, N, K, a_kc, b_kc, rng, True)
    for split in (True, False):
        C = rf.rf_test_gemm(dA, dB, M, N, K, a_kc, b_kc, split=split).cpu().numpy()
        mag = np.abs(A) @ np.abs(B)
        assert np.all(np.abs(C - A @ B) <= (K + 2) * U32 * mag + 1e-30), np.max(np.abs(C - A @ B) / (mag + 1e-30))


@pytest.mark.parametrize("a_kc,b_kc", [(1, 0), (0, 0), (0, 1)])
@pytest.mark.parametrize("M,N,K", [(600, 700, 300), (300, 40, 1000)])
def test_gemm_f32_a_rounded_on_load(a_kc, b_kc, M, N, K):
    """A stored FP32 and rounded to BF16 (RNE) as it is loaded: the result is the
    BF16 product of round(A) and B."""
    rng = np.random.default_rng(M + N + K)
    A32 = rng.standard_normal((M, K)).astype(np.float32)
    At16, A = bf16_round(A32)
    Bt, B = bf16_round(rng.standard_normal((K, N)))
    Astore = torch.from_numpy(A32) if a_kc else torch.from_numpy(A32.T.copy())
    Bstore = Bt.t().contiguous() if b_kc else Bt
    C = rf.rf_test_gemm(Astore.to(DEV), Bstore.to(DEV), M, N, K, a_kc, b_kc).cpu().numpy()
    mag = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(C - A @ B) <= (K + 2) * U32 * mag + 1e-30)


@pytest.mark.parametrize("b_kc", [0, 1])
@pytest.mark.parametrize("M,N,K", [(600, 300, 1000), (520, 700, 257), (1030, 64, 4100)])
def test_gemm_fp8_block_scaled_a(b_kc, M, N, K):
    """A stored as e4m3 with 128 x 128 block scales (K x M), dequantised and rounded
    to BF16 as it is loaded: the result is the BF16 product of round(dequant(A)) and B."""
    rng = np.random.default_rng(M + 3 * N + K)
    X = rng.standard_normal((K, M)) * np.exp(rng.standard_normal((K, 1)))
    codes, scales = fp8_ref.quantize_blocks(X)
    Adeq = fp8_ref.dequantize(codes, scales)
    _, A = bf16_round(Adeq.T)                           # op(A) = A^T of the stored K x M
    Bt, B = bf16_round(rng.standard_normal((K, N)))
    Bstore = Bt.t().contiguous() if b_kc else Bt
    C = rf.rf_test_gemm_fp8a(torch.from_numpy(codes).to(DEV), torch.from_numpy(scales).to(DEV), Bstore.to(DEV),
                             M, N, K, b_kc).cpu().numpy()
    mag = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(C - A @ B) <= (K + 2) * U32 * mag + 1e-30)


@pytest.mark.parametrize("M,N,K", [(600, 300, 1000), (520, 700, 257), (1030, 64, 4100), (256, 256, 128),
                                   (300, 2000, 1300), (1, 1, 1)])
def test_gemm_fp8_times_fp8_q(M, N, K):
    """FP8 x FP8 on MFMA: A stored as e4m3 with 128 x 128 block scales (K x M), Q
    (K x N FP32) taken to its operand form (e4m3, E8M0 scale per 32 rows and
    column), against the FP64 product of the two dequantised operands.  Error
    sources: (1) the FP8 instruction sums each group of 8 products with about 13
    bits below the group's largest product (measured on gfx950: 448 + 2^-5 is kept,
    448 + 2^-6 and 448 + 2^-9 are not, sums across groups and the accumulator
    input are exact FP32 additions), so a group errs by less than
    8 * 2^-13 * max|p| <= 2^-10 * sum|p|; (2) FP32 accumulation over K terms and
    the accumulator rescaling when the A block scale changes (two roundings per
    128-row block)."""
    rng = np.random.default_rng(M + 3 * N + 5 * K)
    X = rng.standard_normal((K, M)) * np.exp(2 * rng.standard_normal((K, 1)))
    codes, scales = fp8_ref.quantize_blocks(X)
    Adeq = fp8_ref.dequantize(codes, scales)
    Qf = (rng.standard_normal((K, N)) * np.exp(rng.standard_normal((K, 1)))).astype(np.float32)
    _, _, Qd = fp8_ref.quantize_q_operand(Qf.astype(np.float64))
    dA, dS, dQ = (torch.from_numpy(x).to(DEV) for x in (codes, scales, Qf))
    C = rf.rf_test_gemm_fp8(dA, dS, dQ, M, N, K).cpu().numpy()
    ref = Adeq.T @ Qd
    mag = np.abs(Adeq).T @ np.abs(Qd)
    bound = ((K + 2 + 2 * ((K + 127) // 128)) * U32 + 2.0 ** -10) * mag
    assert np.all(np.abs(C - ref) <= bound + 1e-30), np.max(np.abs(C - ref) / (bound + 1e-30))
    # the product really uses the e4m3 operand form of Q: the unquantised one is farther off
    if K >= 128:
        assert np.max(np.abs(C - Adeq.T @ Qf.astype(np.float64)) / (bound + 1e-30)) > 1.0
    # without split-K (one pass over K per tile): the same bound
    C1 = rf.rf_test_gemm_fp8(dA, dS, dQ, M, N, K, split=False).cpu().numpy()
    assert np.all(np.abs(C1 - ref) <= bound + 1e-30)


@pytest.mark.parametrize("bf16", [False, True])
def test_gemm_upper_triangular_b(bf16):
    rng = np.random.default_rng(9)
    M, N = 500, 300
    A = rng.standard_normal((M, N))
    R = np.triu(rng.standard_normal((N, N)))
    if bf16:
        At, A = bf16_round(A)
        Rt, R = bf16_round(R)
    else:
        At, Rt = torch.from_numpy(A.astype(np.float32)), torch.from_numpy(R.astype(np.float32))
        A, R = A.astype(np.float32).astype(np.float64), R.astype(np.float32).astype(np.float64)
    C = rf.rf_test_gemm(At.to(DEV), Rt.to(DEV), M, N, N, 1, 0, b_upper=True).cpu().numpy()
    mag = np.abs(A) @ np.abs(R)
    assert np.all(np.abs(C - A @ R) <= (N + 2) * U32 * mag + 1e-30)


# ---------------------------------------------------------------- FP64 Gram / Cholesky / inverse / eig
@pytest.mark.parametrize("K,M,N,sym", [(5000, 100, 100, True), (300, 70, 130, False), (65, 1, 1, True),
                                       (20000, 257, 257, True)])
def test_gram_f64(K, M, N, sym):
    rng = np.random.default_rng(K + M)
    X = rng.standard_normal((K, M)).astype(np.float32)
    Y = X if sym else rng.standard_normal((K, N)).astype(np.float32)
    dX = torch.from_numpy(X).to(DEV)
    dY = dX if sym else torch.from_numpy(Y).to(DEV)
    C = rf.rf_test_gram(dX, dY, sym=sym).cpu().numpy()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    ref = X64.T @ Y64
    mag = np.abs(X64).T @ np.abs(Y64)
    assert np.all(np.abs(C - ref) <= (K + 2) * 2.0 ** -53 * mag + 1e-300)
    if sym:
        assert np.array_equal(C, C.T)


@pytest.mark.parametrize("N", [1, 5, 64, 100, 129, 300, 1000, 2000, 4096])
def test_cholesky_and_inverse(N):
    rng = np.random.default_rng(N)
    X = rng.standard_normal((N + 20, N)) * np.logspace(0, -3, N)[None, :]
    G = X.T @ X
    R, Rinv, cnt = rf.rf_test_cholqr_factor(torch.from_numpy(G).to(DEV))
    R = np.triu(R.cpu().numpy())
    Rinv = Rinv.cpu().numpy()
    assert int(cnt[0].item()) == 0
    Rref = np.linalg.cholesky(G).T
    assert np.allclose(R, Rref, rtol=1e-9, atol=1e-12 * np.abs(Rref).max())
    assert np.allclose(Rinv @ R, np.eye(N), atol=1e-9)
    assert np.allclose(np.tril(Rinv, -1), 0)


def test_cholesky_flags_dependent_columns():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((60, 10)).astype(np.float32).astype(np.float64)
    X[:, 7] = X[:, 2] + X[:, 3]          # exactly dependent in FP64 (and nearly in FP32)
    G = X.T @ X
    _, Rinv, cnt = rf.rf_test_cholqr_factor(torch.from_numpy(G).to(DEV))
    assert int(cnt[0].item()) == 1
    assert np.all(np.isfinite(Rinv.cpu().numpy()))


@pytest.mark.parametrize("N,kind", [(1, "rand"), (2, "rand"), (31, "rand"), (64, "rand"), (100, "psd"),
                                    (257, "rand"), (1000, "psd"), (300, "cluster")])
def test_eig(N, kind):
    rng = np.random.default_rng(N)
    if kind == "rand":
        G = rng.standard_normal((N, N)); G = G + G.T
    elif kind == "psd":
        X = rng.standard_normal((N, 3 * N)) * np.logspace(0, -4, N)[:, None]
        G = X @ X.T
    else:
        Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
        lam = np.concatenate([np.ones(N // 3), 1e-3 * np.ones(N // 3), np.zeros(N - 2 * (N // 3))])
        G = (Q * lam) @ Q.T
        G = 0.5 * (G + G.T)
    lam, V = rf.rf_test_eig(torch.from_numpy(G).to(DEV))
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    ref = np.sort(np.linalg.eigvalsh(G))[::-1]
    nrm = np.abs(ref).max()
    e_lam = np.max(np.abs(lam - ref)) / nrm
    e_orth = np.max(np.abs(V.T @ V - np.eye(N)))
    e_res = np.max(np.abs(G @ V - V * lam[None, :])) / nrm
    print("eig N=%d %s: lam err %.2e orth %.2e resid %.2e" % (N, kind, e_lam, e_orth, e_res))
    assert np.all(np.diff(lam) <= 0)
    assert e_orth <= 1e-10
    if kind == "cluster":
        # three exactly multiple eigenvalues: Jacobi (block or classic cyclic)
        # converges only linearly here; bound what 24 sweeps deliver
        assert e_lam <= 1e-11 and e_res <= 1e-6
    else:
        assert e_lam <= 1e-12 * max(1, math.sqrt(N))
        assert e_res <= 1e-10


@pytest.mark.parametrize("N", [100, 1000])
def test_eig_fp32_output_tolerance(N):
    """The tolerance rf_svd / rf_nystrom use (1e-7): Ritz-like spectrum with a
    clustered tail; sigma = sqrt(lambda) to 1e-7 relative, residual and
    orthonormality at the FP32 level."""
    rng = np.random.default_rng(N + 1)
    sig = np.maximum(np.arange(1, N + 1) ** -1.5, 1e-4 * rng.uniform(0.33, 1.0, N))
    sig = np.sort(sig)[::-1]
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    G = (Q * sig ** 2) @ Q.T
    G = 0.5 * (G + G.T)
    lam, V, tr = rf.rf_test_eig(torch.from_numpy(G).to(DEV), trace=True, tol=1e-7)
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    ref = np.sort(np.linalg.eigvalsh(G))[::-1]
    print("sweep trace", tr.cpu().numpy()[:21])
    s_g, s_r = np.sqrt(np.maximum(lam, 0)), np.sqrt(np.maximum(ref, 0))
    assert np.max(np.abs(s_g - s_r) / s_r) < 1e-7
    assert np.max(np.abs(V.T @ V - np.eye(N))) < 1e-10
    # off-diagonal of V^T G V relative to sqrt(l_i l_j) is the tolerance
    D = V.T @ G @ V
    d = np.sqrt(np.abs(np.diag(D)))
    off = np.abs(D - np.diag(np.diag(D))) / np.maximum(np.outer(d, d), 16 * 2.2e-16 * np.linalg.norm(G) / 1e-7)
    assert off.max() < 2e-7


# ---------------------------------------------------------------- tuning table
@pytest.mark.parametrize("bf16", [False, True])
def test_gemm_every_tuned_config_is_correct(bf16):
    """Each tile / split-K choice the autotuner may install gives the product."""
    from paper_2605_09755_amd import autotune
    rng = np.random.default_rng(77)
    M, N, K = 700, 600, 5000
    dA, dB, A, B = _operands(M, N, K, 0, 0, rng, bf16)
    ref = A @ B
    mag = np.abs(A) @ np.abs(B)
    big = 1 << 62
    try:
        for tile, split in autotune.candidates(2 if bf16 else 0):
            rf.set_gemm_rules([(2 if bf16 else 0, tile, split, big, big, big)])
            C = rf.rf_test_gemm(dA, dB, M, N, K, 0, 0).cpu().numpy()
            assert np.all(np.abs(C - ref) <= (K + 2) * U32 * mag + 1e-30), (tile, split)
    finally:
        rf.set_gemm_rules([])


def test_autotune_writes_rules():
    from paper_2605_09755_amd import autotune
    try:
        rules = autotune.tune(autotune.QUICK, reps=1, log=lambda *a: None)
    finally:
        rf.set_gemm_rules([])
    assert len(rules) == 2 * len(autotune.QUICK)
    for r in rules:
        assert (r["tile"], r["split"]) in autotune.candidates(r["dtype"])
        assert r["max_m"] >= r["shape"][0] and r["max_n"] >= r["shape"][1] and r["max_k"] >= r["shape"][2]


def test_eig_graph_replays_follow_buffer_contents():
    """Repeated rf_test_eig calls on the same buffers replay one captured graph:
    each replay must read the buffers' current contents (another matrix, then the
    first again, bit-identical), with eager work and synchronisation in between."""
    N = 300
    rng = np.random.default_rng(77)
    mats = []
    for _ in range(2):
        X = rng.standard_normal((N, 2 * N)) * np.logspace(0, -3, N)[:, None]
        mats.append(X @ X.T)
    L = rf.lib()
    G = torch.empty((N, N), dtype=torch.float64, device=DEV)
    lam = torch.empty(N, dtype=torch.float64, device=DEV)
    V = torch.empty((N, N), dtype=torch.float64, device=DEV)
    ws = torch.empty(int(L.rf_test_eig_ws(N)), dtype=torch.uint8, device=DEV)
    st = rf._stream(G.device)
    results = []
    for rep, which in enumerate([0, 1, 0, 1, 0]):
        G.copy_(torch.from_numpy(mats[which]))
        rf._check("rf_test_eig", L.rf_test_eig(rf._ptr(G), N, 1e-12, rf._ptr(lam), rf._ptr(V), rf._ptr(None),
                                               rf._ptr(ws), st))
        torch.cuda.synchronize()
        results.append((which, lam.cpu().numpy().copy(), V.cpu().numpy().copy()))
        junk = torch.randn(512, 512, device=DEV) @ torch.randn(512, 512, device=DEV)  # eager work between replays
        torch.cuda.synchronize()
        del junk
    for which, l, v in results:
        ref = np.sort(np.linalg.eigvalsh(mats[which]))[::-1]
        assert np.max(np.abs(l - ref)) <= 1e-12 * np.abs(ref).max() * math.sqrt(N)
        assert np.max(np.abs(mats[which] @ v - v * l[None, :])) <= 1e-10 * np.abs(ref).max()
    for a in range(len(results)):
        for b in range(a + 1, len(results)):
            if results[a][0] == results[b][0]:
                assert np.array_equal(results[a][1], results[b][1]) and np.array_equal(results[a][2], results[b][2])
