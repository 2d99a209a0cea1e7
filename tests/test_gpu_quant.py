"""The library's storage-form kernels (rf_quantize_bf16, rf_quantize_fp8_b128)
against CPU definitions, bit for bit: torch's CPU FP32 -> BF16 conversion
(round to nearest, ties to even) and the NumPy OCP e4m3 encoder with amax/448
block scales in tests/fp8_ref.py."""
import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf
from tests import fp8_ref

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bf16_bits_cpu(x32):
    return torch.from_numpy(x32).to(torch.bfloat16).view(torch.int16).numpy()


@pytest.mark.parametrize("m,n,ld", [(333, 517, 517), (64, 1024, 1030), (1, 3, 3), (129, 7, 9)])
def test_bf16_bit_exact(m, n, ld):
    rng = np.random.default_rng(m + n)
    x = (rng.standard_normal((m, ld)) * 10.0 ** rng.uniform(-30, 30, (m, ld))).astype(np.float32)
    # exact ties: low 16 bits = 0x8000 with both parities of bit 16
    bits = x.view(np.uint32)
    bits[:, ::5] = (bits[:, ::5] & 0xFFFF0000) | 0x8000
    x[0, 0] = 0.0
    if n > 1:
        x[0, 1] = -0.0
    dA = torch.from_numpy(x).to(DEV)[:, :n]
    got = rf.rf_quantize_bf16(dA).view(torch.int16).cpu().numpy()
    assert np.array_equal(got, _bf16_bits_cpu(np.ascontiguousarray(x[:, :n])))


def test_bf16_nan_inf():
    x = np.array([[np.nan, np.inf, -np.inf, 3.0e38, -3.4e38, 1e-40]], dtype=np.float32)
    got = rf.rf_quantize_bf16(torch.from_numpy(x).to(DEV)).float().cpu().numpy()
    assert np.isnan(got[0, 0])
    assert np.array_equal(got[0, 1:], torch.from_numpy(x[0, 1:]).to(torch.bfloat16).float().numpy())


@pytest.mark.parametrize("m,n", [(300, 270), (128, 128), (1, 200), (257, 129)])
def test_fp8_block_bit_exact(m, n):
    rng = np.random.default_rng(3 * m + n)
    A = rng.standard_normal((m, n))
    # blocks of very different magnitude, an all-zero block, exact e4m3 ties
    A[:128, :128] *= 1e-6
    if m > 128 and n > 128:
        A[128:256, 128:256] *= 1e5
        A[128:256, :128] = 0.0
    A32 = A.astype(np.float32)
    codes_ref, scales_ref = fp8_ref.quantize_blocks(A32.astype(np.float64))
    codes, scales = rf.rf_quantize_fp8_b128(torch.from_numpy(A32).to(DEV))
    assert np.array_equal(scales.cpu().numpy(), scales_ref)
    assert np.array_equal(codes.cpu().numpy(), codes_ref)


def test_fp8_ties_and_saturation():
    """Values placed exactly on the midpoints of adjacent e4m3 codes (after the
    block scale) must round to the even code; the block maximum maps to 448."""
    dec = fp8_ref.DECODE[:0x7e]
    mids = (dec[:-1] + dec[1:]) / 2
    row = np.concatenate([mids, [448.0], -mids[::7]])
    A = np.zeros((2, 128), dtype=np.float32)
    A[0, :len(row[:128])] = row[:128]
    A[1, :len(row[128:256])] = row[128:256]
    A32 = A.astype(np.float32)
    codes_ref, scales_ref = fp8_ref.quantize_blocks(A32.astype(np.float64))
    assert scales_ref[0, 0] == 1.0      # amax = 448 exactly
    codes, scales = rf.rf_quantize_fp8_b128(torch.from_numpy(A32).to(DEV))
    assert np.array_equal(codes.cpu().numpy(), codes_ref)
    assert np.array_equal(scales.cpu().numpy(), scales_ref)


def test_fp8_nonfinite_encodes_nan_and_keeps_scale():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((130, 140)).astype(np.float32)
    A[5, 6] = np.nan
    A[7, 8] = np.inf
    codes, scales = rf.rf_quantize_fp8_b128(torch.from_numpy(A).to(DEV))
    codes = codes.cpu().numpy()
    B = A.copy()
    B[5, 6] = 0.0
    B[7, 8] = 0.0
    _, scales_ref = fp8_ref.quantize_blocks(B.astype(np.float64))
    assert np.array_equal(scales.cpu().numpy(), scales_ref)
    assert codes[5, 6] & 0x7F == 0x7F and codes[7, 8] & 0x7F == 0x7F


def test_fp8_large_sampled_blocks():
    """A 4096 x 8192 matrix (the precision workload's law): sampled blocks
    bit-exact against the CPU encoder."""
    g = torch.Generator(device=DEV)
    g.manual_seed(7)
    A = torch.randn((4096, 8192), generator=g, device=DEV) * 0.01
    codes, scales = rf.rf_quantize_fp8_b128(A)
    Ah = A.cpu().numpy()
    rng = np.random.default_rng(0)
    for bi, bj in zip(rng.integers(0, 32, 12), rng.integers(0, 64, 12)):
        blk = Ah[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128].astype(np.float64)
        c_ref, s_ref = fp8_ref.quantize_blocks(blk)
        assert scales[bi, bj].item() == s_ref[0, 0]
        assert np.array_equal(codes[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128].cpu().numpy(), c_ref)
    bf = rf.rf_quantize_bf16(A)
    assert torch.equal(bf.cpu(), A.cpu().to(torch.bfloat16))


@pytest.mark.parametrize("m,k", [(300, 70), (128, 256), (1, 1), (513, 300), (4096, 2000)])
def test_q_operand_form_bit_exact(m, k):
    """The FP8 operand form of Q (e4m3 codes in MFMA order, E8M0 scale per 32 rows
    and column) against tests/fp8_ref.quantize_q_operand, byte for byte: rows of
    very different magnitude, an all-zero 32-row block, exact e4m3 ties after the
    power-of-two scaling, a NaN and an Inf."""
    rng = np.random.default_rng(m + 7 * k)
    Q = rng.standard_normal((m, k)) * 10.0 ** rng.uniform(-20, 20, (m, 1)) / np.sqrt(m)
    if m >= 64:
        Q[32:64] = 0.0
    if m > 96 and k > 3:
        # ties: 448 * 2^x sets the block exponent, mids of adjacent codes below it
        Q[96, :3] = [448.0, 0.5 * (fp8_ref.DECODE[0x50] + fp8_ref.DECODE[0x51]), -3.25]
        Q[97, 0] = 0.5 * (fp8_ref.DECODE[0x52] + fp8_ref.DECODE[0x53])
    if m > 200 and k > 5:
        Q[200, 4] = np.nan
        Q[201, 5] = -np.inf
    Q32 = Q.astype(np.float32)
    codes_ref, scales_ref, _ = fp8_ref.quantize_q_operand(Q32.astype(np.float64))
    codes, scales = rf.rf_test_quant_q_fp8(torch.from_numpy(Q32).to(DEV))
    assert np.array_equal(scales.cpu().numpy(), scales_ref)
    assert np.array_equal(codes.cpu().numpy(), codes_ref)
