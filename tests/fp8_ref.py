"""Reference OCP FP8 E4M3 encode/decode for building FP8 test inputs (NumPy).

decode: e4m3 byte -> value = (-1)^s 2^(e-7) (1 + m/8) for e >= 1, 2^-6 m/8 for
e = 0; code 0x7f/0xff is NaN.  encode: round to nearest representable value,
ties to even mantissa, saturating at +-448.  Block scales: one FP32 scale per
128 x 128 block, amax / 448 (1 if the block is all zero).
"""
import numpy as np

_codes = np.arange(256)
_s = (_codes >> 7) & 1
_e = (_codes >> 3) & 0xF
_m = _codes & 7
_vals = np.where(_e == 0, (2.0 ** -6) * _m / 8.0, (2.0 ** (_e - 7.0)) * (1.0 + _m / 8.0))
_vals = np.where(_s == 1, -_vals, _vals)
_nan = (_e == 15) & (_m == 7)
DECODE = np.where(_nan, np.nan, _vals)

# positive finite codes sorted by value (0x00..0x7e)
_pos = np.arange(0x7F)
_posv = DECODE[_pos]


def decode(b):
    return DECODE[np.asarray(b, dtype=np.uint8)]


def encode(x):
    x = np.asarray(x, dtype=np.float64)
    ax = np.minimum(np.abs(x), 448.0)
    i = np.searchsorted(_posv, ax)              # first code with value >= ax
    i = np.clip(i, 1, len(_posv) - 1)
    lo, hi = _pos[i - 1], _pos[i]
    dlo, dhi = ax - _posv[i - 1], _posv[i] - ax
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((hi & 1) == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(ax == 0, 0, code)
    code = np.where(x < 0, code | 0x80, code)
    return code.astype(np.uint8)


def quantize_blocks(A, blk=128):
    m, n = A.shape
    bm, bn = -(-m // blk), -(-n // blk)
    scales = np.ones((bm, bn), dtype=np.float32)
    codes = np.zeros((m, n), dtype=np.uint8)
    for bi in range(bm):
        for bj in range(bn):
            blkA = A[bi * blk:(bi + 1) * blk, bj * blk:(bj + 1) * blk]
            amax = float(np.max(np.abs(blkA))) if blkA.size else 0.0
            sc = np.float32(amax / 448.0) if amax > 0 else np.float32(1.0)
            scales[bi, bj] = sc
            codes[bi * blk:(bi + 1) * blk, bj * blk:(bj + 1) * blk] = encode(blkA / np.float64(sc))
    return codes, scales


def dequantize(codes, scales, blk=128):
    m, n = codes.shape
    S = np.repeat(np.repeat(scales.astype(np.float64), blk, 0), blk, 1)[:m, :n]
    return decode(codes) * S
