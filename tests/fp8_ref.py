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


def e8m0_exponent(amax):
    """Smallest x in [-127, 127] with 448 * 2**x >= amax (-127 where amax == 0).
    With amax = f 2**E (f in [1/2, 1)) and 448 = 0.875 * 2**9 the condition reads
    2**(9 + x - E) >= f / 0.875, so x = E - 9 when f <= 0.875, else E - 8."""
    amax = np.asarray(amax, dtype=np.float64)
    f, E = np.frexp(amax)
    x = E.astype(np.int64) - 9 + (f > 0.875)
    x = np.where(amax > 0, x, -127)
    return np.clip(x, -127, 127)


def quantize_q_operand(Q):
    """The FP8 operand form of Q (m x k) read by the FP8 product A^T Q: e4m3 codes
    with one power-of-two scale per 32 rows and column, laid out as
    codes[st, jb, ch, p, lane, e] = code of row 128 st + 64 ch + 32 p + 16 (lane // 32) + e,
    column 32 jb + lane % 32, and scales[st, jb, lane, ch] = 127 + x of rows
    128 st + 64 ch + 32 (lane // 32) + [0, 32), column 32 jb + lane % 32 (jb < 8 ceil(k / 256)).
    Returns (codes, scales) flattened to bytes and the dequantised Q (m x k)."""
    Q = np.asarray(Q, dtype=np.float64)
    m, k = Q.shape
    S = -(-m // 128)
    njb = -(-k // 256) * 8
    Mp, Kp = 128 * S, 32 * njb
    Qp = np.zeros((Mp, Kp))
    Qp[:m, :k] = Q
    fin = np.isfinite(Qp)
    blocks = np.where(fin, np.abs(Qp), 0.0).reshape(Mp // 32, 32, Kp)
    x = e8m0_exponent(blocks.max(axis=1))                      # (Mp/32, Kp)
    X = np.repeat(x, 32, axis=0)                               # per element
    with np.errstate(invalid="ignore"):
        codes_full = encode(np.where(fin, np.ldexp(np.where(fin, Qp, 0.0), -X), 0.0))
    bad = ~fin
    codes_full[bad] = np.where(Qp[bad] < 0, 0xFF, 0x7F).astype(np.uint8)
    deq = decode(codes_full) * np.ldexp(1.0, X)
    codes = codes_full.reshape(S, 2, 2, 2, 16, njb, 32).transpose(0, 5, 1, 2, 3, 6, 4).reshape(-1)
    scales = (x + 127).astype(np.uint8).reshape(S, 2, 2, njb, 32).transpose(0, 3, 2, 4, 1).reshape(-1)
    return codes, scales, deq[:m, :k]
