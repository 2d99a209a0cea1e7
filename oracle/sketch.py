"""The random matrices of the method: the sparse sign sketch S and the Gaussian
start matrix Omega.

* S (n x r1) is "CountSketch-type": every row of S (one per column of A) holds s
  nonzeros of the form +-1/sqrt(s)  -- Lemma 3.2, item 2; s = 1 is the plain
  CountSketch used in the experiments of Section 4.
* Omega (r1 x r2) is Gaussian -- Algorithm 1 inputs, Theorem 2.1, Section 4.

Readings taken where the paper is silent (listed in the design doc as well):
* placement of the s nonzeros: block layout.  The r1 columns of S are cut into
  s contiguous blocks [lo_t, hi_t), lo_t = floor(t*r1/s); nonzero t of row j
  sits in block t at a uniformly hashed column.  This gives exactly s distinct
  columns per row without rejection, and s = 1 is CountSketch.
* hash: Philox4x32-10 on counter (j*s + t, stream, b); bucket = lo_t +
  floor(x0 * w_t / 2**32) (multiply-shift range reduction), sign = -1 iff the
  top bit of x1 is set.
* Omega: N(0,1) entries by the Box-Muller transform (Box & Muller, 1958) of
  Philox words; entries 4p..4p+3 (row-major) come from counter p.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
import math
import numpy as np
import scipy.sparse as sp

from .philox import draw

STREAM_S1 = 0      # S of Algorithm 1 / S1 of Algorithm 2 / S of Algorithm 3
STREAM_OMEGA = 1   # Omega
STREAM_S2 = 2      # S2 of Algorithm 2
STREAM_DENSE = 4   # dense sub-Gaussian S (Lemma 3.2, item 1)
STREAM_SRHT_D = 5  # random signs D of the SRHT (Lemma 3.2, item 3)
STREAM_SRHT_P = 6  # the sampled column subset of the SRHT
SIGN_BIT = np.int64(1) << 31

SKETCH_FAMILIES = ("sparse", "rademacher", "gaussian", "srht")


def block_bounds(r1, s):
    """lo_t for t = 0..s (so block t is [lo[t], lo[t+1]))."""
    return np.array([(t * r1) // s for t in range(s + 1)], dtype=np.int64)


def sketch_table(n, s, r1, seed, stream=STREAM_S1, b=0):
    """Bucket/sign table of an n x r1 sparse sign sketch with s nonzeros per row.

    Returns int32 array (n, s): entry (j, t) = bucket | (negative << 31), bucket
    in [lo_t, lo_{t+1}).  Integer arithmetic only, so the GPU must match bit
    for bit.
    """
    if not (1 <= s <= r1):
        raise ValueError("need 1 <= s <= r1")
    lo = block_bounds(r1, s)
    w = (lo[1:] - lo[:-1]).astype(np.uint64)
    idx = np.arange(n, dtype=np.uint64)[:, None] * np.uint64(s) + np.arange(s, dtype=np.uint64)[None, :]
    x0, x1, _, _ = draw(idx, seed, stream, b)
    bucket = lo[:-1][None, :].astype(np.uint64) + ((x0 * w[None, :]) >> np.uint64(32))
    neg = (x1 >> np.uint64(31)).astype(np.int64)
    entry = bucket.astype(np.int64) | (neg << 31)
    return entry.astype(np.uint32).view(np.int32).reshape(n, s)


def decode_table(table):
    """(bucket int64 array, sign float64 array of +-1) from a table."""
    t = table.astype(np.int64) & 0xFFFFFFFF
    bucket = t & 0x7FFFFFFF
    sign = np.where(t >> 31, -1.0, 1.0)
    return bucket, sign


def sketch_matrix(table, r1):
    """S as a scipy CSR matrix (n x r1) with entries sign/sqrt(s)."""
    n, s = table.shape
    bucket, sign = decode_table(table)
    rows = np.repeat(np.arange(n), s)
    vals = (sign / math.sqrt(s)).ravel()
    return sp.csr_matrix((vals, (rows, bucket.ravel())), shape=(n, r1))


def gaussian(rows, cols, seed, stream=STREAM_OMEGA, b=0):
    """rows x cols matrix of N(0,1) entries (float64), row-major position e uses
    Philox counter e // 4; within a counter the word pairs (x0, x1) and (x2, x3)
    each give two normals by Box-Muller: u = (x + 1/2) / 2**32 in (0, 1),
    z_even = sqrt(-2 ln u_a) cos(2 pi u_b), z_odd = sqrt(-2 ln u_a) sin(2 pi u_b)."""
    total = rows * cols
    ncnt = (total + 3) // 4
    x0, x1, x2, x3 = draw(np.arange(ncnt, dtype=np.uint64), seed, stream, b)
    scale = 2.0 ** -32

    def pair(xa, xb):
        ua = (xa.astype(np.float64) + 0.5) * scale
        ub = (xb.astype(np.float64) + 0.5) * scale
        rad = np.sqrt(-2.0 * np.log(ua))
        return rad * np.cos(2.0 * np.pi * ub), rad * np.sin(2.0 * np.pi * ub)

    z0, z1 = pair(x0, x1)
    z2, z3 = pair(x2, x3)
    z = np.stack([z0, z1, z2, z3], axis=1).ravel()[:total]
    return z.reshape(rows, cols)


def omega(r1, r2, seed, b=0, dtype=np.float32):
    """Omega as the GPU stores it (rounded to `dtype`), returned in float64."""
    return gaussian(r1, r2, seed, STREAM_OMEGA, b).astype(dtype).astype(np.float64)


# ---- Lemma 3.2, item 1: dense sub-Gaussian sketches ----------------------------
def dense_sketch(n, r1, seed, kind, b=0):
    """S (n x r1) with independent entries scaled by 1/sqrt(r1) (Lemma 3.2 item 1).

    kind "rademacher": +-1/sqrt(r1); entry e = i*r1 + j is negative iff the top
    bit of word x0 of Philox counter e (stream 4) is set.
    kind "gaussian": N(0, 1/r1) = gaussian(n, r1, seed, stream 4) / sqrt(r1),
    with the FP32 rounding of the N(0,1) draws the GPU stores."""
    if kind == "rademacher":
        x0, _, _, _ = draw(np.arange(n * r1, dtype=np.uint64), seed, STREAM_DENSE, b)
        sign = np.where(x0 >> np.uint64(31), -1.0, 1.0)
        return sign.reshape(n, r1) / math.sqrt(r1)
    if kind == "gaussian":
        z = gaussian(n, r1, seed, STREAM_DENSE, b).astype(np.float32).astype(np.float64)
        return z / math.sqrt(r1)
    raise ValueError(kind)


# ---- Lemma 3.2, item 3: subsampled randomised Hadamard transform ---------------
def srht_size(n):
    """n' = the smallest power of two >= n (A is padded with zero columns)."""
    p = 1
    while p < n:
        p *= 2
    return p


def _feistel(x, bits, seed, b):
    """Keyed permutation of [0, 2**bits) (bits even): four Feistel rounds on two
    halves of bits/2 bits, round function = word x0 of Philox counter
    (half | round << 32) on stream 6 (Luby-Rackoff construction)."""
    h = bits // 2
    mask = np.uint64((1 << h) - 1)
    left = (x >> np.uint64(h)) & mask
    right = x & mask
    for rnd in range(4):
        f, _, _, _ = draw(right | (np.uint64(rnd) << np.uint64(32)), seed, STREAM_SRHT_P, b)
        left, right = right, (left ^ f) & mask
    return (left << np.uint64(h)) | right


def srht_draws(n, r1, seed, b=0):
    """(d, picks) of S = D H I_{:,P} / sqrt(r1) (Lemma 3.2 item 3) on n' = srht_size(n).

    d: n' signs, d_j = -1 iff the top bit of x0 of Philox counter j (stream 5) is set.
    picks: the r1-element subset P of [0, n'), ascending: the images of 0..r1-1
    under a keyed permutation of [0, n') -- a 4-round Feistel network on the
    even number of bits >= log2 n', walked along its cycle until the value falls
    below n' (cycle walking keeps it a permutation of [0, n'))."""
    n2 = srht_size(n)
    if not (1 <= r1 <= n2):
        raise ValueError("need 1 <= r1 <= n'")
    x0, _, _, _ = draw(np.arange(n2, dtype=np.uint64), seed, STREAM_SRHT_D, b)
    d = np.where(x0 >> np.uint64(31), -1.0, 1.0)
    bits = max(2, (n2 - 1).bit_length())
    bits += bits & 1
    v = _feistel(np.arange(r1, dtype=np.uint64), bits, seed, b)
    out = v >= np.uint64(n2)
    while np.any(out):                      # cycle walking, element by element
        v[out] = _feistel(v[out], bits, seed, b)
        out = v >= np.uint64(n2)
    return d, np.sort(v.astype(np.int64))


def srht_matrix(n, r1, seed, b=0):
    """The SRHT as a dense n x r1 matrix: S = D H[:, P] / sqrt(r1), H the
    Sylvester-Hadamard matrix of order n' (entries +-1, H H^T = n' I), rows
    restricted to the first n (the zero padding of A)."""
    import scipy.linalg as sla
    d, picks = srht_draws(n, r1, seed, b)
    H = sla.hadamard(srht_size(n))
    return (d[:, None] * H[:, picks])[:n] / math.sqrt(r1)
