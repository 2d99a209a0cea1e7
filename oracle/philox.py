"""Philox4x32-10, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11.  A 4x32-bit counter is mixed with a 2x32-bit
key through ten rounds; each round multiplies counter words 0 and 2 by fixed
odd constants, splits the 64-bit products into high and low halves and
exchanges them with words 1 and 3 xor-ed with the key; the key is advanced by
two Weyl constants between rounds.

The paper being reproduced does not say how its random sketches are drawn
(Section 4 only says CountSketch and Gaussian); a counter-based generator makes
every entry of S and Omega a pure function of (seed, stream, matrix index,
position), so the oracle and the GPU can draw the same matrices independently.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# round multipliers and key increments of Philox4x32 (SC'11, Table 2 / Section 5)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.

    c0..c3: arrays (any shape, broadcastable) of counter words < 2**32.
    k0, k1: key words < 2**32 (scalars).
    Returns four uint64 arrays holding the 32-bit output words.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0          # < 2**64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def draw(index, seed, stream, b=0):
    """The four output words for 64-bit counter position `index` on
    (seed, stream, matrix b): counter = (index lo, index hi, stream, b),
    key = (seed lo, seed hi)."""
    index = np.asarray(index, dtype=np.uint64)
    seed = int(seed)
    return philox4x32_10(index & MASK32, index >> np.uint64(32),
                         np.uint64(stream), np.uint64(b),
                         seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
