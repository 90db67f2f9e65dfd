"""Philox counter-based generators, written from their published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, Section 3 (the Philox S-box: a
round multiplies two of the four counter words by fixed odd constants, takes
the high and low halves of each product, xors the high halves with the other
two words and the round key, and permutes; the key is bumped by Weyl
constants between rounds; 10 rounds).

Pins (tests/test_oracle_philox.py):
* the 4x64 instance equals ``numpy.random.Philox`` (a library implementation
  of Philox4x64-10) bit for bit, which fixes the round structure, the
  permutation and the key schedule;
* the 4x32 instance reproduces the published known-answer vectors of the
  Random123 distribution (tests/golden/philox4x32_10_kat.txt).
"""
from __future__ import annotations

import numpy as np

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1

# multipliers and Weyl key increments (Salmon et al., Section 3)
PHILOX_M4x32 = (0xD2511F53, 0xCD9E8D57)
PHILOX_W32 = (0x9E3779B9, 0xBB67AE85)
PHILOX_M4x64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def _philox4(ctr, key, bits, mults, weyl, rounds=10):
    mask = (1 << bits) - 1
    c0, c1, c2, c3 = (int(v) & mask for v in ctr)
    k0, k1 = (int(v) & mask for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + weyl[0]) & mask
            k1 = (k1 + weyl[1]) & mask
        p0 = mults[0] * c0
        p1 = mults[1] * c2
        hi0, lo0 = p0 >> bits, p0 & mask
        hi1, lo1 = p1 >> bits, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [c0, c1, c2, c3]


def philox4x32_10(ctr, key):
    """Philox4x32-10 on one 4-word counter and 2-word key (Python ints)."""
    return _philox4(ctr, key, 32, PHILOX_M4x32, PHILOX_W32)


def philox4x64_10(ctr, key):
    """Philox4x64-10 on one 4-word counter and 2-word key (Python ints)."""
    return _philox4(ctr, key, 64, PHILOX_M4x64, PHILOX_W64)


def philox4x32_10_vec(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32-10: counter words are equal-length uint arrays.

    32x32-bit products fit in uint64, so the high and low halves are exact.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & np.uint64(M32)
    c1 = np.asarray(c1, dtype=np.uint64) & np.uint64(M32)
    c2 = np.asarray(c2, dtype=np.uint64) & np.uint64(M32)
    c3 = np.asarray(c3, dtype=np.uint64) & np.uint64(M32)
    k0 = int(k0) & M32
    k1 = int(k1) & M32
    m0 = np.uint64(PHILOX_M4x32[0])
    m1 = np.uint64(PHILOX_M4x32[1])
    s32 = np.uint64(32)
    msk = np.uint64(M32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W32[0]) & M32
            k1 = (k1 + PHILOX_W32[1]) & M32
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & msk
        hi1, lo1 = p1 >> s32, p1 & msk
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return c0, c1, c2, c3
