"""Sparse sign sketch S (s x n), generated column by column from Philox4x32-10.

The paper applies a Clarkson-Woodruff sketch, one +-1 per column in a random
row (Section 4.1); the solver here generalises it to zeta distinct nonzero
rows per column with independent random signs and values +-1/sqrt(zeta), so
that E||Sx||^2 = ||x||^2 (zeta = 1 is the paper's sketch).  S is a subspace
embedding in the sense of eq. (1.1) with high probability.

Definition of column r (0-based), for a 64-bit seed:
* key = (seed mod 2^32, seed div 2^32);
* random words w[0], w[1], ...: block c of four words is
  Philox4x32-10(counter = (r, c, 0, 0), key), word 4c+q = output q;
* rows by Floyd's sampling (Bentley & Floyd, "Programming pearls: a sample of
  brilliance", CACM 30(9), 1987): for d = 0..zeta-1, with i = s - zeta + d,
  u = w[d] >> 1 (31 bits), t = floor(u (i+1) / 2^31) is uniform on 0..i;
  the d-th row is t unless t was already chosen, in which case it is i;
* the sign of the d-th nonzero is -1 if w[d] is odd, else +1.

Pins (tests/test_oracle_sketch.py): exactly zeta distinct rows per column,
uniform row occupancy and balanced signs (chi-square), E||Sx||^2 = ||x||^2,
singular values of S U for orthonormal U inside the Marchenko-Pastur edges
(the subspace-embedding property of eq. (1.1)), and a brute-force check of
Floyd's sampling on tiny (s, zeta) against the exact uniform distribution.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_10_vec

SKETCH_CTR_LAYOUT = "(column, block, 0, 0)"


def sketch_columns(n: int, s: int, zeta: int, seed: int, cols=None):
    """Rows (len(cols) x zeta, int64) and signs (+1/-1, int8) of columns of S."""
    if not (1 <= zeta <= s):
        raise ValueError("need 1 <= zeta <= s")
    r = np.arange(n, dtype=np.uint64) if cols is None else np.asarray(cols, dtype=np.uint64)
    k0 = seed & 0xFFFFFFFF
    k1 = (seed >> 32) & 0xFFFFFFFF
    nblk = (zeta + 3) // 4
    words = []
    zero = np.zeros_like(r)
    for c in range(nblk):
        out = philox4x32_10_vec(r, zero + np.uint64(c), zero, zero, k0, k1)
        words.extend(out)
    rows = np.empty((r.shape[0], zeta), dtype=np.int64)
    signs = np.empty((r.shape[0], zeta), dtype=np.int8)
    for d in range(zeta):
        i = s - zeta + d
        w = words[d]
        u = w >> np.uint64(1)
        t = ((u * np.uint64(i + 1)) >> np.uint64(31)).astype(np.int64)
        taken = np.zeros(r.shape[0], dtype=bool)
        for e in range(d):
            taken |= rows[:, e] == t
        rows[:, d] = np.where(taken, i, t)
        signs[:, d] = np.where((w & np.uint64(1)) == 1, -1, 1)
    return rows, signs


def sketch_scale(zeta: int) -> float:
    """The common magnitude 1/sqrt(zeta) of every nonzero of S."""
    return 1.0 / math.sqrt(zeta)


def sketch_matrix(n: int, s: int, zeta: int, seed: int):
    """S as (scipy CSR s x n holding the +-1 pattern, scale 1/sqrt(zeta))."""
    rows, signs = sketch_columns(n, s, zeta, seed)
    cols = np.repeat(np.arange(n, dtype=np.int64), zeta)
    S = sp.csr_matrix((signs.reshape(-1).astype(np.float64), (rows.reshape(-1), cols)), shape=(s, n))
    return S, sketch_scale(zeta)


def apply_sketch(S, w):
    """S w for S given as (pattern, scale): the +-1 sum, then one scaling."""
    pat, scale = S
    return scale * (pat @ w)
