"""Incremental 2-norm condition estimate of an upper-triangular matrix.

Condition C2 of Section 3 stops the inner sGMRES when cond(S A B_k) exceeds a
threshold, noting that the condition number follows cheaply from the QR
factor R_k of S A B_k.  cond(S A B_k) = cond(R_k); this module estimates it
with incremental condition estimation (C. Bischof, "Incremental condition
estimation", SIAM J. Matrix Anal. Appl. 11(2), 1990), updated once per new
column in O(k) work.

Appending a column [v; gamma] to R (k x k -> (k+1) x (k+1)):
* largest singular value: keep a unit x with sigma = ||x^T R||; the new
  vector is [s x; c] with (s, c) the top unit eigenvector of
  [[sigma^2 + a^2, a gamma], [a gamma, gamma^2]], a = x.v, and the new
  sigma^2 is its top eigenvalue;
* smallest singular value: keep a unit x with z = R^{-T} x, ||z|| estimating
  1/sigma_min; the new z is [s z; (c - s b)/gamma] with (s, c) the top unit
  eigenvector of [[||z||^2 + b^2/gamma^2, -b/gamma^2], [-b/gamma^2,
  1/gamma^2]], b = z.v, and the new ||z||^2 is its top eigenvalue.
The estimate is sigma * ||z|| (a lower bound of the true condition number; it
is exact for k <= 2 and for diagonal R).  gamma = 0 gives +inf.

Pins (tests/test_oracle_ice.py): exact on 1x1, 2x2 and diagonal matrices,
never above the SVD condition number, and within a small factor of it on
random and graded triangular matrices.
"""
from __future__ import annotations

import math

import numpy as np


def _top_eig(a, b, d):
    """Top eigenvalue and unit eigenvector of the symmetric [[a, b], [b, d]]."""
    w, V = np.linalg.eigh(np.array([[a, b], [b, d]], dtype=np.float64))
    return float(w[1]), float(V[0, 1]), float(V[1, 1])


class IncrementalCond:
    def __init__(self):
        self.k = 0
        self.x = None       # unit vector for sigma_max
        self.smax = 0.0
        self.z = None       # R^{-T} x for sigma_min
        self.znorm = 0.0
        self.singular = False

    def append(self, col) -> float:
        col = np.asarray(col, dtype=np.float64)
        gamma = float(col[-1])
        v = col[:-1]
        if self.singular or gamma == 0.0:
            self.singular = True
            self.k += 1
            return math.inf
        if self.k == 0:
            self.x = np.array([1.0])
            self.smax = abs(gamma)
            self.z = np.array([1.0 / gamma])
            self.znorm = 1.0 / abs(gamma)
        else:
            a = float(self.x @ v)
            lam, s, c = _top_eig(self.smax ** 2 + a * a, a * gamma, gamma * gamma)
            self.x = np.concatenate((s * self.x, [c]))
            self.smax = math.sqrt(lam)
            b = float(self.z @ v)
            g2 = gamma * gamma
            lam, s, c = _top_eig(self.znorm ** 2 + b * b / g2, -b / g2, 1.0 / g2)
            self.z = np.concatenate((s * self.z, [(c - s * b) / gamma]))
            self.znorm = math.sqrt(lam)
        self.k += 1
        return self.smax * self.znorm

    @property
    def estimate(self) -> float:
        return math.inf if self.singular else self.smax * self.znorm
