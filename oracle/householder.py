"""Householder QR of the sketched matrix S A B_k, grown one column at a time.

The sketched least-squares problem y_k = argmin ||S v_j - S A B_k y|| of
eq. (1.2) / Section 3 is solved by a QR factorisation of S A B_k (Section 3,
condition C2 remark: the same factorisation gives the condition number).  This
is the textbook Householder algorithm (Golub & Van Loan, Matrix Computations,
Algs. 5.1.1 and 5.2.1): a new column is multiplied by the existing reflectors
in order, then a new reflector annihilates its subdiagonal part; the
right-hand side is carried along as d = Q^T S v_j, so the least-squares
residual norm is ||d[k:]|| (Golub & Van Loan, Section 5.3.3) and y solves
R_k y = d[:k].

Reflector convention (as LAPACK's dlarfg): for x = [alpha; x2],
beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta, v = [1; x2/(alpha-beta)];
tau = 0 when x2 = 0.

Pins (tests/test_oracle_qr.py): R agrees with numpy.linalg.qr up to row signs,
Q^T Q = I and QR = C to rounding, the residual norm equals the one of a
dense least-squares solve on well-conditioned problems.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


class HouseholderQR:
    def __init__(self, s: int, kmax: int):
        self.s = s
        self.refl = []  # (v restricted to rows l..s-1, tau)
        self.R = np.zeros((kmax, kmax))
        self.k = 0
        self.d = None

    def set_rhs(self, d0):
        self.d = np.array(d0, dtype=np.float64, copy=True)

    def append(self, col):
        k = self.k
        c = np.array(col, dtype=np.float64, copy=True)
        for l, (v, tau) in enumerate(self.refl):
            c[l:] -= tau * v * (v @ c[l:])
        alpha = c[k]
        x2 = c[k + 1:]
        xnorm = float(np.linalg.norm(x2))
        if xnorm == 0.0:
            tau, beta = 0.0, alpha
            v = np.zeros(self.s - k)
            v[0] = 1.0
        else:
            beta = -math.copysign(math.hypot(alpha, xnorm), alpha)
            tau = (beta - alpha) / beta
            v = np.concatenate(([1.0], x2 / (alpha - beta)))
        self.R[:k, k] = c[:k]
        self.R[k, k] = beta
        if self.d is not None:
            self.d[k:] -= tau * v * (v @ self.d[k:])
        self.refl.append((v, tau))
        self.k += 1
        return self.R[:k + 1, k]

    def residual_norm(self, k=None):
        """||d[k:]||: the least-squares residual with the first k columns.

        Only valid for k = self.k (the current factorisation)."""
        k = self.k if k is None else k
        return float(np.linalg.norm(self.d[k:]))

    def solve(self, k):
        """y with R[:k,:k] y = d[:k] (leading k columns; d[:k] is not touched
        by reflectors k+1, k+2, ...)."""
        return sla.solve_triangular(self.R[:k, :k], self.d[:k], lower=False)
