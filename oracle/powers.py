"""Matrix powers: the t = 0 inner basis generated several vectors at a time.

Section 5 suggests precomputing a few matrix powers A, A^2, ..., A^p for the
t = 0 variant, whose inner basis needs no inner products: with t = 0 the
truncated Arnoldi of Section 4.1 only normalises, so b_{i+l} is A^l b_i
divided by its norm, and the vectors A b_i, ..., A^p b_i (and their
sketches and norms) can be formed before any of them is normalised.

This module is that definition written out: repeated products with A, then
the sketch and the norm of each product.  Pins (tests/test_oracle_powers.py):
closed form for a diagonal A; normalised, the products are the t = 0 basis
of the oracle's sGMRES cycle.
"""
from __future__ import annotations

import numpy as np


def matrix_powers(A, u, p, sketch=None):
    """Y[:, l-1] = A^l u for l = 1..p, with C[:, l-1] = S A^l u (when a sketch
    function is given) and norms[l-1] = ||A^l u||."""
    y = np.asarray(u, dtype=np.float64)
    cols, sks, norms = [], [], []
    for _ in range(p):
        y = A @ y
        cols.append(y)
        norms.append(float(np.linalg.norm(y)))
        if sketch is not None:
            sks.append(sketch(y))
    Y = np.column_stack(cols)
    C = np.column_stack(sks) if sks else None
    return Y, C, np.asarray(norms)
