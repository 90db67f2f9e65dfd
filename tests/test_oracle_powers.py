"""Pins of oracle/powers.py (matrix powers for the t = 0 basis, Section 5)."""
import numpy as np
import scipy.sparse as sp

import oracle
from oracle.powers import matrix_powers
import workloads as W


def test_diagonal_closed_form():
    d = np.linspace(0.5, 2.0, 50)
    u = np.random.default_rng(1).standard_normal(50)
    Y, C, nrm = matrix_powers(sp.diags(d).tocsr(), u, 4)
    for l in range(1, 5):
        assert np.allclose(Y[:, l - 1], d ** l * u, rtol=1e-15, atol=0)
        assert np.isclose(nrm[l - 1], np.linalg.norm(d ** l * u), rtol=1e-15)


def test_normalised_powers_are_the_t0_basis():
    A = W.convdiff2d(10, 1.0, (10.0, 10.0)).to_scipy()
    n = A.shape[0]
    v = np.random.default_rng(2).standard_normal(n)
    v /= np.linalg.norm(v)
    S = oracle.sketch_matrix(n, 40, 8, 5)
    sk = lambda w: oracle.apply_sketch(S, w)  # noqa: E731
    p = 5
    _, info = oracle.sgmres_cycle(A, v, sk, m=p + 1, t=0, tol_abs=0.0, factor=1.0,
                                  cond_threshold=1e300, forced_k=p + 1)
    Y, C, nrm = matrix_powers(A, v, p, sk)
    for l in range(1, p + 1):
        assert np.allclose(Y[:, l - 1] / nrm[l - 1], info["basis"][l], rtol=1e-13, atol=1e-15)
        assert np.allclose(C[:, l - 1], sk(Y[:, l - 1]), rtol=1e-15, atol=0)
