"""GPU tests of the inner SpMV's diagonal storage.  A stencil-like matrix
(every nonzero on at most 8 diagonals j - i, rows of at most 8 nonzeros) is
read by diagonal, without its column indices.  Each row sum keeps the CSR
path's order and rounding, and the tiles, lanes and sketch scatter stay the
same, so whole solves must equal the CSR path's bit for bit.  (The systems
here have whole 64-row tiles, or a last tile of at least 32 rows: the CSR
path sums the rows of a shorter tile with lane groups, in another order.)
The CSR path itself is checked against the oracle by the other solve
tests."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, ragged_powerlaw

pytestmark = [pytest.mark.gpu, requires_gpu]


def _system(name):
    if name == "convdiff2d_64":
        A, nd = W.convdiff2d(64, 1.0, (10.0, 10.0)), 5
    elif name == "convdiff3d_16":
        A, nd = W.convdiff3d(16, 1.0, (50.0, 50.0, 50.0)), 7
    elif name == "convdiff3d_10":   # 1000 rows: a last tile of 40 rows
        A, nd = W.convdiff3d(10, 1.0, (50.0, 50.0, 50.0)), 7
    else:
        A, nd = W.convdiff3d_varcoef(16, np.random.default_rng([31, 0])), 7
    b = np.random.default_rng([32, 1]).uniform(-1.0, 1.0, A.n)
    return A, b, nd


def _pair(A, b, **prm):
    rp, ci, va = to_dev(A)
    out = {}
    for fmt in ("csr", "auto"):
        x, info = P.solve(rp, ci, va, tvec(b), matrix_format=fmt, **prm)
        out[fmt] = (x.cpu().numpy(), info)
    return out


def _same(out):
    (xc, ic), (xd, idd) = out["csr"], out["auto"]
    assert list(ic["inner_k"]) == list(idd["inner_k"])
    assert list(ic["stop_reason"]) == list(idd["stop_reason"])
    assert np.array_equal(np.asarray(ic["residual_history"]), np.asarray(idd["residual_history"]))
    assert np.array_equal(xc, xd)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("t", [0, 2, 5])
@pytest.mark.parametrize("name", ["convdiff2d_64", "convdiff3d_16", "convdiff3d_10",
                                  "varcoef3d_16"])
def test_diagonal_storage_equals_csr_bit_for_bit(name, t, precision):
    A, b, nd = _system(name)
    out = _pair(A, b, m=30, t=t, s=90, zeta=8, tol=1e-10, seed=13, max_outer=15,
                precision=precision)
    assert out["csr"][1]["dia_diagonals"] == 0
    assert out["auto"][1]["dia_diagonals"] == nd
    _same(out)


@pytest.mark.parametrize("src", ["table", "gen"])
def test_diagonal_storage_with_either_sketch_source(src):
    A, b, _ = _system("varcoef3d_16")
    out = _pair(A, b, m=30, t=2, s=90, zeta=8, tol=1e-10, seed=13, max_outer=15,
                sketch_source=src)
    assert out["auto"][1]["sketch_generated"] == (src == "gen")
    _same(out)


def test_diagonal_storage_in_the_adjoint():
    A, b, _ = _system("convdiff3d_16")
    rp, ci, va = to_dev(A)
    prm = dict(m=30, t=2, s=90, zeta=8, tol=1e-10, seed=13, max_outer=15)
    x, _ = P.solve(rp, ci, va, tvec(b), matrix_format="csr", **prm)
    g = tvec(np.random.default_rng([33, 3]).uniform(-1.0, 1.0, A.n))
    res = {}
    for fmt in ("csr", "auto"):
        lam, gv, info = P.solve_adjoint(rp, ci, va, g, x, matrix_format=fmt, **prm)
        res[fmt] = (lam.cpu().numpy(), gv.cpu().numpy(), info)
    assert res["auto"][2]["dia_diagonals"] == 7 and res["csr"][2]["dia_diagonals"] == 0
    assert np.array_equal(res["csr"][0], res["auto"][0])
    assert np.array_equal(res["csr"][1], res["auto"][1])


def test_matrices_off_a_few_diagonals_stay_csr():
    # rows longer than 8 nonzeros
    A = ragged_powerlaw(3000, 34)
    b = np.random.default_rng([34, 1]).standard_normal(A.n)
    x, info = P.solve(*to_dev(A), tvec(b), m=30, t=2, s=90, zeta=8, tol=1e-8, seed=13,
                      max_outer=20)
    assert info["dia_diagonals"] == 0 and info["converged"]
    # a stencil with one entry off its diagonals (and its transpose)
    S = W.convdiff2d(32, 1.0, (10.0, 10.0)).to_scipy().tolil()
    S[5, 700] = -0.01
    S[700, 5] = -0.01
    S = sp.csr_matrix(S)
    S.sort_indices()
    A2 = W.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
               S.data.astype(np.float64))
    b2 = np.random.default_rng([35, 1]).uniform(0.0, 1.0, A2.n)
    x2, i2 = P.solve(*to_dev(A2), tvec(b2), m=30, t=2, s=90, zeta=8, tol=1e-8, seed=13,
                     max_outer=20)
    assert i2["dia_diagonals"] == 0 and i2["converged"]
    assert np.linalg.norm(S @ x2.cpu().numpy() - b2) <= 1e-8 * np.linalg.norm(b2) * (1 + 1e-6)


def test_matrix_format_is_checked():
    A, b, _ = _system("convdiff2d_64")
    with pytest.raises(KeyError):
        P.solve(*to_dev(A), tvec(b), m=30, t=2, s=90, matrix_format="ell")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["convdiff2d_64", "convdiff3d_10", "varcoef3d_16"])
def test_ilu_preconditioned_solve_by_diagonal_equals_csr_bit_for_bit(name, precision):
    """ILU(0) right preconditioning: the inner SpMV reads M^{-1} u_i, by
    diagonal or through CSR, with the same results."""
    A, b, _ = _system(name)
    out = _pair(A, b, m=30, t=2, s=90, zeta=8, tol=1e-10, seed=13, max_outer=15,
                precision=precision, precond="ilu0")
    _same(out)
