"""Pins of the oracle's ILU(0) right preconditioner (oracle/ilu.py) and of
its use in sketched FGMRES: library LU where ILU(0) is exact, the defining
property (L U)_ij = a_ij on the pattern, library triangular solves, the
colouring against the sequential greedy colouring it must equal."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import ilu as I
import workloads as W


def _tridiag(n=40, seed=0):
    rng = np.random.default_rng(seed)
    lo, up = rng.uniform(-1, 0, n - 1), rng.uniform(-1, 0, n - 1)
    d = 3.0 + rng.uniform(0, 1, n)
    return sp.diags([lo, d, up], [-1, 0, 1], format="csr")


def _matrices():
    return {
        "convdiff2d_12": W.convdiff2d(12, 1.0, (20.0, 5.0)).to_scipy(),
        "powerlaw_200": W.powerlaw_random(200, np.random.default_rng(3), Lmin=4, Lmax=30,
                                          mean=8).to_scipy(),
        "varcoef3d_6": W.convdiff3d_varcoef(6, np.random.default_rng(4)).to_scipy(),
    }


def test_tridiagonal_natural_order_is_exact_lu():
    """No fill-in exists for a tridiagonal matrix in the natural order, so
    ILU(0) is the LU factorisation (library LU, natural order, no pivoting)."""
    A = _tridiag()
    M = I.ILU0(A, "natural")
    L, U = M.factors()
    lu = spla.splu(A.tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    assert np.array_equal(lu.perm_r, np.arange(A.shape[0]))
    assert np.array_equal(lu.perm_c, np.arange(A.shape[0]))
    assert np.allclose(L.toarray(), lu.L.toarray(), rtol=1e-13, atol=1e-15)
    assert np.allclose(U.toarray(), lu.U.toarray(), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind", ["natural", "multicolor"])
@pytest.mark.parametrize("name", ["convdiff2d_12", "powerlaw_200", "varcoef3d_6"])
def test_lu_equals_a_on_the_pattern(name, kind):
    """The defining property of ILU(0) (in the elimination order): the
    product of the factors equals A wherever A has an entry."""
    A = _matrices()[name]
    M = I.ILU0(A, kind)
    L, U = M.factors()
    LU = (L @ U).tocsr()
    pos = M.pos
    Ap = A.tocoo()
    got = np.asarray(LU[pos[Ap.row], pos[Ap.col]]).ravel()
    assert np.allclose(got, Ap.data, rtol=1e-12, atol=1e-12 * abs(Ap.data).max())
    # and the factors sit on A's pattern only
    assert (L - sp.identity(A.shape[0])).nnz + U.nnz <= A.nnz


def test_full_pattern_gives_the_exact_lu():
    rng = np.random.default_rng(5)
    n = 30
    D = rng.standard_normal((n, n)) + n * np.eye(n)
    M = I.ILU0(sp.csr_matrix(D), "multicolor")
    L, U = M.factors()
    P = np.zeros((n, n))
    P[M.pos, np.arange(n)] = 1.0
    assert np.allclose((L @ U).toarray(), P @ D @ P.T, rtol=1e-12, atol=1e-12 * n)


@pytest.mark.parametrize("kind", ["natural", "multicolor"])
def test_solve_matches_library_triangular_solves(kind):
    A = _matrices()["powerlaw_200"]
    M = I.ILU0(A, kind)
    L, U = M.factors()
    r = np.random.default_rng(6).standard_normal(A.shape[0])
    z = M.solve(r)
    y = spla.spsolve_triangular(L, r[M.order], lower=True, unit_diagonal=True)
    zp = spla.spsolve_triangular(U, y, lower=False)
    assert np.allclose(z[M.order], zp, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name", ["convdiff2d_12", "powerlaw_200", "varcoef3d_6"])
def test_coloring_is_proper_and_equals_sequential_greedy(name):
    A = _matrices()[name]
    c = I.jp_coloring(A)
    G = I.neighbours(A).tocoo()
    assert np.all(c[G.row] != c[G.col])
    assert np.array_equal(c, I.greedy_coloring_by_priority(A))
    assert c.max() + 1 <= I.neighbours(A).sum(axis=1).max() + 1   # greedy bound


def test_priorities_are_distinct():
    p = I.priority(np.arange(1 << 16))
    assert np.unique(p).size == 1 << 16


def test_exact_preconditioner_converges_in_one_outer_step():
    """Tridiagonal A: ILU(0) = A, so A M^{-1} = I; the first sketched cycle
    solves exactly (k = 1) and FGMRES is exact after one step (Section 2.1)."""
    A = _tridiag(200, 7)
    b = np.random.default_rng(8).standard_normal(200)
    M = I.ILU0(A, "natural")
    r = oracle.sfgmres(A, b, m=10, t=2, s=40, zeta=8, tol=1e-12, seed=3, max_outer=5,
                       precond=M)
    assert r.outer_iters == 1 and r.inner_k == [1]
    assert np.linalg.norm(b - A @ r.x) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("kind", ["natural", "multicolor"])
def test_preconditioned_solve_matches_dense_solve(kind):
    A = _matrices()["convdiff2d_12"]
    b = np.random.default_rng(9).uniform(0, 1, A.shape[0])
    M = I.ILU0(A, kind)
    r = oracle.sfgmres(A, b, m=10, t=2, s=40, zeta=8, tol=1e-10, seed=11, max_outer=100,
                       precond=M)
    Ad = A.toarray()
    x = np.linalg.solve(Ad, b)
    assert r.status == 0
    assert np.linalg.norm(b - Ad @ r.x) <= 1.01e-10 * np.linalg.norm(b)
    assert np.linalg.norm(r.x - x) <= 2 * np.linalg.cond(Ad) * 1e-10 * np.linalg.norm(x)
    h = np.array(r.residual_history)
    assert np.all(h[1:] <= h[:-1])
    plain = oracle.sfgmres(A, b, m=10, t=2, s=40, zeta=8, tol=1e-10, seed=11, max_outer=100)
    assert r.outer_iters <= plain.outer_iters


def test_identity_sketch_inner_is_right_preconditioned_gmres():
    """S = I: the inner cycle is GMRES(k) on A M^{-1}, and z = M^{-1} u."""
    A = _matrices()["powerlaw_200"]
    n = A.shape[0]
    M = I.ILU0(A, "multicolor")
    v = np.random.default_rng(12).standard_normal(n)
    v /= np.linalg.norm(v)
    k = 8
    r = oracle.sfgmres(A, v, m=k, t=2, s=n, zeta=1, tol=1e-300, seed=0, max_outer=1,
                       sketch=lambda w: np.array(w, copy=True), cond_threshold=1e300,
                       forced_k=[k], precond=M)
    op = spla.LinearOperator((n, n), matvec=lambda u: A @ M.solve(u))
    u, _ = spla.gmres(op, v, x0=np.zeros(n), restart=k, maxiter=1, rtol=1e-300, atol=0)
    xg = M.solve(u)
    assert np.linalg.norm(r.x - xg) <= 1e-10 * np.linalg.norm(xg)
