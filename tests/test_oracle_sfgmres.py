"""Pins of the oracle's FGMRES / sGMRES (oracle/sfgmres.py) against the
mathematics: dense solves, textbook special cases, the paper's invariants."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads as W

IDENT = staticmethod(lambda w: np.array(w, copy=True))


def _ident(w):
    return np.array(w, copy=True)


def _small_systems():
    A1 = W.convdiff2d(16, 1.0, (10.0, 10.0)).to_scipy()
    b1 = np.random.default_rng(0).uniform(0, 1, A1.shape[0])
    A2 = W.powerlaw_random(300, np.random.default_rng(1), Lmin=4, Lmax=40, mean=8).to_scipy()
    b2 = np.random.default_rng(2).standard_normal(300)
    A3 = W.convdiff3d(7, 1.0, (50.0, 50.0, 50.0)).to_scipy()
    b3 = np.random.default_rng(3).uniform(-1, 1, A3.shape[0])
    return [(A1, b1), (A2, b2), (A3, b3)]


@pytest.mark.parametrize("idx", [0, 1, 2])
@pytest.mark.parametrize("t", [0, 2])
def test_matches_dense_solve(idx, t):
    A, b = _small_systems()[idx]
    n = A.shape[0]
    r = oracle.sfgmres(A, b, m=10, t=t, s=40, zeta=8, tol=1e-10, seed=11, max_outer=200)
    assert r.status == oracle.sfgmres.__globals__["STATUS_OK"]
    Ad = A.toarray()
    x = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(r.x - x) <= 2 * kappa * 1e-10 * np.linalg.norm(x)
    assert np.linalg.norm(b - Ad @ r.x) <= 1.01e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("t", [0, 1, 2, 7])
def test_identity_sketch_inner_is_gmres(t):
    """S = I: sGMRES minimises the true residual over K_k(A, v), i.e. GMRES(k),
    whatever the truncation t (the basis spans the same Krylov space)."""
    A = W.convdiff2d(12).to_scipy()
    n = A.shape[0]
    v = np.random.default_rng(4).standard_normal(n)
    v /= np.linalg.norm(v)
    k = 7
    z, info = oracle.sgmres_cycle(A, v, _ident, m=k, t=t, tol_abs=0.0, factor=1.0,
                                  cond_threshold=1e300, forced_k=k)
    zs, _ = spla.gmres(A, v, x0=np.zeros(n), restart=k, maxiter=1, rtol=1e-300, atol=0)
    assert np.linalg.norm(z - zs) <= 1e-12 * np.linalg.norm(zs)


def test_inner_dimension_one_is_full_gmres():
    """m = 1 makes z_j a multiple of v_j, so FGMRES is unrestarted GMRES."""
    A, b = _small_systems()[0]
    r = oracle.sfgmres(A, b, m=1, t=0, s=40, zeta=8, tol=1e-9, seed=3, max_outer=300)
    hist = []
    spla.gmres(A, b, x0=np.zeros_like(b), restart=400, maxiter=1, rtol=1e-9,
               callback=lambda pr: hist.append(pr), callback_type="pr_norm")
    J = min(len(hist), r.outer_iters)
    ours = np.array(r.residual_history[1:J + 1])
    ref = np.array(hist[:J])
    assert J > 20
    assert np.all(np.abs(ours - ref) <= 1e-8 * ref + 1e-13)


def test_exact_preconditioner_converges_in_one_step():
    """An exact inner solve makes the first FGMRES iterate exact (Section 2.1)."""
    A = W.powerlaw_random(60, np.random.default_rng(5), Lmin=4, Lmax=12, mean=6).to_scipy()
    b = np.random.default_rng(6).standard_normal(60)
    r = oracle.sfgmres(A, b, m=60, t=60, s=60, zeta=1, tol=1e-12, seed=0, max_outer=5,
                       sketch=_ident, cond_threshold=1e300, forced_k=[60] * 5)
    assert r.outer_iters == 1
    assert r.residual_history[1] < 1e-13


@pytest.fixture(scope="module")
def c1_run():
    A, b, p = W.make_workload(1)
    As = A.to_scipy()
    r = oracle.sfgmres(As, b, m=p["m"], t=p["t"], s=p["s"], zeta=p["zeta"], tol=p["tol"],
                       seed=p["seed"], max_outer=p["max_outer"], keep_basis=True)
    return As, b, r


def test_invariants_monotone_and_ffom(c1_run):
    A, b, r = c1_run
    h = np.array(r.residual_history)
    assert np.all(h[1:] <= h[:-1])                       # non-increasing (Sections 1, 3)
    tr = np.array(r.true_residual_history)
    assert np.all(tr[1:] <= tr[:-1] * (1 + 1e-6) + 1e-13)
    nb = np.linalg.norm(b)
    for j in range(r.outer_iters):                       # ||r_j|| <= ||r~_j||
        assert h[j + 1] * nb <= r.ffom_residual[j] * (1 + 1e-12)


def test_bound_eq_2_2(c1_run):
    A, b, r = c1_run
    nb = np.linalg.norm(b)
    for j in range(r.outer_iters):
        rho = r.residual_history[j + 1] * nb
        assert rho <= r.bound[j] * (1 + 1e-8) + 1e-14 * nb


def test_ffom_closed_form_against_explicit_residual(c1_run):
    """eq. (2.1): ||b - A x~_j|| = h_{j+1,j} |e_j^T H_j^{-1} beta e1|."""
    A, b, r = c1_run
    beta = r.residual_history[0] * np.linalg.norm(b)
    checked = 0
    for j in range(1, r.outer_iters + 1):
        Hj = r.H[:j, :j]
        e1 = np.zeros(j)
        e1[0] = beta
        yF = np.linalg.solve(Hj, e1)
        xF = r.Z[:, :j] @ yF
        expl = np.linalg.norm(b - A @ xF)
        if expl > 1e-6 * beta:
            assert abs(expl - r.ffom_residual[j - 1]) <= 1e-7 * expl
            checked += 1
    assert checked >= 5


def test_arnoldi_like_relation(c1_run):
    """A Z_J = V_{J+1} H_J (Section 2) and V orthonormal."""
    A, b, r = c1_run
    J = r.outer_iters
    AZ = A @ r.Z
    VH = r.V[:, :J + 1] @ r.H
    normA = spla.norm(A, 2) if False else abs(A).sum(axis=1).max()
    assert np.abs(AZ - VH).max() <= 1e-12 * normA * np.abs(r.Z).max() * math.sqrt(A.shape[0])
    G = r.V[:, :J + 1].T @ r.V[:, :J + 1]
    assert np.abs(G - np.eye(J + 1)).max() < 1e-6   # MGS: loss ~ u cond(A Z)


def test_fig1_analogue_fgmres_converges_where_restarted_gmres_stagnates():
    """Section 2.1, Fig. 1 setting: A = randn(1000) + 30 I, inner = 100 GMRES steps."""
    rng = np.random.default_rng(7)
    n = 1000
    A = rng.standard_normal((n, n)) + 30 * np.eye(n)
    b = rng.standard_normal(n)
    r = oracle.sfgmres(A, b, m=100, t=100, s=n, zeta=1, tol=1e-8, seed=0, max_outer=40,
                       sketch=_ident, cond_threshold=1e300, forced_k=[100] * 40,
                       record_true_residual=False)
    assert r.status == 0 and r.outer_iters <= 30
    x, _ = spla.gmres(A, b, restart=100, maxiter=r.outer_iters, rtol=1e-12)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) > 1e-2


def test_fig2_analogue_superlinear():
    """Section 2.3, Fig. 2 setting: diag(1..1000), inner GMRES(5)."""
    rng = np.random.default_rng(8)
    D = sp.diags(np.arange(1, 1001.0)).tocsr()
    b = rng.standard_normal(1000)
    r = oracle.sfgmres(D, b, m=5, t=5, s=1000, zeta=1, tol=1e-10, seed=0, max_outer=80,
                       sketch=_ident, cond_threshold=1e300, forced_k=[5] * 80,
                       record_true_residual=False)
    h = np.array(r.residual_history)
    J = r.outer_iters
    early = (h[10] / h[1]) ** (1 / 9)
    late = (h[J] / h[J - 10]) ** (1 / 10)
    assert late < 0.8 * early
    x, _ = spla.gmres(D, b, restart=5, maxiter=J, rtol=1e-14)
    assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) > 1e3 * h[J]


def test_forced_replay_reproduces_run(c1_run):
    A, b, r = c1_run
    A1, b1, p = W.make_workload(1)
    r2 = oracle.sfgmres(A, b, m=p["m"], t=p["t"], s=p["s"], zeta=p["zeta"], tol=p["tol"],
                        seed=p["seed"], max_outer=p["max_outer"], forced_k=r.inner_k)
    assert r2.residual_history == r.residual_history
    assert np.array_equal(r2.x, r.x)


def test_tiny_cond_threshold_forces_k1_and_stays_monotone():
    A, b = _small_systems()[0]
    r = oracle.sfgmres(A, b, m=10, t=2, s=40, zeta=8, tol=1e-8, seed=2, max_outer=300,
                       cond_threshold=1.0 + 1e-12)
    assert set(r.inner_k) == {1}
    assert set(r.stop_reason) <= {"C2", "C3"}
    h = np.array(r.residual_history)
    assert np.all(h[1:] <= h[:-1])


def test_power_basis_c2_engages_and_ice_close_to_exact():
    """t = 0 gives a power basis whose sketch condition grows until C2 stops it."""
    A, b, p = W.make_workload(1)
    As = A.to_scipy()
    kw = dict(m=30, t=0, s=60, zeta=8, tol=1e-8, seed=p["seed"], max_outer=60, record_true_residual=False)
    r_ice = oracle.sfgmres(As, b, cond_threshold=1e8, **kw)
    r_ex = oracle.sfgmres(As, b, cond_threshold=1e8, c2_rule="exact", **kw)
    assert "C2" in r_ice.stop_reason
    assert abs(r_ice.inner_k[0] - r_ex.inner_k[0]) <= 2
    assert r_ice.status == 0 and r_ex.status == 0


def test_edge_cases():
    A, b = _small_systems()[0]
    kw = dict(m=10, t=2, s=40, zeta=8, tol=1e-8, seed=2)
    r = oracle.sfgmres(A, np.zeros_like(b), **kw)
    assert r.outer_iters == 0 and not r.x.any()
    x = np.linalg.solve(A.toarray(), b)
    r = oracle.sfgmres(A, b, x0=x, **kw)
    assert r.outer_iters == 0 and np.array_equal(r.x, x)
    r = oracle.sfgmres(A, b, max_outer=1, **kw)
    assert r.status == 1 and r.outer_iters == 1
    assert np.linalg.norm(b - A @ r.x) / np.linalg.norm(b) == pytest.approx(r.residual_history[1], rel=1e-8)
    with pytest.raises(ValueError):
        oracle.sfgmres(A, b, m=40, t=2, s=40, zeta=8, tol=1e-8, seed=1)


def test_transpose_brute_force():
    A = W.powerlaw_random(50, np.random.default_rng(9), Lmin=4, Lmax=20, mean=8)
    rp, ci, v, perm = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    ent = sorted((int(A.col_idx[p]), i, p) for i in range(A.n) for p in range(A.row_ptr[i], A.row_ptr[i + 1]))
    for q, (col, row, p) in enumerate(ent):
        assert ci[q] == row and perm[q] == p and v[q] == A.val[p]
    assert list(rp) == list(np.searchsorted([e[0] for e in ent], np.arange(A.n + 1)))


def test_adjoint_against_dense_gradient():
    """L = ||x - xt||^2 with A x = b: dL/db = A^{-T} g, dL/dA = -lam x^T."""
    Am = W.convdiff2d(10, 1.0, (10.0, 10.0))
    A = Am.to_scipy()
    n = A.shape[0]
    rng = np.random.default_rng(10)
    b = rng.uniform(0, 1, n)
    xt = rng.uniform(0, 1, n)
    kw = dict(m=20, t=2, s=60, zeta=8, tol=1e-13, seed=4, max_outer=100)
    x = oracle.sfgmres(A, b, **kw).x
    g = 2 * (x - xt)
    rp, ci, vT, perm = oracle.transpose_csr(Am.row_ptr, Am.col_idx, Am.val, n)
    AT = sp.csr_matrix((vT, ci, rp), shape=(n, n))
    lam = oracle.sfgmres(AT, g, **kw).x
    grad = oracle.adjoint_gradient(Am.row_ptr, Am.col_idx, lam, x)
    Ad = A.toarray()
    xd = np.linalg.solve(Ad, b)
    lamd = np.linalg.solve(Ad.T, 2 * (xd - xt))
    G = -np.outer(lamd, xd)
    rows = np.repeat(np.arange(n), np.diff(Am.row_ptr))
    assert np.allclose(lam, lamd, rtol=1e-9, atol=1e-11)
    assert np.allclose(grad, G[rows, Am.col_idx], rtol=1e-8, atol=1e-11)
    # central finite differences on a few values
    for p in [0, 7, 100, len(Am.val) - 1]:
        h = 1e-6
        Ap = Ad.copy()
        Ap[rows[p], Am.col_idx[p]] += h
        Lp = np.sum((np.linalg.solve(Ap, b) - xt) ** 2)
        Ap[rows[p], Am.col_idx[p]] -= 2 * h
        Lm = np.sum((np.linalg.solve(Ap, b) - xt) ** 2)
        assert abs((Lp - Lm) / (2 * h) - grad[p]) <= 1e-5 * max(1.0, abs(grad[p]))


def test_recursive_bound_eq_2_3(c1_run):
    """Section 2.3: while every delta_i (i <= j) is below one, the FGMRES
    residual contracts at least by delta_j per step, with delta_j built
    from the inner residuals alone."""
    A, b, r = c1_run
    h = np.array(r.residual_history)
    d = np.array(r.delta)
    rh = np.array(r.inner_true_residual)
    assert d[0] == pytest.approx(rh[0], rel=1e-15)      # delta_1 = ||r^_1|| (delta_0 = 0)
    valid = np.cumprod(np.nan_to_num(d, nan=2.0) < 1.0).astype(bool)
    assert valid.sum() >= 3
    for j in np.nonzero(valid)[0]:
        assert h[j + 1] <= d[j] * h[j] * (1 + 1e-10)


def test_recursive_bound_turns_nan_once_delta_reaches_one():
    """m = 1 (FGMRES = GMRES): the inner residual is ||v - c A v|| with the
    best scalar c, close to one, so delta exceeds one after a few steps and
    the recursion has no real value from then on."""
    A, b = _small_systems()[0]
    r = oracle.sfgmres(A, b, m=1, t=0, s=40, zeta=8, tol=1e-9, seed=3, max_outer=20)
    d = np.array(r.delta)
    assert np.isnan(d).any()
    first = int(np.argmax(np.isnan(d)))
    assert first >= 1 and d[first - 1] >= 1.0
    assert np.isnan(d[first:]).all()
