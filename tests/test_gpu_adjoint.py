"""Adjoint (A^T lambda = g) and the gradients dL/db = lambda,
dL/dA_ij = -lambda_i x_j, through the HIP library and torch.autograd."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, hist_close

pytestmark = [pytest.mark.gpu, requires_gpu]


def test_adjoint_dense_reference_tiny():
    A = W.convdiff2d(10, 1.0, (10.0, 10.0))
    n = A.n
    rng = np.random.default_rng(1)
    b = rng.uniform(0, 1, n)
    xt = rng.uniform(0, 1, n)
    prm = dict(m=20, t=2, s=60, zeta=8, tol=1e-13, seed=4, max_outer=100)
    rp, ci, va = to_dev(A)
    x, _ = P.solve(rp, ci, va, tvec(b), **prm)
    g = 2 * (x - tvec(xt))
    lam, gv, info = P.solve_adjoint(rp, ci, va, g, x, **prm)
    Ad = A.to_scipy().toarray()
    xd = np.linalg.solve(Ad, b)
    lamd = np.linalg.solve(Ad.T, 2 * (xd - xt))
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    assert np.allclose(lam.cpu().numpy(), lamd, rtol=1e-9, atol=1e-11)
    assert np.allclose(gv.cpu().numpy(), -lamd[rows] * xd[A.col_idx], rtol=1e-8, atol=1e-11)


@pytest.mark.parametrize("precision", ["fp64"])
def test_adjoint_parity_with_oracle(precision):
    A, b, p = W.make_workload(4, 64)
    prm = dict(m=60, t=2, s=240, zeta=8, tol=1e-8, seed=p["seed"], max_outer=50)
    rp, ci, va = to_dev(A)
    x, _ = P.solve(rp, ci, va, tvec(b), **prm)
    g = 2 * (x - tvec(p["x_target"]))
    lam, gv, info = P.solve_adjoint(rp, ci, va, g, x, precision=precision, **prm)
    rpt, cit, vt, perm = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    AT = sp.csr_matrix((vt, cit, rpt), shape=(A.n, A.n))
    gn = g.cpu().numpy()
    ref = oracle.sfgmres(AT, gn, m=60, t=2, s=240, zeta=8, tol=1e-8, seed=p["seed"], max_outer=50)
    assert list(info["inner_k"]) == ref.inner_k
    rf = oracle.sfgmres(AT, gn, m=60, t=2, s=240, zeta=8, tol=1e-8, seed=p["seed"], max_outer=50,
                        forced_k=list(info["inner_k"]))
    hist_close(info["residual_history"], rf.residual_history)
    lam_n = lam.cpu().numpy()
    assert np.linalg.norm(lam_n - rf.x) <= 1e-9 * np.linalg.norm(rf.x)
    grad_ref = oracle.adjoint_gradient(A.row_ptr, A.col_idx, lam_n, x.cpu().numpy())
    assert np.array_equal(gv.cpu().numpy(), grad_ref)


def test_dot_product_identity():
    """<A^{-T} c, d> = <c, A^{-1} d> for the two solves (tol 1e-12)."""
    A = W.convdiff3d(16)
    n = A.n
    rng = np.random.default_rng(3)
    c = rng.standard_normal(n)
    d = rng.standard_normal(n)
    prm = dict(m=60, t=2, s=240, zeta=8, tol=1e-12, seed=9, max_outer=100)
    rp, ci, va = to_dev(A)
    y, _ = P.solve(rp, ci, va, tvec(d), **prm)
    lam, _, _ = P.solve_adjoint(rp, ci, va, tvec(c), None, **prm)
    lhs = float(lam.cpu().numpy() @ d)
    rhs = float(c @ y.cpu().numpy())
    assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("precision,tol,gtol", [("fp64", 1e-12, 1e-5), ("mixed", 1e-12, 1e-5)])
def test_autograd_theta_finite_differences(precision, tol, gtol):
    """C4-style operator A(theta) on a 64 x 64 grid: dL/dtheta through
    SFGMRESSolve vs central differences of the loss (solves at tol 1e-12)."""
    N = 64
    pat, ux, uy, patch = W.theta_convdiff2d_parts(N, 8)
    d = torch.device("cuda:0")
    rp = torch.from_numpy(pat.row_ptr).to(d)
    ci = torch.from_numpy(pat.col_idx).to(d)
    lap, uxt, uyt = (torch.from_numpy(a).to(d) for a in (pat.val, ux, uy))
    pt = torch.from_numpy(patch).to(d)
    rng = np.random.default_rng([4, 2])
    theta0 = torch.from_numpy(rng.standard_normal(64)).to(d)
    b = torch.from_numpy(np.random.default_rng([4, 1]).uniform(0, 1, pat.n)).to(d)
    xt = torch.from_numpy(np.random.default_rng([4, 3]).uniform(0, 1, pat.n)).to(d)
    prm = P.SolveParams(m=60, t=2, s=240, zeta=8, tol=tol, seed=1004, max_outer=200,
                        precision=precision)

    def loss(theta, bb):
        val = W.theta_convdiff2d_values(theta, lap, uxt, uyt, pt)
        x = P.sfgmres_solve(rp, ci, val, bb, prm)
        return ((x - xt) ** 2).sum()

    th = theta0.clone().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    L0 = loss(th, bb)
    L0.backward()
    gth = th.grad.cpu().numpy()
    gb = bb.grad.cpu().numpy()
    h = 1e-4
    for k in [0, 9, 36, 63]:
        e = torch.zeros_like(theta0)
        e[k] = h
        with torch.no_grad():
            fd = (loss(theta0 + e, b) - loss(theta0 - e, b)).item() / (2 * h)
        assert abs(fd - gth[k]) <= gtol * max(abs(fd), 1e-3 * np.abs(gth).max())
    for i in [0, 1000, 4095]:
        e = torch.zeros_like(b)
        e[i] = 1e-3
        with torch.no_grad():
            fd = (loss(theta0, b + e) - loss(theta0, b - e)).item() / 2e-3
        assert abs(fd - gb[i]) <= gtol * max(abs(fd), 1e-3 * np.abs(gb).max())
