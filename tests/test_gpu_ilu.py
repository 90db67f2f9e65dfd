"""The zero-fill ILU right preconditioner on the GPU (Section 4.4, the "-p"
rows of Table 1) against the oracle: the colouring bit for bit, the factor
values, preconditioned solves element by element (FP64), the mixed and
adjoint paths, and the errors of the option."""
import warnings

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from oracle import ilu as OI
import paper_2506_18408_amd as P
import paper_2506_18408_amd._lib as L
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, hist_close, ragged_powerlaw

pytestmark = [pytest.mark.gpu, requires_gpu]

KAPPA_STRICT = 1e7


def _systems():
    return {
        "convdiff2d_24": (W.convdiff2d(24, 1.0, (10.0, 10.0)),
                          np.random.default_rng([1, 1]).uniform(0, 1, 576)),
        "powerlaw_3000": (ragged_powerlaw(3000, 5, Lmax=64, mean=12),
                          np.random.default_rng(6).standard_normal(3000)),
        "varcoef3d_10": (W.convdiff3d_varcoef(10, np.random.default_rng([5, 0])),
                         np.random.default_rng([5, 1]).uniform(-1, 1, 1000)),
    }


@pytest.mark.parametrize("name", ["convdiff2d_24", "powerlaw_3000", "varcoef3d_10"])
def test_ilu_colouring_and_factors_match_the_oracle(name):
    A, _ = _systems()[name]
    lu, color = P.ilu0(*to_dev(A))
    M = OI.ILU0(A.to_scipy(), "multicolor")
    assert np.array_equal(color.cpu().numpy(), M.color)        # integer work: bit for bit
    lu = lu.cpu().numpy()
    scale = np.abs(M.lu).max()
    assert np.allclose(lu, M.lu, rtol=1e-12, atol=1e-14 * scale)


@pytest.mark.parametrize("name", ["convdiff2d_24", "powerlaw_3000", "varcoef3d_10"])
@pytest.mark.parametrize("t", [0, 2])
def test_ilu_preconditioned_solve_matches_the_oracle(name, t):
    A, b = _systems()[name]
    prm = dict(m=20, t=t, s=60, zeta=8, tol=1e-9, seed=1001, max_outer=60)
    x, info = P.solve(*to_dev(A), tvec(b), precond="ilu0", record_true_residual=True, **prm)
    assert info["converged"]
    M = OI.ILU0(A.to_scipy(), "multicolor")
    free = oracle.sfgmres(A.to_scipy(), b, precond=M, **prm)
    # (the replay records the exact condition numbers of S A M^{-1} B_k: a
    # power basis of the well-clustered A M^{-1} degenerates within a few
    # steps, and the incremental estimate can then sit far below the SVD)
    ref = oracle.sfgmres(A.to_scipy(), b, precond=M, forced_k=list(info["inner_k"]),
                         c2_rule="exact", **prm)
    kap = np.maximum(np.asarray(info["cond_at_stop"]), np.asarray(ref.cond_at_stop))
    p = int(np.argmax(kap > KAPPA_STRICT)) if (kap > KAPPA_STRICT).any() else info["outer_iters"]
    # (decisions agree up to the first ill-conditioned cycle, whose y, and
    # so everything after it, is determined only to about u kappa)
    assert list(info["inner_k"][:p + 1]) == free.inner_k[:p + 1]
    hist_close(info["residual_history"][:p + 1], ref.residual_history[:p + 1])
    hist_close(info["true_residual_history"][:p], ref.true_residual_history[:p], atol=1e-13)
    if p == info["outer_iters"]:
        xs = x.cpu().numpy()
        assert np.linalg.norm(xs - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    else:
        h = np.asarray(info["residual_history"])
        r = np.asarray(ref.residual_history)
        assert np.all(np.abs(np.log(h[1:] / r[1:])) <= np.log(10.0))
        assert np.all(h[1:] <= h[:-1])
    plain = oracle.sfgmres(A.to_scipy(), b, **prm)
    assert info["outer_iters"] <= plain.outer_iters


@pytest.mark.parametrize("name", ["convdiff2d_24", "powerlaw_3000", "varcoef3d_10"])
def test_ilu_power_basis_forced_short_cycles_strict(name):
    """t = 0 with cycles forced to k = 3 (a well-conditioned power basis of
    A M^{-1}): strict parity over the whole solve."""
    A, b = _systems()[name]
    prm = dict(m=20, t=0, s=60, zeta=8, tol=1e-9, seed=1001, max_outer=200)
    fk = [3] * prm["max_outer"]
    x, info = P.solve(*to_dev(A), tvec(b), precond="ilu0", forced_k=fk, **prm)
    M = OI.ILU0(A.to_scipy(), "multicolor")
    ref = oracle.sfgmres(A.to_scipy(), b, precond=M, forced_k=fk, c2_rule="exact", **prm)
    assert np.all(np.asarray(ref.cond_at_stop) <= KAPPA_STRICT)
    assert info["outer_iters"] == ref.outer_iters
    hist_close(info["residual_history"], ref.residual_history)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_ilu_mixed_precision_and_adjoint():
    A, b = _systems()["varcoef3d_10"]
    prm = dict(m=20, t=2, s=60, zeta=8, tol=1e-8, seed=1001, max_outer=60)
    rp, ci, va = to_dev(A)
    x64, i64 = P.solve(rp, ci, va, tvec(b), precond="ilu0", **prm)
    xm, im = P.solve(rp, ci, va, tvec(b), precond="ilu0", precision="mixed", **prm)
    assert im["converged"] and im["true_rel_residual"] <= 1e-8 * (1 + 1e-6)
    err = (torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)).item()
    assert err <= 1e-6
    g = tvec(np.random.default_rng(3).standard_normal(A.n))
    lam, gv, ia = P.solve_adjoint(rp, ci, va, g, x64, precond="ilu0", **prm)
    assert ia["converged"]
    rpT, ciT, vT, perm = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    AT = sp.csr_matrix((vT, ciT, rpT), shape=(A.n, A.n))
    MT = OI.ILU0(AT, "multicolor")
    ref = oracle.sfgmres(AT, g.cpu().numpy(), precond=MT, forced_k=list(ia["inner_k"]), **prm)
    hist_close(ia["residual_history"], ref.residual_history)
    lr = lam.cpu().numpy()
    assert np.linalg.norm(lr - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    want = oracle.adjoint_gradient(A.row_ptr, A.col_idx, lr, x64.cpu().numpy())
    assert np.array_equal(gv.cpu().numpy(), want)


def test_ilu_option_errors():
    A, b = _systems()["convdiff2d_24"]
    prm = dict(m=20, t=2, s=60, zeta=8, tol=1e-8, seed=1001, max_outer=5)
    with pytest.raises(P.SFGMRESError) as e:
        P.solve(*to_dev(A), tvec(b), precond="ilu0", outer="restarted", **prm)
    assert e.value.code == L.ERR_INVALID
    # unsorted columns in one row
    ci = A.col_idx.copy()
    r = 100
    ci[A.row_ptr[r]:A.row_ptr[r + 1]] = ci[A.row_ptr[r]:A.row_ptr[r + 1]][::-1]
    vals = A.val.copy()
    vals[A.row_ptr[r]:A.row_ptr[r + 1]] = vals[A.row_ptr[r]:A.row_ptr[r + 1]][::-1]
    B = W.CSR(A.n, A.row_ptr, ci, vals)
    with pytest.raises(P.SFGMRESError) as e:
        P.solve(*to_dev(B), tvec(b), precond="ilu0", **prm)
    assert e.value.code == L.ERR_INVALID
    # a row without its diagonal entry
    keep = np.ones(A.nnz, dtype=bool)
    row = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    keep[(row == 7) & (A.col_idx == 7)] = False
    rp = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row[keep], minlength=A.n), out=rp[1:])
    C = W.CSR(A.n, rp.astype(np.int32), A.col_idx[keep], A.val[keep])
    with pytest.raises(P.SFGMRESError) as e:
        P.solve(*to_dev(C), tvec(b), precond="ilu0", **prm)
    assert e.value.code == L.ERR_INVALID
    # the same matrices without the preconditioner still solve
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        P.solve(*to_dev(B), tvec(b), **prm)


@pytest.mark.parametrize("n", [1, 777])
def test_ilu_of_a_diagonal_matrix_is_the_matrix(n):
    """No off-diagonal entries: one colour, empty L and U, the factor is A
    itself, and M^{-1} = A^{-1} solves in one inner step."""
    d = np.random.default_rng([40, n]).uniform(1.0, 3.0, n)
    A = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    lu, color = P.ilu0(*to_dev(A))
    assert np.array_equal(color.cpu().numpy(), np.zeros(n, np.int32))
    assert np.array_equal(lu.cpu().numpy(), d)
    if n < 60:
        return
    b = np.random.default_rng([41, n]).uniform(-1.0, 1.0, n)
    x, info = P.solve(*to_dev(A), tvec(b), precond="ilu0", m=20, t=2, s=60, zeta=8, tol=1e-12,
                      seed=5, max_outer=5)
    assert info["converged"] and info["outer_iters"] == 1 and list(info["inner_k"]) == [1]
    assert np.linalg.norm(x.cpu().numpy() - b / d) <= 1e-14 * np.linalg.norm(b / d)


def test_ilu_of_a_block_diagonal_matrix_is_exact():
    """Independent 2 x 2 blocks: two colours, and ILU(0) without fill is
    the exact LU, so the preconditioned solve takes one inner step."""
    nb = 400
    rng = np.random.default_rng(42)
    blocks = [np.array([[rng.uniform(3, 4), rng.uniform(-1, 1)],
                        [rng.uniform(-1, 1), rng.uniform(3, 4)]]) for _ in range(nb)]
    S = sp.csr_matrix(sp.block_diag(blocks))
    S.sort_indices()
    A = W.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
              S.data.astype(np.float64))
    lu, color = P.ilu0(*to_dev(A))
    M = OI.ILU0(A.to_scipy(), "multicolor")
    assert np.array_equal(color.cpu().numpy(), M.color)
    assert set(np.unique(M.color)) == {0, 1}
    assert np.allclose(lu.cpu().numpy(), M.lu, rtol=1e-14, atol=0.0)
    b = rng.uniform(-1.0, 1.0, A.n)
    x, info = P.solve(*to_dev(A), tvec(b), precond="ilu0", m=20, t=2, s=60, zeta=8, tol=1e-12,
                      seed=5, max_outer=5)
    assert info["converged"] and info["outer_iters"] == 1 and list(info["inner_k"]) == [1]
    xe = np.linalg.solve(S.toarray(), b)
    assert np.linalg.norm(x.cpu().numpy() - xe) <= 1e-13 * np.linalg.norm(xe)


def test_ilu_zero_pivot_is_a_breakdown():
    """A zero pivot, met as a divisor or left on U's diagonal, is reported as
    a breakdown by the factorisation and by a preconditioned solve (the
    oracle's factorisation stops on the same pivot)."""
    rng = np.random.default_rng(43)
    good = [np.array([[4.0, rng.uniform(-1, 1)], [rng.uniform(-1, 1), 4.0]]) for _ in range(50)]
    S = sp.csr_matrix(sp.block_diag(good[:20] + [np.ones((2, 2))] + good[20:]))
    S.sort_indices()
    n = 100
    d = np.r_[np.full(40, 2.0), 0.0, np.full(59, 2.0)]
    cases = {
        # rows (40, 41) = [[1, 1], [1, 1]]: u = 1 - 1 * 1 = 0 on the second one
        "eliminated_to_zero": W.CSR(S.shape[0], S.indptr.astype(np.int32),
                                    S.indices.astype(np.int32), S.data.astype(np.float64)),
        # an explicit zero on the diagonal of a row nothing depends on
        "zero_diagonal": W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                               d),
    }
    for name, A in cases.items():
        with pytest.raises(ZeroDivisionError):
            OI.ILU0(A.to_scipy(), "multicolor")
        with pytest.raises(P.SFGMRESError) as e:
            P.ilu0(*to_dev(A))
        assert e.value.code == L.ERR_BREAKDOWN, name
        b = np.ones(A.n)
        with pytest.raises(P.SFGMRESError) as e:
            P.solve(*to_dev(A), tvec(b), precond="ilu0", m=20, t=2, s=60, zeta=8, tol=1e-8,
                    seed=5, max_outer=5)
        assert e.value.code == L.ERR_BREAKDOWN, name
