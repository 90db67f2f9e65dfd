"""A seeded sweep of small random systems and option combinations.  Each
case is solved on the GPU with its inner dimensions forced, and the oracle
replays the same dimensions: residual histories within 1e-9 relative and
the solution within 1e-9, step for step.  The cases cover:
- sizes off the 64-row tile multiples;
- ragged rows, banded matrices the inner SpMV reads by diagonal, and a few
  long rows;
- every Arnoldi window from 0 to min(m, 8);
- both matrix storages and both sketch sources;
- ILU(0) or no preconditioner."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import ilu as OI
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, hist_close

pytestmark = [pytest.mark.gpu, requires_gpu]

NCASES = 48


def _random_system(rng):
    """A strictly diagonally dominant matrix (so ILU(0) has nonzero pivots
    and the forced cycles stay well conditioned) of one of three shapes."""
    n = int(rng.choice([64, 65, 127, 300, 1000, 4097, 9999]))
    kind = int(rng.integers(3))
    if kind == 0:    # banded: a few diagonals, read by diagonal under "auto"
        nd = int(rng.integers(2, 7))
        offs = sorted(set(int(o) for o in rng.integers(-n // 4 - 1, n // 4 + 2, size=nd)) - {0})
        offs = offs or [1]
        M = sp.diags([rng.uniform(-1, 1, n - abs(o)) for o in offs], offs, shape=(n, n))
    elif kind == 1:  # random pattern, 0..20 off-diagonal entries per row
        lens = rng.integers(0, 21, size=n)
        rows = np.repeat(np.arange(n), lens)
        cols = rng.integers(0, n, size=rows.size)
        M = sp.coo_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(n, n))
    else:            # mostly short rows, a few of up to 200 entries
        lens = rng.integers(1, 8, size=n)
        lens[rng.integers(0, n, size=max(1, n // 200))] = min(200, n)
        rows = np.repeat(np.arange(n), lens)
        cols = rng.integers(0, n, size=rows.size)
        M = sp.coo_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(n, n))
    M = sp.csr_matrix(M)
    M.setdiag(0.0)
    M.eliminate_zeros()
    rowsum = np.asarray(abs(M).sum(axis=1)).ravel()
    d = (rowsum + 1.0) * rng.uniform(1.5, 3.0, n) * rng.choice([-1.0, 1.0], n)
    S = sp.csr_matrix(M + sp.diags(d))
    S.sort_indices()
    A = W.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32),
              S.data.astype(np.float64))
    b = rng.uniform(-1.0, 1.0, n)
    return A, b, kind


def _random_options(rng):
    m = int(rng.integers(4, 25))
    t = int(rng.integers(0, min(m, 8) + 1))
    s = int(rng.integers(m + 1, min(1024, 3 * m + 40) + 1))
    zeta = int(rng.integers(1, min(s, 16) + 1))
    precond = "ilu0" if rng.random() < 0.4 else "none"
    # (the power basis of a well-clustered A M^{-1} degenerates within a few
    # steps: short cycles there)
    kmax = 3 if (t == 0 and precond == "ilu0") else min(m, 6)
    max_outer = int(rng.integers(1, 7))
    forced = [int(k) for k in rng.integers(1, kmax + 1, size=max_outer)]
    src = "gen" if (zeta <= 8 and rng.random() < 0.5) else "table"
    fmt = "csr" if rng.random() < 0.3 else "auto"
    return dict(m=m, t=t, s=s, zeta=zeta, tol=1e-14, seed=int(rng.integers(2**62)),
                max_outer=max_outer), forced, precond, src, fmt


@pytest.mark.filterwarnings("ignore:sfgmres")   # (max_outer reached: the forced cases stop there)
@pytest.mark.parametrize("case", range(NCASES))
def test_random_case_matches_the_oracle(case):
    rng = np.random.default_rng([2506, 18408, case])
    A, b, kind = _random_system(rng)
    prm, forced, precond, src, fmt = _random_options(rng)
    x, info = P.solve(*to_dev(A), tvec(b), forced_k=forced, precond=precond, sketch_source=src,
                      matrix_format=fmt, **prm)
    M = OI.ILU0(A.to_scipy(), "multicolor") if precond == "ilu0" else None
    ref = oracle.sfgmres(A.to_scipy(), b, forced_k=forced, precond=M, **prm)
    what = (case, A.n, kind, prm, forced, precond, src, fmt)
    assert info["outer_iters"] == ref.outer_iters, what
    assert list(info["inner_k"]) == list(ref.inner_k), what
    assert list(info["inner_k"]) == forced[:info["outer_iters"]], what
    hist_close(info["residual_history"], ref.residual_history)
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - ref.x) <= 1e-9 * np.linalg.norm(ref.x), what


@pytest.mark.filterwarnings("ignore:sfgmres")
@pytest.mark.parametrize("case", range(0, NCASES, 2))
def test_random_case_adjoint_matches_the_oracle(case):
    """The adjoint solve A^T lam = g of the same cases (the transpose built
    on the device, its own ILU(0) when preconditioned), against the oracle
    on A^T with the same forced dimensions; dL/dA from the GPU's lam and x
    equals the product formula exactly."""
    rng = np.random.default_rng([2506, 18408, case])
    A, b, kind = _random_system(rng)
    prm, forced, precond, src, fmt = _random_options(rng)
    g = np.random.default_rng([2506, 18409, case]).uniform(-1.0, 1.0, A.n)
    xv = np.random.default_rng([2506, 18410, case]).uniform(-1.0, 1.0, A.n)
    lam, gv, info = P.solve_adjoint(*to_dev(A), tvec(g), tvec(xv), forced_k=forced,
                                    precond=precond, sketch_source=src, matrix_format=fmt, **prm)
    rpT, ciT, vT, _ = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    AT = sp.csr_matrix((vT, ciT, rpT), shape=(A.n, A.n))
    M = OI.ILU0(AT, "multicolor") if precond == "ilu0" else None
    ref = oracle.sfgmres(AT, g, forced_k=forced, precond=M, **prm)
    what = (case, A.n, kind, prm, forced, precond, src, fmt)
    assert list(info["inner_k"]) == list(ref.inner_k), what
    hist_close(info["residual_history"], ref.residual_history)
    lr = lam.cpu().numpy()
    assert np.linalg.norm(lr - ref.x) <= 1e-9 * np.linalg.norm(ref.x), what
    want = oracle.adjoint_gradient(A.row_ptr, A.col_idx, lr, xv)
    assert np.array_equal(gv.cpu().numpy(), want), what


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("precond", ["none", "ilu0"])
@pytest.mark.parametrize("fmt", ["auto", "csr"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_smallest_systems_solve(n, fmt, precond, precision):
    """Systems of one to three unknowns: one tile with most lanes idle, a
    matrix by diagonal of one to three diagonals, a one- or two-colour ILU;
    the Krylov space is exhausted within the first cycle (an exact breakdown
    of the Arnoldi recurrence at the latest after n steps)."""
    rng = np.random.default_rng([77, n])
    D = np.diag(rng.uniform(2.0, 3.0, n)) + (np.triu(rng.uniform(-0.5, 0.5, (n, n)), 1)
                                             + np.tril(rng.uniform(-0.5, 0.5, (n, n)), -1))
    S = sp.csr_matrix(D)
    A = W.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    b = rng.uniform(-1.0, 1.0, n)
    m = n + 1
    x, info = P.solve(*to_dev(A), tvec(b), m=m, t=1, s=m + 2, zeta=1, tol=1e-12, seed=3,
                      max_outer=10, precond=precond, matrix_format=fmt, precision=precision)
    assert info["converged"], info
    xe = np.linalg.solve(D, b)
    assert np.linalg.norm(x.cpu().numpy() - xe) <= 1e-10 * np.linalg.norm(xe)
