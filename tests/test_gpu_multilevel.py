"""Two-level FGMRES on the GPU (Section 5's multi-level FGMRES): each outer
step is preconditioned by a lower-level FGMRES solve of at most mid_outer
steps, against the oracle's two-level solve."""
import numpy as np
import pytest

import oracle
import oracle.ilu as OI
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, hist_close

pytestmark = [pytest.mark.gpu, requires_gpu]


def _sys():
    A = W.convdiff2d(20, 1.0, (10.0, 10.0))
    b = np.random.default_rng(4).uniform(0, 1, A.n)
    return A, b


@pytest.mark.parametrize("mid", [1, 2, 5])
def test_two_level_matches_the_oracle(mid):
    A, b = _sys()
    prm = dict(m=12, t=2, s=48, zeta=8, tol=1e-9, seed=21, max_outer=60)
    x, info = P.solve(*to_dev(A), tvec(b), mid_outer=mid, record_true_residual=True, **prm)
    ref = oracle.sfgmres(A.to_scipy(), b, mid_outer=mid, **prm)
    assert info["converged"] and ref.status == 0
    assert list(info["inner_k"]) == ref.inner_k
    assert set(info["stop_reason"]) == {"mid"}
    hist_close(info["residual_history"], ref.residual_history)
    hist_close(info["true_residual_history"], ref.true_residual_history, atol=1e-13)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    nb = np.linalg.norm(b)
    h = np.asarray(info["residual_history"]) * nb
    assert np.all(h[1:] <= np.asarray(info["bound"]) * (1 + 1e-8) + 1e-14 * nb)
    if mid == 1:
        # one lower-level step is one sGMRES cycle, rescaled: the one-level solve
        x1, i1 = P.solve(*to_dev(A), tvec(b), **prm)
        hist_close(info["residual_history"], i1["residual_history"])


def test_two_level_mixed_precision_reaches_tol():
    A, b = _sys()
    prm = dict(m=12, t=2, s=48, zeta=8, tol=1e-8, seed=21, max_outer=60)
    x, info = P.solve(*to_dev(A), tvec(b), mid_outer=4, precision="mixed", **prm)
    assert info["converged"] and info["true_rel_residual"] <= 1e-8 * (1 + 1e-6)
    assert info["total_inner"] >= sum(info["inner_k"])


def test_two_level_with_ilu_matches_the_oracle():
    """ILU(0) inside the lower level's sGMRES cycles: the top level factors A
    once and every lower-level solve applies those factors."""
    A, b = _sys()
    prm = dict(m=12, t=2, s=48, zeta=8, tol=1e-9, seed=21, max_outer=60)
    x, info = P.solve(*to_dev(A), tvec(b), mid_outer=3, precond="ilu0", **prm)
    M = OI.ILU0(A.to_scipy(), "multicolor")
    ref = oracle.sfgmres(A.to_scipy(), b, mid_outer=3, precond=M, **prm)
    assert info["converged"] and ref.status == 0
    assert list(info["inner_k"]) == ref.inner_k
    hist_close(info["residual_history"], ref.residual_history)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_two_level_with_ilu_mixed_precision_reaches_tol():
    """The mixed-precision lower levels share the top level's factors (their
    FP32 copy for the cycles' FP32 vectors, the same copy for the FP64
    inner solutions)."""
    A, b = _sys()
    prm = dict(m=12, t=2, s=48, zeta=8, tol=1e-8, seed=21, max_outer=60)
    rp, ci, va = to_dev(A)
    x64, i64 = P.solve(rp, ci, va, tvec(b), mid_outer=3, precond="ilu0", **prm)
    xm, im = P.solve(rp, ci, va, tvec(b), mid_outer=3, precond="ilu0", precision="mixed", **prm)
    assert i64["converged"] and im["converged"]
    assert im["true_rel_residual"] <= 1e-8 * (1 + 1e-6)
    # both within their residuals of the solution: ||x_m - x_64|| / ||x|| is at
    # most cond(A) (r_m + r_64) / (1 - cond(A) r_64) in relative terms
    kappa = np.linalg.cond(A.to_scipy().toarray())
    rm, r64 = im["true_rel_residual"], i64["true_rel_residual"]
    xs, xr = xm.cpu().numpy(), x64.cpu().numpy()
    bound = kappa * (rm + r64) / (1.0 - kappa * r64)
    assert np.linalg.norm(xs - xr) <= bound * np.linalg.norm(xr)
