"""The library's limits (SFGMRES_MAX_S = 1024 sketch rows, SFGMRES_MAX_ZETA =
16 nonzeros per sketch column, SFGMRES_MAX_T = 8, SFGMRES_MAX_M = 512):
strict parity where the sketched least-squares problem stays well
conditioned, validity for a full 512-column cycle."""
import warnings

import numpy as np
import pytest

import oracle
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, hist_close

pytestmark = [pytest.mark.gpu, requires_gpu]


def _system():
    A = W.convdiff3d(16)  # n = 4096 >= s
    b = np.random.default_rng([16, 1]).uniform(-1, 1, A.n)
    return A, b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_max_sketch_zeta_window_forced_replay(precision):
    """s = 1024, zeta = 16 (four packed groups per sketch column), t = 8 (the
    wide-window kernels), k = 24 per cycle: FP64 matches the oracle to 1e-9;
    mixed precision reaches the same residuals to FP32 accuracy."""
    A, b = _system()
    prm = dict(m=64, t=8, s=1024, zeta=16, tol=1e-300, seed=77, max_outer=4)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        x, info = P.solve(*to_dev(A), tvec(b), forced_k=[24] * 4, precision=precision, **prm)
    ref = oracle.sfgmres(A.to_scipy(), b, m=64, t=8, s=1024, zeta=16, tol=1e-300, seed=77,
                         max_outer=4, forced_k=[24] * 4, record_true_residual=False)
    assert max(ref.cond_at_stop) <= 1e7
    if precision == "fp64":
        hist_close(info["residual_history"], ref.residual_history)
        assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    else:
        # (the FP32 basis perturbs each direction z_j by ~ u32 sqrt(k); the change
        # in a minimised residual is that times the previous residual)
        hist_close(info["residual_history"], ref.residual_history, rtol=1e-3, atol=1e-12)


def test_full_512_column_cycle():
    """m = 512 = SFGMRES_MAX_M with a forced full cycle (64 decision panels):
    the truncated basis is far too ill conditioned for rounding-level parity,
    so the checks are the method's own: the minimised residual is finite, no
    larger than beta, and equals the true residual of the returned iterate."""
    A, b = _system()
    prm = dict(m=512, t=2, s=1024, zeta=8, tol=1e-300, seed=5, max_outer=1)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        x, info = P.solve(*to_dev(A), tvec(b), forced_k=[512], record_true_residual=True, **prm)
    assert info["inner_k"][0] == 512 and info["stop_reason"][0] == "forced"
    h = np.asarray(info["residual_history"])
    assert np.all(np.isfinite(h)) and h[1] <= h[0] * (1 + 1e-12)
    tr = np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) / np.linalg.norm(b)
    assert abs(tr - h[1]) <= 1e-6 * max(tr, 1e-300) + 1e-14


def test_unforced_at_the_limits_reaches_tol():
    A, b = _system()
    prm = dict(m=512, t=8, s=1024, zeta=16, tol=1e-10, seed=9, max_outer=100)
    x, info = P.solve(*to_dev(A), tvec(b), **prm)
    assert info["converged"]
    tr = np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) / np.linalg.norm(b)
    assert tr <= 1e-10 * (1 + 1e-4)
    assert np.all(np.asarray(info["cond_at_stop"]) <= 1e15 * (1 + 1e-12))
