"""Pins of two-level FGMRES (Section 5's multi-level FGMRES) in the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W


def _sys():
    A = W.convdiff2d(20, 1.0, (10.0, 10.0)).to_scipy()
    b = np.random.default_rng(4).uniform(0, 1, A.shape[0])
    return A, b


def test_one_lower_step_is_one_level_fgmres():
    """mid_outer = 1: the lower level is one FGMRES step, i.e. one sGMRES
    cycle times the scalar that minimises its residual, with the same C3
    condition (its factor is 1 and its tolerance tol ||b|| / ||r~_{j-1}||);
    a rescaled z_j leaves span(Z) and so every top-level iterate unchanged."""
    A, b = _sys()
    kw = dict(m=12, t=2, s=48, zeta=8, tol=1e-9, seed=21, max_outer=80)
    one = oracle.sfgmres(A, b, **kw)
    two = oracle.sfgmres(A, b, mid_outer=1, **kw)
    assert two.outer_iters == one.outer_iters
    h1, h2 = np.array(one.residual_history), np.array(two.residual_history)
    assert np.all(np.abs(h2 - h1) <= 1e-9 * h1 + 1e-15)
    assert np.linalg.norm(two.x - one.x) <= 1e-9 * np.linalg.norm(one.x)


@pytest.mark.parametrize("mid", [2, 5])
def test_two_levels_converge_with_the_top_level_invariants(mid):
    A, b = _sys()
    kw = dict(m=12, t=2, s=48, zeta=8, tol=1e-10, seed=21, max_outer=60)
    r = oracle.sfgmres(A, b, mid_outer=mid, **kw)
    Ad = A.toarray()
    assert r.status == 0
    assert np.linalg.norm(b - Ad @ r.x) <= 1.01e-10 * np.linalg.norm(b)
    h = np.array(r.residual_history)
    assert np.all(h[1:] <= h[:-1])
    nb = np.linalg.norm(b)
    for j in range(r.outer_iters):
        assert h[j + 1] * nb <= r.bound[j] * (1 + 1e-8) + 1e-14 * nb   # eq. (2.2)
    assert all(1 <= k <= mid for k in r.inner_k)
    one = oracle.sfgmres(A, b, **kw)
    assert r.outer_iters <= one.outer_iters
