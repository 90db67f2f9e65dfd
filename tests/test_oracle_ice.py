"""Pins of the oracle's incremental condition estimate (oracle/ice.py)."""
import math

import numpy as np
import pytest

from oracle.ice import IncrementalCond


def _est(R):
    ice = IncrementalCond()
    out = []
    for j in range(R.shape[1]):
        out.append(ice.append(R[:j + 1, j]))
    return out


def _cond(R):
    sv = np.linalg.svd(R, compute_uv=False)
    return sv[0] / sv[-1]


def test_exact_for_one_and_two_columns():
    rng = np.random.default_rng(0)
    for _ in range(200):
        R = np.triu(rng.standard_normal((2, 2)) * np.exp(rng.uniform(-5, 5, (2, 2))))
        e = _est(R)
        assert abs(e[0] - 1.0) <= 4e-16
        assert abs(e[1] - _cond(R)) <= 1e-10 * _cond(R)


def test_exact_for_diagonal():
    rng = np.random.default_rng(1)
    d = np.exp(rng.uniform(-20, 20, 30)) * rng.choice([-1, 1], 30)
    e = _est(np.diag(d))
    for j in range(1, 31):
        dj = np.abs(d[:j])
        assert abs(e[j - 1] - dj.max() / dj.min()) <= 1e-12 * dj.max() / dj.min()


@pytest.mark.parametrize("grade", [0.0, 1.0, 3.0])
def test_lower_bound_and_close(grade):
    rng = np.random.default_rng(int(grade * 10) + 2)
    worst = 1.0
    for trial in range(20):
        k = 40
        R = np.triu(rng.standard_normal((k, k)))
        R = R * np.exp(-grade * np.arange(k) / 4)[None, :]
        R[np.diag_indices(k)] += np.sign(np.diag(R)) * 0.5
        e = _est(R)
        for j in (5, 20, 40):
            c = _cond(R[:j, :j])
            assert e[j - 1] <= c * (1 + 1e-10)
            worst = max(worst, c / e[j - 1])
    assert worst < 50.0


def test_singular_column_gives_inf():
    R = np.array([[1.0, 2.0], [0.0, 0.0]])
    e = _est(R)
    assert abs(e[0] - 1.0) <= 4e-16 and math.isinf(e[1])
