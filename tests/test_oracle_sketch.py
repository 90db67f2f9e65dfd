"""Pins of the oracle's sparse sign sketch (oracle/sketch.py)."""
import itertools
import math

import numpy as np
import pytest
import scipy.stats as st

from oracle.philox import philox4x32_10
from oracle.sketch import sketch_columns, sketch_matrix, apply_sketch


def test_columns_distinct_rows_and_range():
    for (n, s, zeta) in [(5000, 60, 8), (3000, 400, 8), (2000, 20, 20), (1000, 7, 1), (800, 50, 13)]:
        rows, signs = sketch_columns(n, s, zeta, seed=99)
        assert rows.shape == (n, zeta)
        assert rows.min() >= 0 and rows.max() < s
        srt = np.sort(rows, axis=1)
        assert np.all(srt[:, 1:] != srt[:, :-1])
        assert set(np.unique(signs)) <= {-1, 1}


def test_column_definition_scalar():
    """Re-derive a few columns with the scalar generator and Floyd's loop."""
    n, s, zeta, seed = 50, 37, 10, (7 << 32) | 5
    rows, signs = sketch_columns(n, s, zeta, seed)
    for r in [0, 1, 17, 49]:
        words = []
        for c in range((zeta + 3) // 4):
            words += philox4x32_10([r, c, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        chosen = []
        for d in range(zeta):
            i = s - zeta + d
            t = ((words[d] >> 1) * (i + 1)) >> 31
            chosen.append(i if t in chosen else t)
            assert signs[r, d] == (-1 if words[d] & 1 else 1)
        assert list(rows[r]) == chosen


def test_floyd_subset_distribution_uniform():
    """Floyd's sampling gives every zeta-subset of {0..s-1} the same probability."""
    s, zeta, n = 6, 3, 120000
    rows, _ = sketch_columns(n, s, zeta, seed=2024)
    keys = [tuple(sorted(r)) for r in rows.tolist()]
    subsets = list(itertools.combinations(range(s), zeta))
    counts = np.array([0] * len(subsets))
    index = {sub: i for i, sub in enumerate(subsets)}
    for k in keys:
        counts[index[k]] += 1
    chi2 = ((counts - n / len(subsets)) ** 2 / (n / len(subsets))).sum()
    assert chi2 < st.chi2.ppf(0.999, len(subsets) - 1)


def test_row_occupancy_and_sign_balance():
    n, s, zeta = 200000, 400, 8
    rows, signs = sketch_columns(n, s, zeta, seed=1002)
    occ = np.bincount(rows.reshape(-1), minlength=s)
    exp = n * zeta / s
    chi2 = ((occ - exp) ** 2 / exp).sum()
    assert chi2 < st.chi2.ppf(0.999, s - 1)
    npos = int((signs > 0).sum())
    tot = signs.size
    assert abs(npos - tot / 2) < 4 * math.sqrt(tot / 4)


def test_norm_preserved_in_expectation():
    """E ||S x||^2 = ||x||^2 for the +-1/sqrt(zeta) scaling."""
    n, s, zeta = 3000, 60, 8
    x = np.random.default_rng(1).standard_normal(n)
    vals = []
    for seed in range(100):
        S = sketch_matrix(n, s, zeta, seed)
        vals.append(float(np.linalg.norm(apply_sketch(S, x)) ** 2))
    vals = np.array(vals)
    mean = vals.mean()
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(mean - x @ x) < 3.5 * se


@pytest.mark.parametrize("s,d", [(400, 101), (240, 61), (1000, 50)])
def test_subspace_embedding_marchenko_pastur(s, d):
    """Singular values of S U (U orthonormal n x d) lie near 1 +- sqrt(d/s)
    (the embedding property of eq. (1.1) with eps from the measured spread)."""
    n = 20000
    U, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((n, d)))
    S = sketch_matrix(n, s, 8, seed=77)
    SU = apply_sketch(S, U)
    sv = np.linalg.svd(SU, compute_uv=False)
    lo, hi = 1 - math.sqrt(d / s), 1 + math.sqrt(d / s)
    assert sv.max() < hi * 1.15 and sv.max() > hi * 0.85
    assert sv.min() > lo * 0.85 - 0.02 and sv.min() < lo * 1.15 + 0.02
    eps = max(sv.max() ** 2 - 1, 1 - sv.min() ** 2)
    assert eps < (hi ** 2 - 1) * 1.3


def test_integer_sketch_is_exact():
    """With integer w the +-1 sums are exact, so S w is one rounding of an
    exact integer sum times 1/sqrt(zeta)."""
    n, s, zeta = 4000, 60, 8
    w = np.random.default_rng(2).integers(-1000, 1000, size=n).astype(np.float64)
    pat, scale = sketch_matrix(n, s, zeta, 5)
    rows, signs = sketch_columns(n, s, zeta, 5)
    exact = np.zeros(s, dtype=np.int64)
    np.add.at(exact, rows.reshape(-1), (signs.astype(np.int64) * w.astype(np.int64)[:, None]).reshape(-1))
    assert np.array_equal(apply_sketch((pat, scale), w), exact.astype(np.float64) * scale)
