"""The matrix-powers export (the t = 0 basis A u, ..., A^p u with sketches and
norms, Section 5) against the oracle's repeated products, for several
slab widths (including the minimum, the bandwidth) and p."""
import numpy as np
import pytest

import oracle
from oracle.powers import matrix_powers
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, ragged_powerlaw

pytestmark = [pytest.mark.gpu, requires_gpu]


def _cases():
    return {
        "convdiff3d_20": W.convdiff3d(20, 1.0, (50.0, 50.0, 50.0)),
        "varcoef3d_16": W.convdiff3d_varcoef(16, np.random.default_rng([5, 0])),
        "powerlaw_5000": ragged_powerlaw(5000, 7, Lmax=64, mean=12),
    }


@pytest.mark.parametrize("name", ["convdiff3d_20", "varcoef3d_16", "powerlaw_5000"])
@pytest.mark.parametrize("p,slab", [(1, 0), (2, 0), (3, 1), (4, 0), (8, 2000)])
def test_matrix_powers_match_the_oracle(name, p, slab):
    A = _cases()[name]
    s, zeta, seed = 120, 8, 77
    u = np.random.default_rng(3).standard_normal(A.n)
    u /= np.linalg.norm(u)
    Y, Cs, nrm = P.matrix_powers(*to_dev(A), tvec(u), p, s, zeta, seed, slab_rows=slab)
    S = oracle.sketch_matrix(A.n, s, zeta, seed)
    Yr, Cr, nr = matrix_powers(A.to_scipy(), u, p, lambda w: oracle.apply_sketch(S, w))
    Y = Y.cpu().numpy()
    for l in range(p):
        ref = Yr[:, l]
        assert np.linalg.norm(Y[:, l] - ref) <= 1e-13 * np.linalg.norm(ref), l
        c = Cs.cpu().numpy()[:, l]
        assert np.linalg.norm(c - Cr[:, l]) <= 1e-13 * np.linalg.norm(Cr[:, l]), l
        assert abs(nrm.cpu().numpy()[l] - nr[l] ** 2) <= 1e-13 * nr[l] ** 2


def test_matrix_powers_integer_data_bit_exact():
    """Integer-valued A and u: every product, sum, sketch accumulation and
    norm is exact, so the order of the slabs cannot matter."""
    n = 3000
    A = ragged_powerlaw(n, 9, Lmax=20, mean=6)
    A = W.CSR(A.n, A.row_ptr, A.col_idx, np.where(A.val > 0, 1.0, -1.0))
    u = np.random.default_rng(4).integers(-2, 3, n).astype(np.float64)
    Y, Cs, nrm = P.matrix_powers(*to_dev(A), tvec(u), 3, 64, 8, 5, slab_rows=500)
    S = oracle.sketch_matrix(n, 64, 8, 5)
    Yr, Cr, nr = matrix_powers(A.to_scipy(), u, 3, lambda w: oracle.apply_sketch(S, w))
    assert np.array_equal(Y.cpu().numpy(), Yr)
    assert np.array_equal(Cs.cpu().numpy(), Cr)
    assert np.array_equal(nrm.cpu().numpy(), (Yr * Yr).sum(axis=0))
