"""GPU parity of the individual kernels against the oracle (bit-exact where
the arithmetic is integer or order-free, tight tolerances otherwise)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, dev, ragged_powerlaw, \
    with_long_and_empty_rows

pytestmark = [pytest.mark.gpu, requires_gpu]

SKETCH_SIZES = [(4096, 60, 8, 1001), (2_097_152, 400, 8, 1002), (1_000_000, 600, 8, 1003),
                (262_144, 240, 8, 1004), (12345, 37, 1, 5), (777, 100, 16, 2**63 + 11),
                (1000, 13, 13, 42)]


@pytest.mark.parametrize("n,s,zeta,seed", SKETCH_SIZES)
def test_sketch_materialize_bit_exact(n, s, zeta, seed):
    rows, signs = P.sketch_materialize(n, s, zeta, seed)
    ro, so = oracle.sketch_columns(n, s, zeta, seed)
    assert np.array_equal(rows.cpu().numpy(), ro)
    assert np.array_equal(signs.cpu().numpy(), so)


def test_sketch_materialize_bit_exact_largest_sampled():
    """All 16.8M columns of the 256^3 workload's sketch on the GPU; a random
    sample of 400k columns recomputed by the oracle."""
    n, s, zeta, seed = 16_777_216, 800, 8, 1005
    rows, signs = P.sketch_materialize(n, s, zeta, seed)
    cols = np.sort(np.random.default_rng(0).choice(n, size=400_000, replace=False))
    cols = np.concatenate(([0, 1, n - 2, n - 1], cols))
    ro, so = oracle.sketch_columns(n, s, zeta, seed, cols=cols)
    idx = torch.from_numpy(cols).to(dev())
    assert np.array_equal(rows[idx].cpu().numpy(), ro)
    assert np.array_equal(signs[idx].cpu().numpy(), so)


@pytest.mark.parametrize("n,s,zeta,seed", [(5000, 60, 8, 1), (300_001, 400, 8, 2), (999, 20, 3, 3)])
def test_sketch_apply_integer_bit_exact(n, s, zeta, seed):
    w = np.random.default_rng(seed).integers(-10**6, 10**6, size=n).astype(np.float64)
    c = P.sketch_apply(tvec(w), s, zeta, seed).cpu().numpy()
    co = oracle.apply_sketch(oracle.sketch_matrix(n, s, zeta, seed), w)
    assert np.array_equal(c, co)


def test_sketch_apply_real():
    n, s, zeta, seed = 200_000, 400, 8, 9
    w = np.random.default_rng(1).standard_normal(n)
    c = P.sketch_apply(tvec(w), s, zeta, seed).cpu().numpy()
    co = oracle.apply_sketch(oracle.sketch_matrix(n, s, zeta, seed), w)
    assert np.abs(c - co).max() <= 1e-13 * np.abs(co).max()


def _int_matrix(A: W.CSR, seed):
    v = np.random.default_rng(seed).integers(-8, 9, size=A.nnz).astype(np.float64)
    return W.CSR(A.n, A.row_ptr, A.col_idx, v)


SPMV_CASES = {
    "convdiff2d_64": lambda: W.convdiff2d(64),
    "convdiff3d_37": lambda: W.convdiff3d(37),
    "powerlaw_3001": lambda: ragged_powerlaw(3001, 4),
    "powerlaw_200k": lambda: ragged_powerlaw(200_000, 5),
    "long_and_empty_rows": lambda: with_long_and_empty_rows(5003, 6),
    "single_row": lambda: W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32),
                                np.array([3.0])),
}


@pytest.mark.parametrize("case", list(SPMV_CASES))
@pytest.mark.parametrize("nwin", [0, 2, 5])
def test_spmv_sketch_integer_bit_exact(case, nwin):
    A = _int_matrix(SPMV_CASES[case](), 7)
    n = A.n
    s = 60 if n >= 60 else max(2, n)
    zeta = min(8, s)
    rng = np.random.default_rng(8)
    u = rng.integers(-8, 9, size=n).astype(np.float64)
    U = rng.integers(-8, 9, size=(n, nwin)).astype(np.float64)
    w, c, d, nrm = P.spmv_sketch(*to_dev(A), tvec(u), s, zeta, 77, scale=1.0,
                                 U=tvec(U) if nwin else None)
    As = A.to_scipy()
    wo = As @ u
    assert np.array_equal(w.cpu().numpy(), wo)
    co = oracle.apply_sketch(oracle.sketch_matrix(n, s, zeta, 77), wo)
    assert np.array_equal(c.cpu().numpy(), co)
    if nwin:
        assert np.array_equal(d.cpu().numpy(), U.T @ wo)
    assert nrm.item() == float(wo @ wo)


@pytest.mark.parametrize("zeta", [1, 5, 9, 13, 16])
def test_spmv_sketch_zeta_groups_integer_bit_exact(zeta):
    """The packed sketch holds ceil(zeta/8) groups of eight entries; zeta of
    1, 5 (one partial group), 9, 13 (a partial second group) and 16 (two
    full groups), through the fused SpMV's scatter and through the plain
    sketch kernel: integers, so every sum is exact and must match bit for
    bit."""
    A = _int_matrix(W.convdiff3d(21), 3)
    n, s, seed = A.n, 300, 2**40 + 7
    u = np.random.default_rng(zeta).integers(-8, 9, size=n).astype(np.float64)
    So = oracle.sketch_matrix(n, s, zeta, seed)
    w, c, _, _ = P.spmv_sketch(*to_dev(A), tvec(u), s, zeta, seed)
    wo = A.to_scipy() @ u
    assert np.array_equal(w.cpu().numpy(), wo)
    assert np.array_equal(c.cpu().numpy(), oracle.apply_sketch(So, wo))
    c2 = P.sketch_apply(tvec(u), s, zeta, seed).cpu().numpy()
    assert np.array_equal(c2, oracle.apply_sketch(So, u))


@pytest.mark.parametrize("case", ["convdiff3d_37", "powerlaw_200k", "long_and_empty_rows"])
def test_spmv_sketch_real(case):
    A = SPMV_CASES[case]()
    A = W.CSR(A.n, A.row_ptr, A.col_idx, np.random.default_rng(1).standard_normal(A.nnz))
    n = A.n
    rng = np.random.default_rng(2)
    u = rng.standard_normal(n)
    U = rng.standard_normal((n, 3))
    w, c, d, nrm = P.spmv_sketch(*to_dev(A), tvec(u), 400, 8, 5, scale=0.37, U=tvec(U))
    As = A.to_scipy()
    wo = 0.37 * (As @ u)
    absA = abs(As) @ np.abs(u) * 0.37
    assert np.all(np.abs(w.cpu().numpy() - wo) <= 1e-14 * absA + 1e-300)
    co = oracle.apply_sketch(oracle.sketch_matrix(n, 400, 8, 5), wo)
    assert np.abs(c.cpu().numpy() - co).max() <= 1e-12 * np.abs(co).max()
    assert np.allclose(d.cpu().numpy(), U.T @ wo, rtol=1e-12, atol=1e-12 * np.linalg.norm(wo))
    assert abs(nrm.item() - wo @ wo) <= 1e-12 * (wo @ wo)


@pytest.mark.parametrize("case", ["convdiff2d_64", "powerlaw_3001", "long_and_empty_rows",
                                  "single_row"])
def test_transpose_bit_exact(case):
    A = SPMV_CASES[case]()
    rp, ci, v, perm = P.transpose(*to_dev(A))
    rpo, cio, vo, permo = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    assert np.array_equal(rp.cpu().numpy(), rpo)
    assert np.array_equal(ci.cpu().numpy(), cio)
    assert np.array_equal(perm.cpu().numpy(), permo)
    assert np.array_equal(v.cpu().numpy(), vo)


def test_transpose_full_size_stencil():
    A = W.convdiff3d(128)
    rp, ci, v, perm = P.transpose(*to_dev(A))
    rpo, cio, vo, permo = oracle.transpose_csr(A.row_ptr, A.col_idx, A.val, A.n)
    assert np.array_equal(rp.cpu().numpy(), rpo)
    assert np.array_equal(ci.cpu().numpy(), cio)
    assert np.array_equal(perm.cpu().numpy(), permo)
