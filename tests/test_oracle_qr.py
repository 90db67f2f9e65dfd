"""Pins of the oracle's incremental Householder QR (oracle/householder.py)."""
import numpy as np
import pytest

from oracle.householder import HouseholderQR


def _build(C, d0):
    qr = HouseholderQR(C.shape[0], C.shape[1])
    qr.set_rhs(d0)
    for j in range(C.shape[1]):
        qr.append(C[:, j])
    return qr


@pytest.mark.parametrize("s,k", [(60, 30), (400, 100), (10, 10), (5, 1)])
def test_R_matches_lapack_up_to_signs(s, k):
    rng = np.random.default_rng(s * 1000 + k)
    C = rng.standard_normal((s, k))
    qr = _build(C, rng.standard_normal(s))
    R0 = np.linalg.qr(C, mode="r")
    R = qr.R[:k, :k]
    sg = np.sign(np.diag(R)) * np.sign(np.diag(R0))
    assert np.allclose(R, sg[:, None] * R0, rtol=1e-12, atol=1e-12 * np.abs(R0).max())


def test_reflectors_orthogonal_and_reproduce_C():
    rng = np.random.default_rng(1)
    s, k = 50, 20
    C = rng.standard_normal((s, k))
    qr = _build(C, rng.standard_normal(s))
    Q = np.eye(s)
    for l, (v, tau) in enumerate(qr.refl):          # Q = H_1 H_2 ... H_k
        Hl = np.eye(s)
        Hl[l:, l:] -= tau * np.outer(v, v)
        Q = Q @ Hl
    assert np.abs(Q.T @ Q - np.eye(s)).max() < 1e-14
    Rfull = np.zeros((s, k))
    Rfull[:k] = qr.R[:k, :k]
    assert np.abs(Q @ Rfull - C).max() < 1e-13 * np.abs(C).max() * s


def test_least_squares_residual_and_solution():
    rng = np.random.default_rng(2)
    s, k = 80, 25
    C = rng.standard_normal((s, k))
    d0 = rng.standard_normal(s)
    qr = _build(C, d0)
    y_ref, *_ = np.linalg.lstsq(C, d0, rcond=None)
    y = qr.solve(k)
    assert np.allclose(y, y_ref, rtol=1e-11, atol=1e-12)
    assert abs(qr.residual_norm() - np.linalg.norm(d0 - C @ y_ref)) < 1e-12 * np.linalg.norm(d0)
    # leading-block solves use the same factorisation
    y5 = qr.solve(5)
    y5_ref, *_ = np.linalg.lstsq(C[:, :5], d0, rcond=None)
    assert np.allclose(y5, y5_ref, rtol=1e-11, atol=1e-12)


def test_zero_subdiagonal_gives_identity_reflector():
    C = np.array([[2.0, 1.0], [0.0, 3.0], [0.0, 0.0]])
    qr = _build(C, np.array([1.0, 1.0, 1.0]))
    assert qr.refl[0][1] == 0.0
    assert qr.R[0, 0] == 2.0
    assert abs(qr.residual_norm() - 1.0) < 1e-15
