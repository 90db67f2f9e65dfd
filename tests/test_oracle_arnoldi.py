"""Pins of the oracle's truncated Arnoldi basis (Section 4.1: each new inner
basis vector is orthogonalised against the previous t vectors only, as in
Saad's incomplete orthogonalisation; t = 0 only normalises).

Every other pin of the solver is blind to the window: the span of
b_1..b_k is the Krylov space K_k(A, v) for any t.  These tests check the
window itself, from properties the definition fixes:
  * t >= k: the basis is orthonormal and satisfies the Arnoldi relation
    A B_{k-1} = B_k H with H upper Hessenberg;
  * 1 <= t < k: b_{i+1} is orthogonal to exactly b_{i-t+1}, ..., b_i (and,
    for a nonsymmetric A, generically not to b_{i-t}); A b_i lies in the
    span of b_{i-t+1}, ..., b_{i+1} (the recurrence has no other term);
  * t = 0: b_{i+1} is the normalised power A^i v;
  * an exact breakdown (A = 2 I) ends the cycle at k = 1.
A planted window mistake (one vector too few or too many, or the newest
vector left out) must fail them: the last test plants each one in the
oracle and checks that the pins catch it.
"""
import importlib

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

MOD = importlib.import_module("oracle.sfgmres")


def _ident(w):
    return np.array(w, copy=True)


def _nonsym(n=120, seed=7):
    """A nonsymmetric sparse matrix (random pattern, dominant diagonal)."""
    return W.powerlaw_random(n, np.random.default_rng(seed), Lmin=4, Lmax=20, mean=8).to_scipy()


def _basis(A, t, k, seed=3, sketch=None):
    n = A.shape[0]
    v = np.random.default_rng(seed).standard_normal(n)
    v /= np.linalg.norm(v)
    sk = sketch or _ident
    _, info = oracle.sgmres_cycle(A, v, sk, m=k, t=t, tol_abs=0.0, factor=1.0,
                                  cond_threshold=1e300, forced_k=k)
    return v, np.column_stack(info["basis"])


def window_violations(A, B, t, tol=1e-12, generic=1e-8):
    """Violations of the truncated-Arnoldi window in the basis B (columns
    b_1..b_k): b_{i+1} must be orthogonal to b_{i-t+1..i}, must not be
    orthogonal to b_{i-t} (nonsymmetric A), must have unit norm, and A b_i
    must lie in span(b_{i-t+1}, ..., b_{i+1})."""
    bad = []
    k = B.shape[1]
    for c in range(1, k):                      # column c holds b_{c+1}
        new = B[:, c]
        if abs(np.linalg.norm(new) - 1.0) > tol:
            bad.append(("norm", c))
        for l in range(max(0, c - t), c):      # the window b_{c-t+1}..b_c
            if abs(new @ B[:, l]) > tol:
                bad.append(("window", c, l))
        if c - t - 1 >= 0 and abs(new @ B[:, c - t - 1]) < generic:
            bad.append(("outside", c, c - t - 1))
        # recurrence: A b_c in span(b_{c-t+1}, ..., b_{c+1})
        span = B[:, max(0, c - 1 - t + 1):c + 1] if t > 0 else B[:, c:c + 1]
        Ab = A @ B[:, c - 1]
        coef, *_ = np.linalg.lstsq(span, Ab, rcond=None)
        if np.linalg.norm(Ab - span @ coef) > tol * 10 * np.linalg.norm(Ab):
            bad.append(("recurrence", c))
    return bad


@pytest.mark.parametrize("k", [6, 12])
def test_full_window_is_arnoldi(k):
    """t >= k: modified Gram-Schmidt against every previous vector, i.e. the
    Arnoldi process: an orthonormal basis with A B_{k-1} = B_k H, H upper
    Hessenberg with a positive subdiagonal."""
    A = _nonsym()
    _, B = _basis(A, t=k, k=k)
    assert B.shape[1] == k
    # modified Gram-Schmidt loses orthogonality in proportion to u times the
    # condition number of the vectors it orthogonalises, [v, A b_1, ...]
    # (Bjorck): ||I - B^T B|| <= c u kappa
    G = B.T @ B
    K = np.column_stack([B[:, 0], A @ B[:, :k - 1]])
    kappa = np.linalg.cond(K)
    bound = 10 * k * np.finfo(float).eps * kappa
    assert np.linalg.norm(G - np.eye(k), 2) <= bound
    H = B.T @ (A @ B[:, :k - 1])
    assert np.allclose(np.tril(H, -2), 0.0, atol=1e-13 * sp.linalg.norm(A))
    assert np.all(np.diag(H, -1) > 0)
    R = A @ B[:, :k - 1] - B @ H
    assert np.linalg.norm(R) <= 1e-13 * sp.linalg.norm(A) * np.sqrt(k)
    assert window_violations(A, B, t=k, tol=max(bound, 1e-13)) == []


@pytest.mark.parametrize("t", [1, 2, 4])
def test_truncated_window(t):
    """1 <= t < k: b_{i+1} is orthogonal to exactly the t previous vectors."""
    A = _nonsym()
    _, B = _basis(A, t=t, k=12)
    assert window_violations(A, B, t) == []
    # generic loss of orthogonality beyond the window (A is nonsymmetric)
    G = np.abs(B.T @ B)
    assert G[0, t + 2] > 1e-6


def test_window_property_on_the_convection_diffusion_operator():
    A = W.convdiff2d(14, 1.0, (20.0, 5.0)).to_scipy()
    for t in (1, 2, 3):
        _, B = _basis(A, t=t, k=10, seed=5)
        assert window_violations(A, B, t) == []


def test_t0_is_the_normalised_power_basis():
    """t = 0: b_{i+1} = A^i v / ||A^i v|| (only a normalisation per step)."""
    A = _nonsym(n=40, seed=11)
    k = 7
    v, B = _basis(A, t=0, k=k)
    p = v.copy()
    for i in range(k):
        assert np.linalg.norm(B[:, i] - p / np.linalg.norm(p)) <= 1e-13
        p = A @ p


def test_exact_breakdown_ends_the_cycle_at_one():
    """A = 2 I, b = e_1: A v_1 = 2 v_1 exactly, so the orthogonalised vector
    is exactly zero and the inner cycle stops at k = 1 (the sketch seeds are
    chosen where the sketched residual is a rounding residue, so C3 with
    tol = 1e-300 does not fire first); the one FGMRES step is exact."""
    n = 50
    A = sp.identity(n, format="csr") * 2.0
    b = np.zeros(n)
    b[0] = 1.0
    for seed in (2, 3):
        r = oracle.sfgmres(A, b, m=5, t=2, s=20, zeta=8, tol=1e-300, seed=seed, max_outer=3)
        assert r.inner_k == [1] and r.stop_reason == ["breakdown"]
        assert r.outer_iters == 1
        assert np.array_equal(r.x, b / 2.0)
    # at t = 0 there is no projection, so no breakdown: the power basis goes on
    z, info = oracle.sgmres_cycle(A, b, _ident, m=4, t=0, tol_abs=0.0, factor=1.0,
                                  cond_threshold=1e300, forced_k=1)
    assert info["k"] == 1 and np.allclose(z, b / 2.0)


@pytest.mark.parametrize("mutant", ["one_less", "one_more", "without_newest"])
def test_planted_window_mistakes_are_caught(monkeypatch, mutant):
    """Each plausible mistake in the window fails the pins above."""
    variants = {
        "one_less": lambda i, t: range(max(0, i - t + 1), i),
        "one_more": lambda i, t: range(max(0, i - t - 1), i),
        "without_newest": lambda i, t: range(max(0, i - t), i - 1),
    }
    monkeypatch.setattr(MOD, "arnoldi_window", variants[mutant])
    A = _nonsym()
    caught = []
    for t in (1, 2, 4):
        _, B = _basis(A, t=t, k=12)
        caught.append(bool(window_violations(A, B, t)))
    assert all(caught), caught
