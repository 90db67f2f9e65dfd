"""Flexible GMRES with a sketched-GMRES inner solve: the method, step by step.

Restated from Guettel & Pearson, arXiv 2506.18408:

* Outer loop -- FGMRES, Algorithm 1 (Section 2): r0 = b - A x0,
  beta = ||r0||, v1 = r0/beta; step j computes z_j = M_j^{-1} v_j, w = A z_j,
  orthogonalises w against v_1..v_j by modified Gram-Schmidt, h_{j+1,j} =
  ||w||, v_{j+1} = w/h_{j+1,j}; the iterate is x0 + Z_j y with y minimising
  ||beta e1 - H_j y|| over the (j+1) x j Hessenberg matrix.
* FFOM residual, eq. (2.1): ||r~_j|| = h_{j+1,j} |e_j^T H_j^{-1} beta e1|.
* Residual bound, eq. (2.2): ||r_j|| <= ||r~_{j-1}|| ||r^_j||, with
  ||r~_0|| read as beta (the j = 1 case of Section 2.1).
* Recursive bound, eq. (2.3) (Section 2.3): ||r_j|| <= delta_j ||r_{j-1}||
  with delta_j = ||r^_j|| / sqrt(1 - delta_{j-1}^2), delta_0 = 0, valid
  while every delta so far is below one (recorded as NaN once
  1 - delta^2 <= 0, where the recursion has no real value).
* Inner solve -- sGMRES, eq. (1.2) and Section 3: B_k spans
  K_k(A, v_j) with b_1 = v_j, built by truncated Arnoldi (Section 4.1: each
  new vector is orthogonalised against the previous t basis vectors only, by
  modified Gram-Schmidt as in Saad's incomplete orthogonalisation; t = 0 only
  normalises); z_j = B_k y_k with y_k = argmin ||S v_j - S A B_k y||.
* Inner dimension k as large as possible subject to (Section 3)
  C1: k <= m; C2: cond(S A B_k) <= threshold (1e15 in the paper);
  C3: the FGMRES residual predicted by eq. (2.2), ||r~_{j-1}|| times the
  (sketched) inner residual, is <= tol.

Readings where the paper is silent (each listed with its reason in the
design notes): tol is relative to ||b||; C2 uses the incremental estimate of
oracle.ice (rule "ice") or the SVD (rule "exact"), and a violation at step i
drops column i (k = i - 1); C3 uses the sketched residual ||S(v_j - A z)||
from the QR; the inner cycle also stops (k = i) if the orthogonalised vector
is exactly zero; the outer loop stops when the minimised residual
|g_{j+1}| <= tol ||b||, or h_{j+1,j} = 0 (exact solution, Section 2.1).

Pins: tests/test_oracle_sfgmres.py (dense LU on tiny systems; S = I reduces
sGMRES to GMRES, checked against scipy.sparse.linalg.gmres; inner m = 1 gives
full GMRES; an exact preconditioner converges in one step; monotone
residuals, ||r_j|| <= ||r~_j||, the bound (2.2), the FFOM closed form against
an explicit residual, and the Arnoldi-like relation A Z = V H).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .householder import HouseholderQR
from .ice import IncrementalCond
from .sketch import sketch_matrix, apply_sketch

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1


@dataclasses.dataclass
class OracleResult:
    x: np.ndarray
    status: int
    outer_iters: int
    residual_history: list          # |g_{j+1}| / ||b||, j = 0..J (entry 0: beta/||b||)
    true_residual_history: list     # ||b - A x_j|| / ||b||, j = 1..J (if recorded)
    inner_k: list
    stop_reason: list
    cond_at_stop: list              # condition estimate of S A B_k at the chosen k
    inner_sketched_residual: list   # ||S(v_j - A z_j)|| at the chosen k
    inner_true_residual: list       # ||v_j - A z_j||
    ffom_residual: list             # ||r~_j|| (absolute)
    bound: list                     # ||r~_{j-1}|| ||r^_j|| (absolute)
    delta: list                     # delta_j of eq. (2.3)
    H: np.ndarray
    nb: float
    trace: list
    Z: np.ndarray = None            # n x J preconditioned basis (keep_basis=True)
    V: np.ndarray = None            # n x (J+1) orthonormal basis (keep_basis=True)


def arnoldi_window(i, t):
    """Basis indices (0-based, oldest first) that w = A b_i is orthogonalised
    against at inner step i (1-based): the t most recent vectors
    b_{i-t+1}, ..., b_i, i.e. Python indices i-t .. i-1, fewer while i < t
    (Section 4.1's truncation to the previous t vectors; t = 0: none)."""
    return range(max(0, i - t), i)


def _cond_exact(R):
    sv = np.linalg.svd(R, compute_uv=False)
    return math.inf if sv[-1] == 0.0 else float(sv[0] / sv[-1])


def sgmres_cycle(A, v, sketch, *, m, t, tol_abs, factor, cond_threshold=1e15,
                 c2_rule="ice", forced_k=None, trace=None):
    """One inner sGMRES solve of A z = v (||v|| = 1), zero initial guess.

    Returns (z, info) with info = dict(k, reason, cond, rho_hat, y, basis);
    basis lists the normalised truncated-Arnoldi vectors b_1, b_2, ... formed
    before the cycle stopped (k of them after a stop by C1, C3 or a forced
    dimension, k + 1 after C2, which drops the last column).
    """
    d0 = sketch(v)
    s = d0.shape[0]
    qr = HouseholderQR(s, m)
    qr.set_rhs(d0)
    ice = IncrementalCond()
    basis = [np.array(v, dtype=np.float64, copy=True)]
    k = None
    reason = None
    conds = []
    rhos = []
    for i in range(1, m + 1):
        w = A @ basis[i - 1]
        c = sketch(w)
        col = qr.append(c)
        if c2_rule == "ice":
            kappa = ice.append(col)
        else:
            kappa = _cond_exact(qr.R[:i, :i])
        conds.append(kappa)
        rho_hat = qr.residual_norm()
        rhos.append(rho_hat)
        if trace is not None:
            trace.append(dict(i=i, c=c.copy(), kappa=kappa, rho_hat=rho_hat))
        if forced_k is not None:
            if i == forced_k:
                k, reason = i, "forced"
                break
        else:
            if i > 1 and kappa > cond_threshold:      # C2: drop column i
                k, reason = i - 1, "C2"
                break
            if factor * rho_hat <= tol_abs:           # C3
                k, reason = i, "C3"
                break
            if i == m:                                # C1
                k, reason = m, "C1"
                break
        # truncated Arnoldi: MGS against the last t basis vectors, oldest first
        for l in arnoldi_window(i, t):
            h = float(w @ basis[l])
            w = w - h * basis[l]
        eta = float(np.linalg.norm(w))
        if eta == 0.0:
            if forced_k is not None:
                raise RuntimeError("inner Krylov breakdown before the forced dimension")
            k, reason = i, "breakdown"
            break
        basis.append(w / eta)
    y = qr.solve(k)
    z = np.zeros_like(basis[0])
    for l in range(k):
        z = z + y[l] * basis[l]
    info = dict(k=k, reason=reason, cond=conds[k - 1], rho_hat=rhos[k - 1], y=y, basis=basis)
    return z, info


class RightPreconditioned:
    """The operator A M^{-1} of right preconditioning (M has .solve)."""

    def __init__(self, A, M):
        self.A = A
        self.M = M

    def __matmul__(self, v):
        return self.A @ self.M.solve(v)


def sfgmres(A, b, x0=None, *, m, t, s, zeta, tol, seed, max_outer=100,
            cond_threshold=1e15, c2_rule="ice", forced_k=None, sketch=None,
            record_true_residual=True, trace=False, keep_basis=False,
            precond=None, mid_outer=0) -> OracleResult:
    """FGMRES (Algorithm 1) preconditioned by one sGMRES cycle per step.

    precond (an object with .solve(r) = M^{-1} r, e.g. oracle.ilu.ILU0):
    right preconditioning; the inner cycle solves A M^{-1} u = v_j and the
    outer step takes z_j = M^{-1} u, so Algorithm 1 keeps A and b - A x.

    mid_outer > 0: two-level FGMRES (Section 5's multi-level FGMRES): z_j is
    the result of a lower-level FGMRES solve of A z = v_j (zero initial
    guess, the same sGMRES cycles as its preconditioner) run for at most
    mid_outer steps; it stops early once eq. (2.2) predicts the top-level
    tolerance, i.e. when ||r~_{j-1}|| times its own residual is below
    tol ||b||.  The entries of inner_k are then the lower level's outer
    steps."""
    A = sp.csr_matrix(A) if not sp.issparse(A) and not hasattr(A, "__matmul__") else A
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    if not (1 <= m < s or sketch is not None) or t < 0 or t > m or not (1 <= zeta <= s) or tol <= 0:
        raise ValueError("invalid (m, t, s, zeta, tol)")
    if sketch is None:
        S = sketch_matrix(n, s, zeta, seed)

        def sketch(w):
            return apply_sketch(S, w)

    nb = float(np.linalg.norm(b))
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    empty = OracleResult(np.zeros(n), STATUS_OK, 0, [], [], [], [], [], [], [], [], [], [],
                         np.zeros((1, 0)), nb, [])
    if nb == 0.0:
        return empty
    r0 = b - A @ x0
    beta = float(np.linalg.norm(r0))
    if not math.isfinite(beta):
        raise FloatingPointError("non-finite initial residual")
    res = empty
    res.x = x0.copy()
    res.residual_history.append(beta / nb)
    if beta <= tol * nb:
        return res
    V = [r0 / beta]
    Z = []
    H = np.zeros((max_outer + 1, max_outer))
    e1 = np.zeros(max_outer + 1)
    e1[0] = beta
    factor = beta                     # ||r~_0|| read as beta
    delta = 0.0                       # delta_0 of eq. (2.3)
    status = STATUS_NOT_CONVERGED
    y = None
    J = 0
    for j in range(max_outer):
        tr = [] if trace else None
        fk = None if forced_k is None else int(forced_k[j])
        A_in = A if precond is None else RightPreconditioned(A, precond)
        if mid_outer > 0:
            # the lower level: FGMRES on A z = v_j (||v_j|| = 1), tolerance
            # relative to 1 chosen so that factor * ||v_j - A z|| <= tol ||b||
            low = sfgmres(A, V[j], m=m, t=t, s=s, zeta=zeta,
                          tol=tol * nb / factor if math.isfinite(factor) else tol * nb,
                          seed=seed, max_outer=mid_outer, cond_threshold=cond_threshold,
                          c2_rule=c2_rule, sketch=sketch, record_true_residual=False,
                          precond=precond)
            z = low.x
            info = dict(k=low.outer_iters, reason="mid", cond=math.nan, rho_hat=math.nan)
        else:
            z, info = sgmres_cycle(A_in, V[j], sketch, m=m, t=t, tol_abs=tol * nb,
                                   factor=factor, cond_threshold=cond_threshold,
                                   c2_rule=c2_rule, forced_k=fk, trace=tr)
            if precond is not None:
                z = precond.solve(z)                  # z_j = M^{-1} B_k y_k
        Z.append(z)
        w = A @ z
        rhat = float(np.linalg.norm(V[j] - w))
        for i in range(j + 1):                        # modified Gram-Schmidt
            H[i, j] = float(V[i] @ w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        Q, R = np.linalg.qr(H[:j + 2, :j + 1], mode="complete")
        g = Q.T @ e1[:j + 2]
        rho = abs(float(g[j + 1]))
        y = sla.solve_triangular(R[:j + 1, :j + 1], g[:j + 1], lower=False)
        try:
            yF = np.linalg.solve(H[:j + 1, :j + 1], e1[:j + 1])
            ffom = H[j + 1, j] * abs(float(yF[-1]))
        except np.linalg.LinAlgError:
            ffom = math.inf
        res.bound.append(factor * rhat)
        factor = ffom if math.isfinite(ffom) else math.inf
        q = 1.0 - delta * delta
        delta = rhat / math.sqrt(q) if q > 0.0 else math.nan
        res.delta.append(delta)
        res.inner_k.append(info["k"])
        res.stop_reason.append(info["reason"])
        res.cond_at_stop.append(info["cond"])
        res.inner_sketched_residual.append(info["rho_hat"])
        res.inner_true_residual.append(rhat)
        res.ffom_residual.append(ffom)
        res.residual_history.append(rho / nb)
        if trace:
            res.trace.append(tr)
        J = j + 1
        if record_true_residual:
            xj = x0 + np.column_stack(Z) @ y
            res.true_residual_history.append(float(np.linalg.norm(b - A @ xj)) / nb)
        if not all(math.isfinite(v) for v in (rho, H[j + 1, j])):
            raise FloatingPointError("non-finite outer quantity")
        if H[j + 1, j] == 0.0:                        # exact solution in span(Z)
            status = STATUS_OK
            break
        V.append(w / H[j + 1, j])
        if rho <= tol * nb:
            status = STATUS_OK
            break
    res.x = x0 + np.column_stack(Z) @ y
    res.status = status
    res.outer_iters = J
    res.H = H[:J + 1, :J]
    if keep_basis:
        res.Z = np.column_stack(Z)
        res.V = np.column_stack(V)
    return res


def transpose_csr(row_ptr, col_idx, val, n):
    """CSR of A^T (columns sorted) and the map perm with val_T = val[perm]."""
    nnz = len(col_idx)
    P = sp.csr_matrix((np.arange(nnz, dtype=np.float64), np.asarray(col_idx), np.asarray(row_ptr)),
                      shape=(n, n))
    T = P.T.tocsr()
    T.sort_indices()
    perm = T.data.astype(np.int64)
    return (T.indptr.astype(np.int32), T.indices.astype(np.int32),
            np.asarray(val, dtype=np.float64)[perm], perm)


def adjoint_gradient(row_ptr, col_idx, lam, x):
    """dL/dA on A's pattern: grad[p] = -lam[row(p)] * x[col(p)] for
    A x = b, A^T lam = dL/dx."""
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(np.asarray(row_ptr)))
    return -np.asarray(lam)[rows] * np.asarray(x)[np.asarray(col_idx)]
