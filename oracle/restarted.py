"""Restarted sketched GMRES, the comparison method of Section 4 of Guettel &
Pearson (arXiv 2506.18408), step by step.

Every cycle j is one sGMRES solve of A z = v_j with v_j = r_j / ||r_j||,
r_j = b - A x_j: the cycle of oracle.sfgmres.sgmres_cycle, with the same
stopping rules C1-C3 (Section 3), the C3 prediction being ||r_j|| times the
sketched inner residual (the residual the restarted iterate would have if
the sketch preserved norms exactly).  Then x_{j+1} = x_j + ||r_j|| z and the
new residual is formed explicitly.  The paper restarts on the same condition
criterion it uses inside FGMRES (Section 4, its Figure 3 comparison); the
iteration stops when ||r_j|| <= tol ||b||.

Pins: tests/test_oracle_restarted.py.  With S = I and a window t >= k, a
cycle is GMRES(k) on the current residual, so the iterates equal those of an
independently written restarted GMRES (Arnoldi relation and a dense least
squares); GMRES cycles cannot increase the residual; a zero right-hand side
and a converged initial guess return at once.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .sfgmres import (OracleResult, STATUS_NOT_CONVERGED, STATUS_OK, sgmres_cycle)
from .sketch import apply_sketch, sketch_matrix


def restarted_sgmres(A, b, x0=None, *, m, t, s, zeta, tol, seed, max_restarts=100,
                     cond_threshold=1e15, c2_rule="ice", forced_k=None,
                     sketch=None) -> OracleResult:
    """Restarted sGMRES; residual_history[j] = ||b - A x_j|| / ||b||."""
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
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    res = OracleResult(x, STATUS_OK, 0, [], [], [], [], [], [], [], [], [], [],
                       np.zeros((1, 0)), nb, [])
    if nb == 0.0:
        res.x = np.zeros(n)
        return res
    r = b - A @ x
    beta = float(np.linalg.norm(r))
    if not math.isfinite(beta):
        raise FloatingPointError("non-finite initial residual")
    res.residual_history.append(beta / nb)
    status = STATUS_NOT_CONVERGED
    if beta <= tol * nb:
        status = STATUS_OK
    J = 0
    for j in range(max_restarts):
        if status == STATUS_OK:
            break
        fk = None if forced_k is None else int(forced_k[j])
        z, info = sgmres_cycle(A, r / beta, sketch, m=m, t=t, tol_abs=tol * nb, factor=beta,
                               cond_threshold=cond_threshold, c2_rule=c2_rule, forced_k=fk)
        x = x + beta * z
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        if not math.isfinite(beta):
            raise FloatingPointError("non-finite residual")
        J = j + 1
        res.inner_k.append(info["k"])
        res.stop_reason.append(info["reason"])
        res.cond_at_stop.append(info["cond"])
        res.inner_sketched_residual.append(info["rho_hat"])
        res.residual_history.append(beta / nb)
        res.true_residual_history.append(beta / nb)
        if beta <= tol * nb:
            status = STATUS_OK
    res.x = x
    res.status = status
    res.outer_iters = J
    return res
