"""Seeded matrix and vector generators (input construction only).

Conventions shared by every generator:

* CSR with ``int32`` ``row_ptr`` (n+1) and ``col_idx`` (nnz), ``float64``
  values, columns sorted ascending inside each row, no explicit zeros.
* Grid node ``(ix, iy[, iz])`` is unknown ``ix + N*iy (+ N*N*iz)``
  (lexicographic order); homogeneous Dirichlet boundaries, i.e. neighbours
  outside the grid are dropped.
* Convection-diffusion rows discretise ``-div(kappa grad u) + c.grad u`` with
  central diffusion and first-order upwind convection, multiplied through by
  ``h^2`` with ``h = 1/(N+1)``: for a face of diffusion coefficient ``k_f`` the
  neighbour entry is ``-k_f`` and the diagonal gains ``k_f``; for a convection
  component ``c`` the upwind neighbour (west for ``c > 0``, east for ``c < 0``)
  gets ``-h|c|`` and the diagonal gains ``h|c|``.
* Random numbers come from ``numpy.random.default_rng([config, purpose])``
  with purpose 0 = matrix, 1 = right-hand side, 2 = parameter vector theta,
  3 = target vector.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _row_col_order(r: np.ndarray, c: np.ndarray, n: int) -> np.ndarray:
    """Stable permutation that sorts entries by row, then column (the order
    of np.lexsort((c, r)), from one integer key: an order of magnitude faster
    at 10^7-10^8 entries)."""
    return np.argsort(r * np.int64(n) + c, kind="stable")


def _assemble(n: int, rows: list, cols: list, vals: list) -> CSR:
    """Assemble CSR from per-offset (row, col, value) arrays; sorts columns."""
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals).astype(np.float64)
    order = _row_col_order(r, c, n)
    r, c, v = r[order], c[order], v[order]
    counts = np.bincount(r, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), c.astype(np.int32), v)


def _stencil_parts(N: int, dim: int):
    """Index helpers for an N^dim grid: node coordinates and the offsets list.

    Returns (coords, offsets) with offsets as (axis, direction) pairs, where
    direction -1 is the lower neighbour (west/south/down) and +1 the upper.
    """
    n = N ** dim
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for _ in range(dim):
        coords.append(rem % N)
        rem = rem // N
    offsets = [(a, d) for a in range(dim) for d in (-1, +1)]
    return idx, coords, offsets


def convdiff2d(N: int, kappa: float = 1.0, c=(10.0, 10.0)) -> CSR:
    """Constant-coefficient 5-point convection-diffusion on an N x N grid."""
    return _convdiff_const(N, 2, kappa, c)


def convdiff3d(N: int, kappa: float = 1.0, c=(50.0, 50.0, 50.0)) -> CSR:
    """Constant-coefficient 7-point convection-diffusion on an N^3 grid."""
    return _convdiff_const(N, 3, kappa, c)


def _assemble_slots(n: int, slots: list) -> CSR:
    """CSR from per-row slots listed in ascending column order: each slot is
    (cols, vals, mask) over all n rows; masked-out entries are dropped.  The
    result equals _assemble of the same entries (rows in order, columns
    ascending) without a sort: entry (r, k) goes to position row_ptr[r] +
    (number of kept slots before k in row r)."""
    counts = np.zeros(n, dtype=np.int64)
    for _, _, m in slots:
        counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = row_ptr[:-1].copy()
    for c, v, m in slots:
        p = pos[m]
        col_idx[p] = c[m]
        val[p] = v[m]
        pos += m
    return CSR(n, row_ptr.astype(np.int32), col_idx, val)


def _stencil_slot_order(dim: int):
    """(axis, direction) of the neighbours in ascending column order, with
    None for the diagonal: -N^(dim-1) ... -1, 0, +1 ... +N^(dim-1)."""
    lower = [(a, -1) for a in reversed(range(dim))]
    upper = [(a, +1) for a in range(dim)]
    return lower + [None] + upper


def _convdiff_const(N, dim, kappa, c) -> CSR:
    h = 1.0 / (N + 1)
    n = N ** dim
    idx, coords, offsets = _stencil_parts(N, dim)
    stride = [N ** a for a in range(dim)]
    slots = []
    for od in _stencil_slot_order(dim):
        if od is None:
            slots.append((idx, np.full(n, 2 * dim * kappa + h * sum(abs(ci) for ci in c)),
                          np.ones(n, dtype=bool)))
            continue
        a, d = od
        ok = coords[a] + d >= 0 if d < 0 else coords[a] + d < N
        ca = c[a]
        upw = h * max(ca, 0.0) if d < 0 else -h * min(ca, 0.0)
        slots.append((idx + d * stride[a], np.full(n, -kappa - upw), ok))
    return _assemble_slots(n, slots)


def convdiff3d_varcoef(N: int, rng: np.random.Generator, kmin=0.1, kmax=10.0,
                       c=(50.0, 50.0, 50.0)) -> CSR:
    """7-point convection-diffusion with nodal diffusion log-uniform in [kmin, kmax].

    The coefficient on the face between nodes i and j is the harmonic mean
    2 k_i k_j / (k_i + k_j); a boundary face uses the node's own coefficient.
    """
    h = 1.0 / (N + 1)
    n = N ** 3
    kap = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=n))
    idx, coords, offsets = _stencil_parts(N, 3)
    stride = [1, N, N * N]
    diag = np.full(n, h * sum(abs(ci) for ci in c))
    off = {}
    # (the diagonal accumulates the faces in the order of `offsets`)
    for a, d in offsets:
        ok = coords[a] + d >= 0 if d < 0 else coords[a] + d < N
        j = np.where(ok, idx + d * stride[a], idx)
        kf = 2.0 * kap * kap[j] / (kap + kap[j])
        diag[ok] += kf[ok]
        diag[~ok] += kap[~ok]
        ca = c[a]
        upw = h * max(ca, 0.0) if d < 0 else -h * min(ca, 0.0)
        off[(a, d)] = (idx + d * stride[a], -kf - upw, ok)
    slots = [(idx, diag, np.ones(n, dtype=bool)) if od is None else off[od]
             for od in _stencil_slot_order(3)]
    return _assemble_slots(n, slots)


def _powerlaw_alpha(Lmin: int, Lmax: int, mean: float) -> float:
    L = np.arange(Lmin, Lmax + 1, dtype=np.float64)

    def m(alpha):
        p = L ** (-alpha)
        return float((L * p).sum() / p.sum())

    lo, hi = 0.0, 5.0  # m() decreases in alpha
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if m(mid) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_random(n: int, rng: np.random.Generator, Lmin=4, Lmax=256, mean=32.0) -> CSR:
    """Random nonsymmetric sparse matrix with power-law row lengths.

    Row lengths L_i (diagonal included) follow P(L) ~ L^-alpha on
    {Lmin..Lmax} with alpha chosen so that E[L] = mean.  Each row holds the
    diagonal plus L_i - 1 distinct off-diagonal columns drawn uniformly; the
    off-diagonal values are N(0,1) and the diagonal is the sum of the row's
    off-diagonal magnitudes plus one (strict diagonal dominance).
    """
    alpha = _powerlaw_alpha(Lmin, Lmax, mean)
    Ls = np.arange(Lmin, Lmax + 1)
    p = Ls.astype(np.float64) ** (-alpha)
    p /= p.sum()
    L = rng.choice(Ls, size=n, p=p).astype(np.int64)
    L = np.minimum(L, n)
    noff = L - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), noff)
    cols = rng.integers(0, n - 1, size=rows.shape[0], dtype=np.int64)
    cols = cols + (cols >= rows)  # skip the diagonal
    # redraw duplicate (row, col) pairs until every row's columns are distinct
    while True:
        order = _row_col_order(rows, cols, n)
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.shape[0], dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            break
        newc = rng.integers(0, n - 1, size=nd, dtype=np.int64)
        cols[dup] = newc + (newc >= rows[dup])
    vals = rng.standard_normal(rows.shape[0])
    diag = np.bincount(rows, weights=np.abs(vals), minlength=n) + 1.0
    idx = np.arange(n, dtype=np.int64)
    return _assemble(n, [rows, idx], [cols, idx], [vals, diag])


def theta_convdiff2d_parts(N: int = 512, patches: int = 8, kappa: float = 1.0):
    """Pieces of the parameterised 2D operator A(theta).

    A(theta) = L + sum_p c_p (Ux_p + Uy_p), where L is the h^2-scaled 5-point
    diffusion with coefficient kappa, the grid is split into patches x patches
    square patches, patch p holds convection c_p (1, 1) with c_p > 0, and
    Ux/Uy are the unit first-order upwind convection stencils (diagonal +h,
    west/south neighbour -h).  Returns (pattern CSR with the diffusion values,
    ux values, uy values, patch index of each nonzero's row); every value array
    is aligned with the CSR pattern.
    """
    h = 1.0 / (N + 1)
    n = N * N
    idx, coords, offsets = _stencil_parts(N, 2)
    stride = [1, N]
    rows, cols, lap, ux, uy = [idx], [idx], [np.full(n, 4 * kappa)], [np.full(n, h)], [np.full(n, h)]
    for a, d in offsets:
        ok = coords[a] + d >= 0 if d < 0 else coords[a] + d < N
        k = int(ok.sum())
        rows.append(idx[ok])
        cols.append(idx[ok] + d * stride[a])
        lap.append(np.full(k, -kappa))
        ux.append(np.full(k, -h if (a == 0 and d < 0) else 0.0))
        uy.append(np.full(k, -h if (a == 1 and d < 0) else 0.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    order = np.lexsort((c, r))
    pat = _assemble(n, rows, cols, lap)
    uxv = np.concatenate(ux)[order]
    uyv = np.concatenate(uy)[order]
    rr = r[order]
    ps = N // patches
    patch = (rr % N) // ps + patches * ((rr // N) // ps)
    return pat, uxv, uyv, patch.astype(np.int64)


def theta_convdiff2d_values(theta, lap, ux, uy, patch):
    """Values of A(theta) with c_p = 10 exp(0.1 theta_p); torch or numpy inputs.

    Differentiable when theta is a torch tensor (the other arrays must then be
    tensors on the same device).
    """
    try:
        import torch
        if isinstance(theta, torch.Tensor):
            cp = 10.0 * torch.exp(0.1 * theta)
            cr = cp[patch]
            return lap + cr * ux + cr * uy
    except ImportError:  # pragma: no cover
        pass
    cp = 10.0 * np.exp(0.1 * np.asarray(theta))
    cr = cp[patch]
    return lap + cr * ux + cr * uy


def rhs(n: int, rng: np.random.Generator, kind: str) -> np.ndarray:
    if kind == "u01":
        return rng.uniform(0.0, 1.0, size=n)
    if kind == "u11":
        return rng.uniform(-1.0, 1.0, size=n)
    if kind == "normal":
        return rng.standard_normal(n)
    raise ValueError(kind)


def sketch_seed(cfg: int) -> int:
    return 1000 + cfg


# Named workloads: (generator, solver parameters).  "m" is the inner sGMRES
# maximum basis dimension, "t" the Arnoldi truncation window, "s" the sketch
# rows, "zeta" the nonzeros per sketch column.
WORKLOADS = {
    1: dict(name="convdiff2d_64", m=30, t=2, s=60, zeta=8, tol=1e-8, max_outer=20, rhs="u01"),
    2: dict(name="convdiff3d_128", m=100, t=2, s=400, zeta=8, tol=1e-8, max_outer=100, rhs="u11"),
    3: dict(name="powerlaw_1M", m=150, t=4, s=600, zeta=8, tol=1e-8, max_outer=100, rhs="normal"),
    4: dict(name="theta_convdiff2d_512", m=60, t=2, s=240, zeta=8, tol=1e-8, max_outer=100, rhs="u01"),
    5: dict(name="varcoef_convdiff3d_256", m=200, t=2, s=800, zeta=8, tol=1e-8, max_outer=100, rhs="u11"),
}


def make_workload(cfg: int, scale: int | None = None):
    """Build (CSR, b, params) for a named workload.

    ``scale`` overrides the grid size N (stencil workloads) or n (power-law)
    to get a smaller instance with the same structure.
    """
    p = dict(WORKLOADS[cfg])
    rng_m = np.random.default_rng([cfg, 0])
    rng_b = np.random.default_rng([cfg, 1])
    if cfg == 1:
        A = convdiff2d(scale or 64, 1.0, (10.0, 10.0))
    elif cfg == 2:
        A = convdiff3d(scale or 128, 1.0, (50.0, 50.0, 50.0))
    elif cfg == 3:
        A = powerlaw_random(scale or 1_000_000, rng_m)
    elif cfg == 4:
        N = scale or 512
        pat, ux, uy, patch = theta_convdiff2d_parts(N, 8 if N >= 8 else 1)
        theta = np.random.default_rng([cfg, 2]).standard_normal(64 if N >= 8 else 1)
        val = theta_convdiff2d_values(theta, pat.val, ux, uy, patch)
        A = CSR(pat.n, pat.row_ptr, pat.col_idx, val)
        p["theta"] = theta
        p["parts"] = (pat.val, ux, uy, patch)
        p["x_target"] = np.random.default_rng([cfg, 3]).uniform(0.0, 1.0, size=A.n)
    elif cfg == 5:
        A = convdiff3d_varcoef(scale or 256, rng_m)
    else:
        raise ValueError(cfg)
    b = rhs(A.n, rng_b, p["rhs"])
    p["seed"] = sketch_seed(cfg)
    p["cfg"] = cfg
    return A, b, p
