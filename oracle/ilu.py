"""Zero-fill incomplete LU (ILU(0)) right preconditioning, restated plainly.

The paper runs its hardest problems with zero-fill ILU right
preconditioning (Section 4.4, the "-p" rows of Table 1; Section 4.1 says
left): M = L U with L unit lower and U upper triangular, both nonzero only
on the pattern of A, built by Gaussian elimination that drops every fill-in
entry, so that (L U)_ij = a_ij on A's pattern.  With right preconditioning
the inner sGMRES cycle works on the operator A M^{-1} and the direction
handed to the outer FGMRES loop is M^{-1} times the inner solution
(z_j = M^{-1} B_k y_k), so the outer residual stays b - A x.

The factorisation follows the IKJ form of Gaussian elimination restricted to
the pattern (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
Section 10.3.2): row i, in the elimination order, takes each of its entries
a_ik with k eliminated before i, in that order, sets a_ik <- a_ik / u_kk and
subtracts a_ik u_kj from every a_ij of its own pattern with j eliminated
after k.

Elimination order (a reading: the paper factors the matrix as given).  ILU(0)
depends on the order in which unknowns are eliminated.  Two orders:
* "natural": i = 0, 1, ..., n-1 (the paper's ILU of the matrix as given);
* "multicolor": unknowns sorted by the colour of a proper colouring of the
  symmetrised graph of A, then by index.  Unknowns of one colour are never
  coupled, so each colour is one step of a parallel factorisation and of
  each triangular solve.  The colouring is Jones & Plassmann's (SIAM J. Sci.
  Comput. 14(3), 1993): in rounds, every uncoloured vertex whose priority is
  above that of all its uncoloured neighbours takes the smallest colour not
  used by its coloured neighbours.  The priority of vertex i is
  p(i) = (2654435761 i) mod 2^32 (Knuth's multiplicative hash, distinct for
  i < 2^32).

Pins (tests/test_oracle_ilu.py): on a tridiagonal matrix (no fill exists in
the natural order) the factors equal the exact LU factors of a library LU
without pivoting; on every test matrix (L U)_ij = a_ij on the pattern; on a
full pattern ILU(0) is the exact LU in the elimination order; the solves
agree with library triangular solves of the explicit factors; the colouring
is proper and equals the sequential greedy colouring in decreasing priority
(the known equivalence for Jones-Plassmann).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HASH_MULT = 2654435761


def priority(i):
    """p(i) = (2654435761 i) mod 2^32 (as uint64 arrays)."""
    return (np.asarray(i, dtype=np.uint64) * np.uint64(HASH_MULT)) & np.uint64(0xFFFFFFFF)


def neighbours(A) -> sp.csr_matrix:
    """Pattern of A + A^T without the diagonal (CSR, sorted)."""
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G = (P + P.T).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return G


def jp_coloring(A) -> np.ndarray:
    """Jones-Plassmann colouring of the symmetrised graph of A (rounds of
    local priority maxima; smallest colour not used by coloured
    neighbours)."""
    G = neighbours(A)
    n = A.shape[0]
    p = priority(np.arange(n))
    color = np.full(n, -1, dtype=np.int64)
    while (color < 0).any():
        winners = []
        for i in np.nonzero(color < 0)[0]:
            nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
            unc = nb[color[nb] < 0]
            if np.all(p[unc] < p[i]):
                winners.append(i)
        # (winners are pairwise non-adjacent: each beats all its uncoloured
        # neighbours, so they can take their colours in any order)
        for i in winners:
            nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
            used = set(int(c) for c in color[nb] if c >= 0)
            c = 0
            while c in used:
                c += 1
            color[i] = c
    return color


def greedy_coloring_by_priority(A) -> np.ndarray:
    """Sequential greedy colouring, vertices taken in decreasing priority."""
    G = neighbours(A)
    n = A.shape[0]
    p = priority(np.arange(n))
    color = np.full(n, -1, dtype=np.int64)
    for i in np.argsort(-p.astype(np.int64), kind="stable"):
        nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
        used = set(int(c) for c in color[nb] if c >= 0)
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def elimination_order(A, kind: str = "multicolor"):
    """(order, pos, color): order[q] is the unknown eliminated q-th, pos its
    inverse; color is the colouring (None for the natural order)."""
    n = A.shape[0]
    if kind == "natural":
        order = np.arange(n)
        color = None
    elif kind == "multicolor":
        color = jp_coloring(A)
        order = np.lexsort((np.arange(n), color))
    else:
        raise ValueError(kind)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    return order, pos, color


class ILU0:
    """ILU(0) of the CSR matrix A (columns sorted) in a given elimination
    order; the factor values live on A's pattern (lu[p] for A.data[p]):
    entries a_ij with pos[j] < pos[i] hold L (unit diagonal implied), the
    others hold U."""

    def __init__(self, A, kind: str = "multicolor"):
        A = sp.csr_matrix(A)
        A.sort_indices()
        self.A = A
        n = A.shape[0]
        self.n = n
        self.order, self.pos, self.color = elimination_order(A, kind)
        ip, ix = A.indptr, A.indices
        lu = np.array(A.data, dtype=np.float64, copy=True)
        diag = np.full(n, -1, dtype=np.int64)
        for i in range(n):
            hit = np.nonzero(ix[ip[i]:ip[i + 1]] == i)[0]
            if hit.size:
                diag[i] = ip[i] + hit[0]
        if (diag < 0).any():
            raise ZeroDivisionError("ILU(0) needs every diagonal entry in the pattern")
        self.diag = diag
        pos = self.pos
        for i in self.order:
            lo, hi = ip[i], ip[i + 1]
            where = {int(ix[q]): q for q in range(lo, hi)}
            lower = [q for q in range(lo, hi) if pos[ix[q]] < pos[i]]
            lower.sort(key=lambda q: pos[ix[q]])
            for q in lower:
                k = int(ix[q])
                ukk = lu[diag[k]]
                if ukk == 0.0:
                    raise ZeroDivisionError(f"zero pivot in row {k}")
                lu[q] = lu[q] / ukk
                for r in range(ip[k], ip[k + 1]):
                    j = int(ix[r])
                    if pos[j] > pos[k] and j in where:
                        lu[where[j]] -= lu[q] * lu[r]
        if np.any(lu[diag] == 0.0):
            raise ZeroDivisionError("zero pivot")
        self.lu = lu

    def factors(self):
        """Explicit L (unit lower) and U in the elimination order, as sparse
        matrices of the permuted system (rows and columns by position)."""
        A = self.A
        rows = np.repeat(np.arange(self.n), np.diff(A.indptr))
        pr, pc = self.pos[rows], self.pos[A.indices]
        low = pc < pr
        L = sp.csr_matrix((self.lu[low], (pr[low], pc[low])), shape=A.shape) + sp.identity(self.n)
        U = sp.csr_matrix((self.lu[~low], (pr[~low], pc[~low])), shape=A.shape)
        return L.tocsr(), U.tocsr()

    def solve(self, r):
        """M^{-1} r: the forward solve with L, then the backward solve with U,
        each in the elimination order."""
        A = self.A
        ip, ix = A.indptr, A.indices
        pos = self.pos
        y = np.array(r, dtype=np.float64, copy=True)
        for i in self.order:
            acc = y[i]
            for q in range(ip[i], ip[i + 1]):
                j = ix[q]
                if pos[j] < pos[i]:
                    acc -= self.lu[q] * y[j]
            y[i] = acc
        z = y
        for i in self.order[::-1]:
            acc = z[i]
            for q in range(ip[i], ip[i + 1]):
                j = ix[q]
                if pos[j] > pos[i]:
                    acc -= self.lu[q] * z[j]
            z[i] = acc / self.lu[self.diag[i]]
        return z
