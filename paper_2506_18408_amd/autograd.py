"""Reverse-mode differentiation of x = A^{-1} b through the HIP solver.

Forward: one sketched-FGMRES solve.  Backward: the adjoint solve
A^T lam = dL/dx with the same method and sketch seed (transposed CSR built
on the device), then dL/db = lam and dL/dA_ij = -lam_i x_j on A's pattern.
"""
from __future__ import annotations

import torch

from .api import SolveParams, solve, solve_adjoint


class SFGMRESSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, row_ptr, col_idx, values, b, params: SolveParams):
        x, info = solve(row_ptr, col_idx, values.detach(), b.detach().contiguous(), params=params)
        ctx.save_for_backward(row_ptr, col_idx, values, x)
        ctx.params = params
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        row_ptr, col_idx, values, x = ctx.saved_tensors
        need_val = ctx.needs_input_grad[2]
        lam, gval, _ = solve_adjoint(row_ptr, col_idx, values.detach(), gx.contiguous(),
                                     x if need_val else None, params=ctx.params,
                                     want_grad_val=need_val)
        gb = lam if ctx.needs_input_grad[3] else None
        return None, None, gval, gb, None


def sfgmres_solve(row_ptr, col_idx, values, b, params: SolveParams):
    """Differentiable solve: gradients flow to ``values`` and ``b``."""
    return SFGMRESSolve.apply(row_ptr, col_idx, values, b, params)
