"""Seeded synthetic inputs for the sketched-FGMRES solver.

This package builds the linear systems that stand in for the paper's sparse
test problems (convection-diffusion stencils and random power-law sparse
matrices, all in CSR with int32 indices and float64 values) and the right-hand
sides drawn from seeded numpy generators.  It holds none of the solver's
arithmetic: both the HIP library's tests/benchmark and the CPU oracle take
their inputs from here, and neither is imported by this package.
"""
from .generators import (  # noqa: F401
    CSR,
    convdiff2d,
    convdiff3d,
    convdiff3d_varcoef,
    powerlaw_random,
    theta_convdiff2d_parts,
    theta_convdiff2d_values,
    rhs,
    WORKLOADS,
    make_workload,
    sketch_seed,
)
