"""MI355X (gfx950) sketched-FGMRES solver: FGMRES (Algorithm 1 of Guettel &
Pearson, arXiv 2506.18408) with one sketched-GMRES cycle as the variable
preconditioner, as hand-written HIP kernels behind the C ABI in
include/sfgmres.h, with a PyTorch binding and an adjoint for autograd."""
from .api import (  # noqa: F401
    SFGMRESError,
    ilu0,
    matrix_powers,
    SolveParams,
    release_workspaces,
    sketch_apply,
    sketch_materialize,
    solve,
    solve_adjoint,
    spmv_sketch,
    transpose,
    workspace_bytes,
)
from .autograd import SFGMRESSolve, sfgmres_solve  # noqa: F401
