"""CPU oracle for the FGMRES-wrapped sketched GMRES solver (test infrastructure).

This package is a plain, slow, float64 restatement of the method in
Guettel & Pearson, "Stabilizing randomized GMRES through flexible GMRES"
(arXiv 2506.18408): the flexible GMRES outer loop (Algorithm 1), the sketched
GMRES inner solve (eq. (1.2) and Section 3) with the stopping rules C1-C3, the
truncated Arnoldi basis and the sparse sketch of Section 4.1, the FFOM residual
(eq. (2.1)) and the FGMRES residual bound (eq. (2.2)) with its recursive
companion (eq. (2.3)); restarted sGMRES, the paper's comparison method
(Section 4); and zero-fill ILU right preconditioning (Section 4.4).

It exists only to check the HIP library: only ``tests/``, the package smoke
check and the benchmark's CPU-baseline leg may import it.  It shares no code
with the HIP path; the two meet only in the seeded inputs of ``workloads/``.

Parity status per function is stated in each module header; every function
here is pinned by a ``-m "not gpu"`` test except where a header says
"parity unpinned".
"""
from .philox import philox4x32_10, philox4x64_10, philox4x32_10_vec  # noqa: F401
from .sketch import sketch_columns, sketch_matrix, apply_sketch, SKETCH_CTR_LAYOUT  # noqa: F401
from .householder import HouseholderQR  # noqa: F401
from .ice import IncrementalCond  # noqa: F401
from .sfgmres import sfgmres, sgmres_cycle, OracleResult, transpose_csr, adjoint_gradient  # noqa: F401
from .restarted import restarted_sgmres  # noqa: F401
from .ilu import ILU0, jp_coloring  # noqa: F401
