"""ctypes view of ``libsfgmres.so`` (declarations of include/sfgmres.h).

Argument marshalling only: every numerical step runs in the HIP library.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfgmres.so")

OK = 0
NOT_CONVERGED = 1
ERR_INVALID = -1
ERR_HIP = -2
ERR_WORKSPACE = -3
ERR_NONFINITE = -4
ERR_BREAKDOWN = -5
ERR_TIMEOUT = -6

FP64 = 0
MIXED = 1

PRECOND_NONE = 0
PRECOND_ILU0 = 1
SKETCH_AUTO = 0
SKETCH_TABLE = 1
SKETCH_GEN = 2
MATRIX_AUTO = 0
MATRIX_CSR = 1

STOP_REASONS = {1: "C1", 2: "C2", 3: "C3", 4: "breakdown", 5: "forced", 6: "mid"}

PHASES = ("setup", "inner", "cycle_end", "outer", "true_residuals", "final", "transpose",
          "gradient")

MAX_ZETA = 16
MAX_S = 1024
MAX_M = 512
MAX_T = 8
MAX_OUTER = 2000


class Csr(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("val", C.c_void_p),
    ]


class Options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("max_outer", C.c_int32),
        ("cond_threshold", C.c_double),
        ("record_true_residual", C.c_int32),
        ("profile", C.c_int32),
        ("lookahead", C.c_int32),
        ("panel", C.c_int32),
        ("outer", C.c_int32),
        ("identity_sketch", C.c_int32),
        ("phase_timers", C.c_int32),
        ("precond", C.c_int32),
        ("mid_outer", C.c_int32),
        ("sketch_source", C.c_int32),
        ("matrix_format", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int32),
        ("converged", C.c_int32),
        ("total_inner", C.c_int32),
        ("status", C.c_int32),
        ("rel_residual", C.c_double),
        ("true_rel_residual", C.c_double),
        ("residual_history", C.POINTER(C.c_double)),
        ("true_residual_history", C.POINTER(C.c_double)),
        ("inner_k", C.POINTER(C.c_int32)),
        ("stop_reason", C.POINTER(C.c_int32)),
        ("cond_at_stop", C.POINTER(C.c_double)),
        ("inner_sketched_residual", C.POINTER(C.c_double)),
        ("inner_true_residual", C.POINTER(C.c_double)),
        ("ffom_residual", C.POINTER(C.c_double)),
        ("forced_k", C.POINTER(C.c_int32)),
        ("spmv_ms", C.c_double),
        ("spmv_launches", C.c_int64),
        ("solve_ms", C.c_double),
        ("bound", C.POINTER(C.c_double)),
        ("delta_bound", C.POINTER(C.c_double)),
        ("ffom_x", C.c_void_p),
        ("phase_ms", C.c_double * 8),
        ("sketch_generated", C.c_int32),
        ("dia_diagonals", C.c_int32),
        ("matrix_streamed", C.c_int32),
        ("reserved_i", C.c_int32),
        ("reserved", C.c_double * 2),
    ]


# name -> (restype, argtypes)
SIGNATURES = {
    "sfgmres_default_options": (C.c_int, [C.POINTER(Options)]),
    "sfgmres_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_int32, C.POINTER(Options), C.c_int32,
                                          C.POINTER(C.c_size_t)]),
    "sfgmres_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "sfgmres_destroy": (None, [C.c_void_p]),
    "sfgmres_last_error": (C.c_char_p, [C.c_void_p]),
    "sfgmres_solve": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                C.c_uint64, C.POINTER(Options), C.POINTER(Info), C.c_void_p,
                                C.c_size_t, C.c_void_p]),
    "sfgmres_solve_adjoint": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_int32, C.c_double, C.c_uint64, C.POINTER(Options),
                                        C.POINTER(Info), C.c_void_p, C.c_size_t, C.c_void_p]),
    "sfgmres_transpose_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "sfgmres_transpose": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "sfgmres_sketch_materialize": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                             C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_size_t, C.c_void_p]),
    "sfgmres_powers_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                                 C.c_int32, C.POINTER(C.c_size_t)]),
    "sfgmres_matrix_powers": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_uint64, C.c_int64, C.c_void_p,
                                        C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "sfgmres_ilu_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "sfgmres_ilu0": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_size_t, C.c_void_p]),
    "sfgmres_sketch_workspace_bytes": (C.c_int, [C.c_int64, C.c_int32, C.c_int32,
                                                 C.POINTER(C.c_size_t)]),
    "sfgmres_sketch_apply": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_uint64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                       C.c_void_p]),
    "sfgmres_spmv_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                               C.POINTER(C.c_size_t)]),
    "sfgmres_spmv_sketch": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_double,
                                      C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p,
                                      C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_size_t, C.c_void_p]),
    "sfgmres_noalloc_scratch_bytes": (C.c_int, [C.POINTER(C.c_size_t)]),
    "sfgmres_spmv_sketch_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_double,
                                              C.c_void_p, C.c_int32, C.c_int32, C.c_uint64,
                                              C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_void_p]),
}

_LIB = None


def load() -> C.CDLL:
    """Load the built library (once) and declare its entry points."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2506_18408_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def header_symbols(header_path: str) -> list:
    """Names of the functions declared in a C header (used by tests)."""
    import re
    text = open(header_path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfgmres_[a-z_0-9]+)\s*\(", text)))
