"""PyTorch-facing binding of the sketched-FGMRES HIP library.

Tensors live on the current HIP device; PyTorch provides the device memory
(inputs, outputs and the one workspace blob) and the stream
(``torch.cuda.current_stream()``).  Every function marshals arguments into
the C ABI of include/sfgmres.h and raises ``SFGMRESError`` on a negative
return code.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import warnings

import numpy as np
import torch

from . import _lib as L


class SFGMRESError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sfgmres error {code}: {msg}")
        self.code = code


@dataclasses.dataclass
class SolveParams:
    """Method parameters (names follow the paper's notation where it has one).

    m: inner sGMRES basis cap k_max (rule C1); t: Arnoldi truncation window;
    s: sketch rows; zeta: nonzeros per sketch column; tol: relative
    tolerance on ||b - A x|| / ||b||; seed: sketch seed; cond_threshold: C2
    threshold (0: 1e15 in FP64, 1e15 * 2**-29 in mixed precision, whose
    basis is FP32); precision: "fp64" or "mixed"; lookahead: inner steps the host
    runs ahead of the device's last decision (0: default); panel: columns
    per decision launch (0: default 8; the stopping rule still acts after
    every column); outer: "fgmres" (Algorithm 1) or "restarted" (restarted
    sGMRES, the paper's comparison method); identity_sketch: S = I (a test
    option: needs s == n and zeta == 1; the inner cycle is then GMRES(k));
    phase_timers: per-phase GPU times into info["phase_ms"]; precond: "none"
    or "ilu0" (zero-fill ILU right preconditioning in a multicolour order,
    FGMRES outer only); mid_outer: N > 0 for two-level FGMRES, each outer
    step preconditioned by a lower-level FGMRES solve of at most N steps;
    sketch_source: "auto", "table" (packed columns of S read by the fused
    SpMV) or "gen" (columns generated inside it; FP64, zeta <= 8) -- the
    same S either way; matrix_format: "auto" (the inner SpMV reads a copy
    of A by diagonal when A is stencil-like, with the same results) or
    "csr".
    """
    m: int = 30
    t: int = 2
    s: int = 60
    zeta: int = 8
    tol: float = 1e-8
    seed: int = 0
    max_outer: int = 100
    cond_threshold: float = 0.0
    precision: str = "fp64"
    lookahead: int = 0
    panel: int = 0
    outer: str = "fgmres"
    identity_sketch: bool = False
    phase_timers: bool = False
    precond: str = "none"
    mid_outer: int = 0
    sketch_source: str = "auto"
    matrix_format: str = "auto"


_HANDLES = {}


def _handle(device: torch.device) -> C.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _HANDLES.get(idx)
    if h is None:
        lib = L.load()
        h = C.c_void_p()
        with torch.cuda.device(idx):
            rc = lib.sfgmres_create(C.byref(h))
        if rc != 0:
            raise SFGMRESError(rc, "sfgmres_create failed")
        _HANDLES[idx] = h
    return h


def _check(rc: int, h) -> int:
    if rc < 0:
        raise SFGMRESError(rc, L.load().sfgmres_last_error(h).decode())
    return rc


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _csr(row_ptr, col_idx, val) -> L.Csr:
    n = row_ptr.numel() - 1
    for name, tns, dt in (("row_ptr", row_ptr, torch.int32), ("col_idx", col_idx, torch.int32),
                          ("val", val, torch.float64)):
        if tns.dtype != dt or not tns.is_cuda or not tns.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} tensor on the GPU")
        if tns.device != row_ptr.device:
            raise ValueError(f"{name} is not on row_ptr's device")
    if col_idx.numel() != val.numel():
        raise ValueError("col_idx and val differ in length")
    return L.Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr(), val.data_ptr())


def check_vector(name: str, t, n: int, device: torch.device) -> None:
    """A vector argument of the C ABI: a contiguous float64 tensor of length n
    on `device` (the device of A).  The library cannot tell a host pointer
    from a device pointer, so anything else is rejected before a launch."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64 (got {t.dtype})")
    if t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} entries (got {t.numel()})")


def check_forced_k(forced_k, m: int) -> None:
    if forced_k is None:
        return
    fk = np.asarray(forced_k)
    if fk.size and (fk.min() < 0 or fk.max() > m):
        raise ValueError(f"forced_k entries must lie in [0, m = {m}]")


def _options(p: SolveParams, record_true_residual=False, profile=False) -> L.Options:
    o = L.Options()
    L.load().sfgmres_default_options(C.byref(o))
    o.precision = {"fp64": L.FP64, "mixed": L.MIXED}[p.precision]
    o.max_outer = p.max_outer
    o.cond_threshold = p.cond_threshold
    o.record_true_residual = 1 if record_true_residual else 0
    o.profile = int(profile)  # False/True -> 0/1; N -> every N-th inner step
    o.lookahead = p.lookahead
    o.panel = p.panel
    o.outer = {"fgmres": 0, "restarted": 1}[p.outer]
    o.identity_sketch = 1 if p.identity_sketch else 0
    o.phase_timers = 1 if p.phase_timers else 0
    o.precond = {"none": L.PRECOND_NONE, "ilu0": L.PRECOND_ILU0}[p.precond]
    o.mid_outer = p.mid_outer
    o.sketch_source = {"auto": L.SKETCH_AUTO, "table": L.SKETCH_TABLE,
                       "gen": L.SKETCH_GEN}[p.sketch_source]
    o.matrix_format = {"auto": L.MATRIX_AUTO, "csr": L.MATRIX_CSR}[p.matrix_format]
    return o


class _InfoBuffers:
    def __init__(self, J: int, forced_k=None):
        self.residual_history = np.full(J + 1, np.nan)
        self.true_residual_history = np.full(J, np.nan)
        self.inner_k = np.zeros(J, dtype=np.int32)
        self.stop_reason = np.zeros(J, dtype=np.int32)
        self.cond_at_stop = np.full(J, np.nan)
        self.inner_sketched_residual = np.full(J, np.nan)
        self.inner_true_residual = np.full(J, np.nan)
        self.ffom_residual = np.full(J, np.nan)
        self.bound = np.full(J, np.nan)
        self.delta_bound = np.full(J, np.nan)
        self.forced = None
        if forced_k is not None:
            fk = np.zeros(J, dtype=np.int32)
            fk[:min(J, len(forced_k))] = np.asarray(forced_k, dtype=np.int32)[:J]
            self.forced = fk
        self.info = L.Info()
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        self.info.residual_history = self.residual_history.ctypes.data_as(dp)
        self.info.true_residual_history = self.true_residual_history.ctypes.data_as(dp)
        self.info.inner_k = self.inner_k.ctypes.data_as(ip)
        self.info.stop_reason = self.stop_reason.ctypes.data_as(ip)
        self.info.cond_at_stop = self.cond_at_stop.ctypes.data_as(dp)
        self.info.inner_sketched_residual = self.inner_sketched_residual.ctypes.data_as(dp)
        self.info.inner_true_residual = self.inner_true_residual.ctypes.data_as(dp)
        self.info.ffom_residual = self.ffom_residual.ctypes.data_as(dp)
        self.info.bound = self.bound.ctypes.data_as(dp)
        self.info.delta_bound = self.delta_bound.ctypes.data_as(dp)
        self.info.forced_k = self.forced.ctypes.data_as(ip) if self.forced is not None else None

    def to_dict(self, rc: int) -> dict:
        J = self.info.outer_iters
        return dict(
            status=rc,
            outer_iters=J,
            converged=bool(self.info.converged),
            total_inner=self.info.total_inner,
            rel_residual=self.info.rel_residual,
            true_rel_residual=self.info.true_rel_residual,
            residual_history=self.residual_history[:J + 1].copy(),
            true_residual_history=self.true_residual_history[:J].copy(),
            inner_k=self.inner_k[:J].copy(),
            stop_reason=[L.STOP_REASONS.get(int(r), "?") for r in self.stop_reason[:J]],
            cond_at_stop=self.cond_at_stop[:J].copy(),
            inner_sketched_residual=self.inner_sketched_residual[:J].copy(),
            inner_true_residual=self.inner_true_residual[:J].copy(),
            ffom_residual=self.ffom_residual[:J].copy(),
            bound=self.bound[:J].copy(),
            delta_bound=self.delta_bound[:J].copy(),
            spmv_ms=self.info.spmv_ms,
            spmv_launches=self.info.spmv_launches,
            solve_ms=self.info.solve_ms,
            phase_ms=dict(zip(L.PHASES, list(self.info.phase_ms))),
            sketch_generated=bool(self.info.sketch_generated),
            dia_diagonals=int(self.info.dia_diagonals),
            matrix_streamed=bool(self.info.matrix_streamed),
        )


_WS = {}


def _workspace(nbytes: int, device, key: str) -> torch.Tensor:
    buf = _WS.get((key, device))
    if buf is None or buf.numel() < nbytes:
        _WS.pop((key, device), None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS[(key, device)] = buf
    return buf


def release_workspaces() -> None:
    _WS.clear()


def workspace_bytes(n, nnz, p: SolveParams, adjoint=False) -> int:
    out = C.c_size_t()
    o = _options(p)
    rc = L.load().sfgmres_workspace_bytes(n, nnz, p.m, p.t, p.s, p.zeta, C.byref(o),
                                          1 if adjoint else 0, C.byref(out))
    if rc != 0:
        raise SFGMRESError(rc, "invalid sizes for the workspace query")
    return out.value


def solve(row_ptr, col_idx, val, b, x0=None, params: SolveParams | None = None, *, out=None,
          forced_k=None, record_true_residual=False, profile=False, want_ffom=False, **kw):
    """Solve A x = b; returns (x, info dict).  ``kw`` overrides fields of params.

    want_ffom: also return the FFOM iterate of the last outer step
    (Algorithm 1) as info["ffom_x"] (a device tensor)."""
    p = dataclasses.replace(params or SolveParams(), **kw)
    A = _csr(row_ptr, col_idx, val)
    dev = row_ptr.device
    check_vector("b", b, A.n, dev)
    if x0 is not None:
        check_vector("x0", x0, A.n, dev)
    if out is not None:
        check_vector("out", out, A.n, dev)
    check_forced_k(forced_k, p.m)
    x = out if out is not None else torch.empty_like(b)
    nbytes = workspace_bytes(A.n, A.nnz, p)
    ws = _workspace(nbytes, dev, "solve")
    h = _handle(dev)
    opt = _options(p, record_true_residual, profile)
    ib = _InfoBuffers(p.max_outer, forced_k)
    xf = torch.empty_like(b) if want_ffom else None
    ib.info.ffom_x = _ptr(xf)
    rc = L.load().sfgmres_solve(h, C.byref(A), b.data_ptr(), _ptr(x0), x.data_ptr(), p.m, p.t, p.s,
                                p.zeta, p.tol, p.seed & (2**64 - 1), C.byref(opt), C.byref(ib.info),
                                ws.data_ptr(), ws.numel(), _stream())
    _check(rc, h)
    if rc == L.NOT_CONVERGED:
        warnings.warn("sfgmres: max_outer reached before tol", RuntimeWarning)
    info = ib.to_dict(rc)
    if want_ffom:
        info["ffom_x"] = xf
    return x, info


def solve_adjoint(row_ptr, col_idx, val, g, x=None, params: SolveParams | None = None, *,
                  want_grad_val=True, forced_k=None, **kw):
    """Solve A^T lam = g; returns (lam, grad_val or None, info dict) with
    grad_val[p] = -lam[row(p)] x[col(p)] when x is given."""
    p = dataclasses.replace(params or SolveParams(), **kw)
    A = _csr(row_ptr, col_idx, val)
    dev = row_ptr.device
    check_vector("g", g, A.n, dev)
    if x is not None:
        check_vector("x", x, A.n, dev)
    check_forced_k(forced_k, p.m)
    lam = torch.empty_like(g)
    gv = torch.empty_like(val) if (want_grad_val and x is not None) else None
    nbytes = workspace_bytes(A.n, A.nnz, p, adjoint=True)
    ws = _workspace(nbytes, dev, "adjoint")
    h = _handle(dev)
    opt = _options(p)
    ib = _InfoBuffers(p.max_outer, forced_k)
    rc = L.load().sfgmres_solve_adjoint(h, C.byref(A), g.data_ptr(), lam.data_ptr(),
                                        _ptr(x) if gv is not None else None, _ptr(gv), p.m, p.t,
                                        p.s, p.zeta, p.tol, p.seed & (2**64 - 1), C.byref(opt),
                                        C.byref(ib.info), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, h)
    if rc == L.NOT_CONVERGED:
        warnings.warn("sfgmres adjoint: max_outer reached before tol", RuntimeWarning)
    return lam, gv, ib.to_dict(rc)


def transpose(row_ptr, col_idx, val=None):
    """CSR of A^T and the value permutation (val_t = val[perm])."""
    if val is None:
        val = torch.zeros(col_idx.numel(), dtype=torch.float64, device=col_idx.device)
        want_val = False
    else:
        want_val = True
    A = _csr(row_ptr, col_idx, val)
    dev = row_ptr.device
    rp_t = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    col_t = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    val_t = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev) if want_val else None
    need = C.c_size_t()
    _check(L.load().sfgmres_transpose_workspace_bytes(A.n, A.nnz, C.byref(need)), None)
    ws = _workspace(need.value, dev, "transpose")
    h = _handle(dev)
    _check(L.load().sfgmres_transpose(h, C.byref(A), rp_t.data_ptr(), col_t.data_ptr(),
                                      _ptr(val_t), perm.data_ptr(), ws.data_ptr(), ws.numel(),
                                      _stream()), h)
    nnz = A.nnz
    return rp_t, col_t[:nnz], (val_t[:nnz] if val_t is not None else None), perm[:nnz]


def matrix_powers(row_ptr, col_idx, val, u, p, s, zeta, seed, slab_rows=0):
    """(Y [n, p], C [s, p], norm2 [p]): Y[:, l-1] = A^l u, C[:, l-1] its
    sketch, norm2 its squared norm (the t = 0 basis before normalisation)."""
    A = _csr(row_ptr, col_idx, val)
    dev = row_ptr.device
    check_vector("u", u, A.n, dev)
    Y = torch.empty(p, A.n, dtype=torch.float64, device=dev)   # column l-1 = row of Y
    Cs = torch.empty(p, s, dtype=torch.float64, device=dev)
    nrm = torch.empty(p, dtype=torch.float64, device=dev)
    need = C.c_size_t()
    _check(L.load().sfgmres_powers_workspace_bytes(A.n, A.nnz, p, s, zeta, C.byref(need)), None)
    ws = _workspace(need.value, dev, "powers")
    h = _handle(dev)
    _check(L.load().sfgmres_matrix_powers(h, C.byref(A), u.data_ptr(), p, s, zeta,
                                          seed & (2**64 - 1), slab_rows, Y.data_ptr(), A.n,
                                          Cs.data_ptr(), nrm.data_ptr(), ws.data_ptr(),
                                          ws.numel(), _stream()), h)
    return Y.t(), Cs.t(), nrm


def ilu0(row_ptr, col_idx, val):
    """(lu [nnz], color [n]) of the ILU(0) factorisation the ilu0
    preconditioner builds: factor values on A's pattern and the colour of
    every row (elimination order: colour, then index)."""
    A = _csr(row_ptr, col_idx, val)
    dev = row_ptr.device
    lu = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    color = torch.empty(A.n, dtype=torch.int32, device=dev)
    need = C.c_size_t()
    _check(L.load().sfgmres_ilu_workspace_bytes(A.n, A.nnz, C.byref(need)), None)
    ws = _workspace(need.value, dev, "ilu")
    h = _handle(dev)
    _check(L.load().sfgmres_ilu0(h, C.byref(A), lu.data_ptr(), color.data_ptr(), ws.data_ptr(),
                                 ws.numel(), _stream()), h)
    return lu[:A.nnz], color


def sketch_materialize(n: int, s: int, zeta: int, seed: int, device="cuda"):
    """(rows [n, zeta] int32, signs [n, zeta] int8) of the sketch S."""
    dev = torch.device(device)
    rows = torch.empty(n * zeta, dtype=torch.int32, device=dev)
    signs = torch.empty(n * zeta, dtype=torch.int8, device=dev)
    need = C.c_size_t()
    _check(L.load().sfgmres_sketch_workspace_bytes(n, s, zeta, C.byref(need)), None)
    ws = _workspace(need.value, dev, "sketch")
    h = _handle(dev)
    _check(L.load().sfgmres_sketch_materialize(h, n, s, zeta, seed & (2**64 - 1), rows.data_ptr(),
                                               signs.data_ptr(), ws.data_ptr(), ws.numel(),
                                               _stream()), h)
    return rows.view(n, zeta), signs.view(n, zeta)


def sketch_apply(w: torch.Tensor, s: int, zeta: int, seed: int) -> torch.Tensor:
    """S w for a float64 vector w."""
    n = w.numel()
    out = torch.empty(s, dtype=torch.float64, device=w.device)
    need = C.c_size_t()
    _check(L.load().sfgmres_sketch_workspace_bytes(n, s, zeta, C.byref(need)), None)
    ws = _workspace(need.value, w.device, "sketch")
    h = _handle(w.device)
    _check(L.load().sfgmres_sketch_apply(h, n, s, zeta, seed & (2**64 - 1),
                                         w.contiguous().data_ptr(), out.data_ptr(), ws.data_ptr(),
                                         ws.numel(), _stream()), h)
    return out


def spmv_sketch(row_ptr, col_idx, val, u, s, zeta, seed, scale=1.0, U=None):
    """One fused inner-step kernel: (w = scale A u, S w, <w, U[:, l]>, ||w||^2)."""
    A = _csr(row_ptr, col_idx, val)
    dev = u.device
    w = torch.empty(A.n, dtype=torch.float64, device=dev)
    c = torch.empty(s, dtype=torch.float64, device=dev)
    nrm = torch.empty(1, dtype=torch.float64, device=dev)
    nwin = 0 if U is None else U.shape[1]
    dots = torch.empty(max(nwin, 1), dtype=torch.float64, device=dev)
    Ucm = None
    if U is not None:
        Ucm = U.t().contiguous()  # column-major storage: column l contiguous
    need = C.c_size_t()
    _check(L.load().sfgmres_spmv_workspace_bytes(A.n, A.nnz, s, zeta, C.byref(need)), None)
    ws = _workspace(need.value, dev, "spmv")
    h = _handle(dev)
    _check(L.load().sfgmres_spmv_sketch(h, C.byref(A), u.contiguous().data_ptr(), scale,
                                        w.data_ptr(), s, zeta, seed & (2**64 - 1), _ptr(Ucm),
                                        A.n, nwin, c.data_ptr(), dots.data_ptr(), nrm.data_ptr(),
                                        ws.data_ptr(), ws.numel(), _stream()), h)
    return w, c, dots[:nwin], nrm[0]
