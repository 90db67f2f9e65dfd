"""The allocation-free entry point sfgmres_spmv_sketch_noalloc against the
workspace entry point sfgmres_spmv_sketch: the same kernels on a static
per-GPU scratch, so every output must agree bit for bit, on two calls in a
row (the second with a smaller input, over the first call's leftovers), and
a problem beyond the scratch is rejected before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2506_18408_amd as P
import paper_2506_18408_amd._lib as L
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec, ragged_powerlaw

pytestmark = [pytest.mark.gpu, requires_gpu]


def _noalloc(A, u, s, zeta, seed, scale=1.0, U=None):
    lib = L.load()
    rp, ci, va = to_dev(A)
    Acsr = L.Csr(A.n, A.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    dev = rp.device
    w = torch.full((A.n,), float("nan"), dtype=torch.float64, device=dev)
    c = torch.full((s,), float("nan"), dtype=torch.float64, device=dev)
    nrm = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    nwin = 0 if U is None else U.shape[1]
    dots = torch.full((max(nwin, 1),), float("nan"), dtype=torch.float64, device=dev)
    Ucm = None if U is None else U.t().contiguous()
    h = P.api._handle(dev)
    rc = lib.sfgmres_spmv_sketch_noalloc(h, C.byref(Acsr), u.data_ptr(), scale, w.data_ptr(), s,
                                         zeta, seed, None if Ucm is None else Ucm.data_ptr(),
                                         A.n, nwin, c.data_ptr(), dots.data_ptr(), nrm.data_ptr(),
                                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc, lib.sfgmres_last_error(h).decode(), (w, c, dots[:nwin], nrm[0])


def _check_pair(A, s, zeta, seed, nwin, rng):
    u = tvec(rng.standard_normal(A.n))
    U = tvec(rng.standard_normal((A.n, nwin))) if nwin else None
    ref = P.api.spmv_sketch(*to_dev(A), u, s, zeta, seed, scale=0.75, U=U)
    rc, msg, out = _noalloc(A, u, s, zeta, seed, scale=0.75, U=U)
    assert rc == L.OK, msg
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


def test_noalloc_matches_the_workspace_entry_point_twice():
    rng = np.random.default_rng(12)
    big = W.convdiff3d(48)                       # 110,592 rows, short-row tiles
    _check_pair(big, 400, 8, 1002, 2, rng)
    small = ragged_powerlaw(3000, 4)             # fewer rows, long rows, other sketch
    _check_pair(small, 120, 5, 77, 4, rng)


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    need = C.c_size_t()
    assert L.load().sfgmres_noalloc_scratch_bytes(C.byref(need)) == L.OK
    n = 6_000_000                                 # packed sketch alone: 72 MB
    A = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    ws = C.c_size_t()
    assert L.load().sfgmres_spmv_workspace_bytes(n, n, 400, 8, C.byref(ws)) == L.OK
    assert ws.value > need.value
    u = torch.ones(n, dtype=torch.float64, device="cuda:0")
    rc, msg, out = _noalloc(A, u, 400, 8, 1)
    assert rc == L.ERR_WORKSPACE and "scratch" in msg
    assert torch.isnan(out[0]).all()              # nothing launched
