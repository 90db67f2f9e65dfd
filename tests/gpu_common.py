"""Shared helpers of the GPU parity tests (inputs to device, oracle calls)."""
import numpy as np
import pytest
import torch

import workloads as W

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def dev():
    return torch.device("cuda:0")


def to_dev(A: W.CSR):
    d = dev()
    return (torch.from_numpy(A.row_ptr).to(d), torch.from_numpy(A.col_idx).to(d),
            torch.from_numpy(A.val).to(d))


def tvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev())


def ragged_powerlaw(n, seed, Lmax=256, mean=32):
    return W.powerlaw_random(n, np.random.default_rng(seed), Lmin=4, Lmax=Lmax, mean=mean)


def with_long_and_empty_rows(n, seed):
    """Random pattern with one row longer than the LDS tile and some empty rows."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        if i % 17 == 5:
            continue                       # empty row
        L = 6000 if i == n // 2 else int(rng.integers(1, 12))
        c = rng.choice(n, size=min(L, n), replace=False)
        rows.append(np.full(c.shape[0], i))
        cols.append(c)
        vals.append(rng.integers(-5, 6, size=c.shape[0]).astype(np.float64))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    return W.CSR(n, rp.astype(np.int32), c.astype(np.int32), v)


def hist_close(gpu, ref, rtol=1e-9, atol=1e-14):
    """Residual histories (relative to ||b||): |g - r| <= rtol r + atol.

    The floor atol covers the rounding of the minimised residual itself:
    |g_{j+1}| is formed from ||b|| e_1 by j rotations, so its absolute error
    is a modest multiple of u ||b|| whatever its size."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (g.shape, r.shape)
    bad = np.abs(g - r) > rtol * np.abs(r) + atol
    assert not bad.any(), (np.nonzero(bad)[0], g[bad], r[bad])
