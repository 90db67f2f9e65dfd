"""GPU tests of the fused inner SpMV's two sources for the columns of the
sparse sign sketch S (Section 3): the packed table built at the start of a
solve, and the columns generated inside the kernel from the same
Philox4x32-10 counters and Floyd's sampling.  Both give the same S, and the
row-to-lane assignment of the scatter does not change, so whole solves must
agree bit for bit; the table path itself is checked against the oracle by
the other solve tests."""
import numpy as np
import pytest

import oracle
import paper_2506_18408_amd as P
import workloads as W
from tests.gpu_common import requires_gpu, to_dev, tvec

pytestmark = [pytest.mark.gpu, requires_gpu]


def _system(name):
    if name == "varcoef3d_16":
        A = W.convdiff3d_varcoef(16, np.random.default_rng([21, 0]))
    elif name == "convdiff2d_64":
        A = W.convdiff2d(64, 1.0, (10.0, 10.0))
    else:  # long rows (4..256 nonzeros): the generated sketch with cached loads
        A = W.powerlaw_random(5000, np.random.default_rng([22, 0]))
    b = np.random.default_rng([23, 1]).uniform(-1.0, 1.0, A.n)
    return A, b


@pytest.mark.parametrize("zeta", [1, 3, 8])
@pytest.mark.parametrize("t", [0, 2, 5])
@pytest.mark.parametrize("name", ["varcoef3d_16", "convdiff2d_64", "powerlaw_5000"])
def test_generated_columns_match_the_table_bit_for_bit(name, t, zeta):
    A, b = _system(name)
    rp, ci, va = to_dev(A)
    prm = dict(m=30, t=t, s=90, zeta=zeta, tol=1e-10, seed=11, max_outer=12)
    out = {}
    for src in ("table", "gen"):
        x, info = P.solve(rp, ci, va, tvec(b), sketch_source=src, **prm)
        out[src] = (x.cpu().numpy(), info)
    (xt, it), (xg, ig) = out["table"], out["gen"]
    assert not it["sketch_generated"] and ig["sketch_generated"]
    assert list(it["inner_k"]) == list(ig["inner_k"])
    assert list(it["stop_reason"]) == list(ig["stop_reason"])
    assert np.array_equal(np.asarray(it["residual_history"]), np.asarray(ig["residual_history"]))
    assert np.array_equal(xt, xg)


def test_generated_columns_solve_matches_the_oracle():
    """One outer step with a forced inner dimension, generated columns,
    against the oracle's cycle (its sketch is the oracle's own Philox and
    Floyd code)."""
    A, b = _system("varcoef3d_16")
    rp, ci, va = to_dev(A)
    prm = dict(m=30, t=2, s=90, zeta=8, tol=1e-14, seed=11, max_outer=1)
    x, info = P.solve(rp, ci, va, tvec(b), sketch_source="gen", forced_k=[12], **prm)
    ref = oracle.sfgmres(A.to_scipy(), b, forced_k=[12], **prm)
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_generated_columns_need_fp64_and_zeta_at_most_8():
    A, b = _system("convdiff2d_64")
    rp, ci, va = to_dev(A)
    prm = dict(m=30, t=2, s=90, tol=1e-8, seed=11, max_outer=2)
    with pytest.raises(P.SFGMRESError, match="sketch_source"):
        P.solve(rp, ci, va, tvec(b), sketch_source="gen", zeta=9, **prm)
    with pytest.raises(P.SFGMRESError, match="sketch_source"):
        P.solve(rp, ci, va, tvec(b), sketch_source="gen", zeta=8, precision="mixed", **prm)
