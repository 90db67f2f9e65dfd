"""Benchmark: time to a 1e-8 relative residual of the sketched-FGMRES solver
on one MI355X, forward plus adjoint, FP64 against mixed precision, with the
fused SpMV+sketch kernel's HBM roofline fraction.

Workload (the default, the largest single-GPU configuration): 3D
convection-diffusion on a 256^3 grid (n = 16,777,216, nnz = 117,047,296, CSR
FP64, 7-point first-order upwind stencil, nodal diffusion log-uniform in
[0.1, 10] with harmonic face means, convection (50, 50, 50)), b uniform in
[-1, 1) from a fixed seed, x0 = 0; inner sGMRES m = 200, Arnoldi window t = 2,
sparse sign sketch s = 800, zeta = 8; FGMRES to tol 1e-8.  The adjoint solves
A^T lambda = g for g = dL/dx of L = ||x - x_target||^2 (x_target uniform in
[0, 1)) and forms dL/dA on A's pattern.

One step = one FP64 forward solve plus one FP64 adjoint solve (the CSR
transpose, the transposed solve and dL/dA), every step of the method on the
GPU (initial residual, inner cycles of fused SpMV+sketch+window dots, sketched
QR and decisions, truncated Arnoldi, z = B y, outer SpMV, Gram-Schmidt,
Givens, final iterate and its true residual).  Inputs are resident in HBM
before the timed region.  The same forward+adjoint in mixed precision (FP32
inner SpMV, sketch input and basis; FP64 sketch accumulation, QR and outer
loop) is timed after it and reported with its speedup and its errors against
the FP64 solution and adjoint.

Output: one JSON line.  ``roofline`` is for the FP64 fused inner
SpMV+sketch kernel of the forward solve: algorithmic bytes per launch,
12 nnz + 20 n + 8 n nwin (values and column indices, row pointers, the input
vector, the output vector, and the nwin Arnoldi window vectors its fused dot
products read; the sketch S counts 0 bytes, since it is defined by a counter
-based generator: the packed copy the kernel reads, 12 n bytes, is reported
separately as implementation traffic), divided by the kernel's mean duration
measured with HIP events on the library's stream over the timed solves
(every 7th inner step's launch, the events recorded by the launch itself at
the kernel's start and end).  ``cpu_baseline`` times the CPU oracle on a
bounded prefix of the same forward solve (the sketch generation and the
first outer step with a forced short inner cycle) and extrapolates it per
inner step to the GPU run's forward and adjoint inner steps.  ``secondary``
holds the 128^3 constant-coefficient system (whose matrix largely fits the
chip's 256 MB last-level cache, so its rate is not an HBM figure) and the 1M
power-law system, each against the 60% target.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X published HBM3E bandwidth
TARGET_FRAC = 0.60      # the fused kernel's target fraction of HBM peak
# HBM bytes per dispatch of the headline fused kernel (FP64, 256^3 system,
# matrix by diagonal, sketch columns generated in the kernel) from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB), each scaled by the factor measured on a
# plain device copy of known size (bench.py --copy-calibration): FETCH_SIZE
# x 2.0 (1605.1 MB, equal to the 128-byte read requests counted directly) +
# WRITE_SIZE x 1.0 (135.8 MB), averaged over the 6058 working dispatches of
# one FP64 forward and adjoint solve.  Valid only for the kernel source it
# was measured on; None whenever that kernel changes.
PMC_TRAFFIC_BYTES = 1740.9e6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 128^3 and power-law rows of the benchmark line")
    ap.add_argument("--matrix-format", default=None, choices=["auto", "csr"],
                    help="the inner SpMV's storage of A (--info runs; default auto)")
    ap.add_argument("--workload", type=int, default=5, choices=[1, 2, 3, 4, 5],
                    help="5 = the benchmark line (256^3, forward + adjoint, FP64 vs mixed); "
                         "2 = 128^3, 3 = 1M power-law, 4 = 512^2 parameterised operator: "
                         "informational timings of the other workloads")
    ap.add_argument("--info", action="store_true",
                    help="informational timings of --workload (any of them) instead of the "
                         "benchmark line")
    ap.add_argument("--m", type=int, default=None, help="override the workload's inner cap k_max")
    ap.add_argument("--t", type=int, default=None, help="override the Arnoldi window")
    ap.add_argument("--s", type=int, default=None, help="override the sketch rows")
    ap.add_argument("--zeta", type=int, default=None, help="override the sketch nonzeros per column")
    ap.add_argument("--precisions", default=None, help="comma list of fp64,mixed (other workloads)")
    ap.add_argument("--cond-threshold", type=float, default=None,
                    help="override the C2 condition threshold (other workloads)")
    ap.add_argument("--outer", default=None, choices=["fgmres", "restarted"],
                    help="outer iteration (other workloads): FGMRES or restarted sGMRES")
    ap.add_argument("--precond", default=None, choices=["none", "ilu0"],
                    help="other workloads: zero-fill ILU right preconditioning")
    ap.add_argument("--mid-outer", type=int, default=None,
                    help="other workloads: two-level FGMRES with lower-level solves of at most N steps")
    ap.add_argument("--adjoint", action="store_true",
                    help="workloads 4 and 5: time the adjoint solve also when --precisions is given")
    ap.add_argument("--phases", action="store_true",
                    help="other workloads: report the solver's per-phase GPU times")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (counter calibration) and exit")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8}), flush=True)


def stream_rates(mib: int = 1024, reps: int = 10):
    """Measured reference rates of this GPU (GB/s): a plain device copy of
    MIB MiB (bytes read + bytes written per second) and a read-only
    reduction of the same buffer (torch's sum; bytes read per second), each
    the best of `reps` runs timed with events on torch's stream."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.rand(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        t = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1) * 1e-3)
        return min(t)
    copy = 2 * n * 8 / best(lambda: y.copy_(x)) / 1e9
    read = n * 8 / best(lambda: x.sum()) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return copy, read


# Time the fused kernel on every 7th inner step (an event-carrying launch
# costs ~10 us of dispatch).  7 is co-prime with the 8 steps of a decision
# panel, so the timed launches cover every position in a panel: the launches
# at a panel's start run beside the decision kernel and take ~5% longer.
PROFILE_STRIDE = 7


def window_sum(inner_k, stop_reason, t, m, panel=8, stride=PROFILE_STRIDE):
    """Sum of the window size min(t, i+1) over the timed working fused launches.

    A cycle runs its inner steps in panels of `panel` steps and decides after
    every column of a panel, so the steps up to the end of the panel holding
    the stopping column (C2 decides one column past k) all do work; the
    library times steps stride-1, 2 stride-1, ... of them."""
    tot = 0
    launches = 0
    for k, r in zip(inner_k, stop_reason):
        decided = int(k) + (1 if r == "C2" else 0)
        steps = min(m, -(-decided // panel) * panel)
        timed = range(stride - 1, steps, stride)
        launches += len(timed)
        tot += sum(min(t, i + 1) for i in timed)
    return tot, launches


def fused_rate(infos, A, t, m, zeta, fp32):
    """Mean duration of the timed working fused launches, their algorithmic
    bytes (matrix values and indices, row pointers, input, output and the
    window vectors of the fused dots; S counts 0 bytes) and the bytes of the
    packed sketch the kernel also reads (implementation traffic; 0 when it
    generates the columns of S itself)."""
    launches = sum(i["spmv_launches"] for i in infos)
    ms = sum(i["spmv_ms"] for i in infos)
    win, wl = 0, 0
    for i in infos:
        a_, b_ = window_sum(i["inner_k"], i["stop_reason"], t, m)
        win += a_
        wl += b_
    if wl != launches:
        raise RuntimeError(f"timed launch count mismatch {wl} vs {launches}")
    vb = 4 if fp32 else 8
    zg = (zeta + 7) // 8  # packed sketch: groups of 12 bytes per column
    alg = (vb + 4) * A.nnz + (4 + 2 * vb) * A.n + vb * A.n * (win / launches)
    sk = 0 if infos[-1].get("sketch_generated") else 12 * zg * A.n
    avg = ms * 1e-3 / launches
    return avg, alg, sk, launches


def kernel_label(info, fp32, nw):
    """The fused inner SpMV instance a solve used, by its template
    parameters (value type, sketch groups, mode, window, operand storage)."""
    dia, gen = info.get("dia_diagonals", 0) > 0, info.get("sketch_generated", False)
    stream = info.get("matrix_streamed", False)
    ld = (("kLdDiaGen" if gen else "kLdDia") if dia else
          "kLdStream" if stream else ("kLdGen" if gen else "kLdCached"))
    what = (("matrix by diagonal" if dia else "CSR, streaming loads" if stream else "CSR")
            + (", sketch columns generated in the kernel" if gen else ", packed sketch"))
    return f"k_spmv<{'float' if fp32 else 'double'}, 1, kModeInner, {nw}, {ld}> ({what})"


def own_bytes(infos, A, t, m, fp32):
    """Bytes the inner SpMV reads and writes in the storage it used: the
    CSR formula, or with the matrix by diagonal (nd diagonals of n values,
    padding included, no row pointers or column indices) nd w n + 2 w n +
    w nwin n; the packed sketch not included."""
    nd = infos[-1].get("dia_diagonals", 0)
    launches = sum(i["spmv_launches"] for i in infos)
    win = sum(window_sum(i["inner_k"], i["stop_reason"], t, m)[0] for i in infos)
    vb = 4 if fp32 else 8
    if nd == 0:
        return (vb + 4) * A.nnz + (4 + 2 * vb) * A.n + vb * A.n * (win / launches), 0
    return vb * nd * A.n + 2 * vb * A.n + vb * A.n * (win / launches), nd


def other_workload(args):
    """Solve times of one of the other workloads (not the benchmark line)."""
    import torch
    import paper_2506_18408_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    t0 = time.time()
    A, b, p = W.make_workload(args.workload)
    log(f"workload {p['name']}: n={A.n} nnz={A.nnz} generated in {time.time() - t0:.1f}s")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    bt = torch.from_numpy(b).to(dev)
    for k in ("m", "t", "s", "zeta"):
        if getattr(args, k) is not None:
            p[k] = getattr(args, k)
    m, t, zeta = p["m"], p["t"], p["zeta"]
    precs = ["mixed"] if args.workload == 5 else ["fp64", "mixed"]
    if args.precisions:
        precs = args.precisions.split(",")
    adjoint = args.workload in (4, 5) and (args.precisions is None or args.adjoint)
    out = {"metric": "time-to-1e-8 rel. residual (s) per solve", "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
           "data": "synthetic",
           "config": {"workload": p["name"], "n": A.n, "nnz": A.nnz, "m": m, "t": t, "s": p["s"],
                      "zeta": zeta, "tol": p["tol"]}}
    for prec in precs:
        prm = P.SolveParams(m=m, t=t, s=p["s"], zeta=zeta, tol=p["tol"], seed=p["seed"],
                            max_outer=p["max_outer"], precision=prec)
        if args.cond_threshold is not None:
            prm.cond_threshold = args.cond_threshold
        if args.outer is not None:
            prm.outer = args.outer
        if args.precond is not None:
            prm.precond = args.precond
        if args.mid_outer is not None:
            prm.mid_outer = args.mid_outer
        if args.matrix_format is not None:
            prm.matrix_format = args.matrix_format
        x = torch.empty_like(bt)
        for _ in range(args.warmup):
            P.solve(rp, ci, va, bt, params=prm, out=x)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        infos = [P.solve(rp, ci, va, bt, params=prm, out=x, profile=PROFILE_STRIDE)[1]
                 for _ in range(args.steps)]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - ts) / args.steps
        inf = infos[-1]
        rec = {"time_to_tol_s": sec, "converged": bool(inf["converged"]),
               "residual_history": [float(v) for v in inf["residual_history"]],
               "true_rel_residual": inf["true_rel_residual"], "outer_iters": inf["outer_iters"],
               "total_inner": inf["total_inner"]}
        avg, alg = float("nan"), float("nan")
        if sum(i["spmv_launches"] for i in infos) > 0:   # (none timed with two levels)
            avg, alg, sk, _ = fused_rate(infos, A, t, m, zeta, prec == "mixed")
            rec.update({"spmv_mean_launch_us": avg * 1e6, "spmv_alg_bytes_per_launch": alg,
                        "packed_sketch_bytes": sk, "spmv_alg_gbs": alg / avg / 1e9,
                        "frac": alg / avg / 1e9 / HBM_PEAK_GBS})
        if args.phases:
            _, ph = P.solve(rp, ci, va, bt, params=prm, out=x, phase_timers=True)
            rec["phase_ms"] = ph["phase_ms"]
            log(f"{prec} phases (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in ph["phase_ms"].items()))
        log(f"{prec}: {sec * 1e3:.2f} ms/solve outer={inf['outer_iters']} "
            f"inner={inf['total_inner']} true_rel_res={inf['true_rel_residual']:.3e} "
            f"fused {avg * 1e6:.1f} us ({alg / avg / 1e9:.0f} GB/s, "
            f"{alg / avg / 1e9 / HBM_PEAK_GBS:.2f} of peak)")
        if adjoint:
            g = 2.0 * (x - bt)  # any right-hand side of the adjoint solve
            for _ in range(args.warmup):
                P.solve_adjoint(rp, ci, va, g, x, params=prm)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(args.steps):
                _, _, ia = P.solve_adjoint(rp, ci, va, g, x, params=prm)
            torch.cuda.synchronize()
            asec = (time.perf_counter() - ts) / args.steps
            rec["adjoint_time_s"] = asec
            rec["adjoint_outer_iters"] = ia["outer_iters"]
            rec["adjoint_converged"] = bool(ia["converged"])
            log(f"{prec} adjoint (transpose + solve + dL/dA): {asec * 1e3:.2f} ms "
                f"outer={ia['outer_iters']}")
        out[prec] = rec
    out["value"] = out[precs[0]]["time_to_tol_s"]
    out["dtype"] = "f64" if precs[0] == "fp64" else "f32+f64"
    print(json.dumps(out), flush=True)


def timed_solves(P, rp, ci, va, bt, prm, steps, warmup, adjoint=None, label=""):
    """Warm-up and timed solves (forward, then the adjoint when `adjoint` =
    (g, x_for_gradient) or "auto" with g = 2 (x - x_target)); returns the
    mean seconds per step, the forward infos, the last x, the adjoint infos
    and the last lambda."""
    import torch
    x = torch.empty_like(bt)

    def one(timed):
        _, inf = P.solve(rp, ci, va, bt, params=prm, out=x,
                         profile=PROFILE_STRIDE if timed else 0)
        ia, lam = None, None
        if adjoint is not None:
            g = adjoint(x)
            lam, _, ia = P.solve_adjoint(rp, ci, va, g, x, params=prm)
        return inf, ia, lam

    for w in range(warmup):
        t0 = time.perf_counter()
        inf, ia, _ = one(False)
        torch.cuda.synchronize()
        log(f"{label} warmup {w}: {time.perf_counter() - t0:.3f} s outer={inf['outer_iters']} "
            f"inner={inf['total_inner']}" + (f" adjoint outer={ia['outer_iters']}" if ia else ""))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, ainfos, lam = [], [], None
    for k in range(steps):
        inf, ia, lam = one(True)
        infos.append(inf)
        if ia is not None:
            ainfos.append(ia)
        if k == 0 or (k + 1) % 5 == 0:
            torch.cuda.synchronize()
            log(f"{label} step {k + 1}/{steps}: {time.perf_counter() - t0:.2f} s so far")
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    return sec, infos, x, ainfos, lam


def secondary_row(P, W, torch, cfg, steps, cpu=False):
    """FP64 and mixed solves of the 128^3 (cfg 2) or power-law (cfg 3)
    system: time to tol and the fused kernel's rate against the target;
    with cpu, also the oracle's whole FP64 solve of the same system (one
    thread, not extrapolated)."""
    dev = torch.device("cuda:0")
    A, b, p = W.make_workload(cfg)
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    bt = torch.from_numpy(b).to(dev)
    row = {"workload": p["name"], "n": A.n, "nnz": A.nnz, "m": p["m"], "t": p["t"], "s": p["s"],
           "zeta": p["zeta"]}
    for prec in ("fp64", "mixed"):
        prm = P.SolveParams(m=p["m"], t=p["t"], s=p["s"], zeta=p["zeta"], tol=p["tol"],
                            seed=p["seed"], max_outer=p["max_outer"], precision=prec)
        sec, infos, _, _, _ = timed_solves(P, rp, ci, va, bt, prm, steps, 1, label=p["name"] + " " + prec)
        avg, alg, sk, nl = fused_rate(infos, A, p["t"], p["m"], p["zeta"], prec == "mixed")
        own, nd = own_bytes(infos, A, p["t"], p["m"], prec == "mixed")
        inf = infos[-1]
        row[prec] = {"time_to_tol_s": sec, "converged": bool(inf["converged"]),
                     "true_rel_residual": inf["true_rel_residual"],
                     "outer_iters": inf["outer_iters"], "total_inner": inf["total_inner"],
                     "fused_mean_launch_us": avg * 1e6, "fused_alg_bytes": alg,
                     "fused_alg_gbs": alg / avg / 1e9, "frac": alg / avg / 1e9 / HBM_PEAK_GBS,
                     "own_storage_bytes": own, "diagonals": nd,
                     "frac_on_own_storage_bytes": own / avg / 1e9 / HBM_PEAK_GBS,
                     "target_frac": TARGET_FRAC, "packed_sketch_bytes": sk,
                     "kernel": kernel_label(inf, prec == "mixed", p["t"])}
        log(f"{p['name']} {prec}: {sec * 1e3:.2f} ms, fused {avg * 1e6:.1f} us "
            f"({alg / avg / 1e9:.0f} GB/s, {alg / avg / 1e9 / HBM_PEAK_GBS:.2f} of peak)")
    if cfg == 2:
        row["note"] = ("the matrix (175 MB) largely fits the 256 MB last-level cache: "
                       "the rate is not an HBM figure")
    if cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        As = A.to_scipy()
        with threadpool_limits(1):
            t0 = time.perf_counter()
            r = oracle.sfgmres(As, b, m=p["m"], t=p["t"], s=p["s"], zeta=p["zeta"], tol=p["tol"],
                               seed=p["seed"], max_outer=p["max_outer"], record_true_residual=False)
            tc = time.perf_counter() - t0
        row["cpu_oracle_fp64"] = {"value": tc, "unit": "s", "cores": 1, "kind": "oracle",
                                  "sample": f"the whole FP64 solve to {p['tol']:g} ({r.outer_iters} "
                                            f"outer / {sum(r.inner_k)} inner steps), not extrapolated"}
        log(f"{p['name']} cpu oracle: {tc:.1f} s for the whole FP64 solve")
    return row


def headline(args):
    import torch
    import paper_2506_18408_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    log("generating the 256^3 variable-coefficient system ...")
    t0 = time.time()
    A, b, p = W.make_workload(5)
    x_target = np.random.default_rng([5, 3]).uniform(0.0, 1.0, size=A.n)
    log(f"workload {p['name']}: n={A.n} nnz={A.nnz} generated in {time.time() - t0:.1f}s")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    bt = torch.from_numpy(b).to(dev)
    xt = torch.from_numpy(x_target).to(dev)
    m, t, s, zeta, tol = p["m"], p["t"], p["s"], p["zeta"], p["tol"]
    prm = P.SolveParams(m=m, t=t, s=s, zeta=zeta, tol=tol, seed=p["seed"],
                        max_outer=p["max_outer"])
    grad_of = lambda x: 2.0 * (x - xt)  # noqa: E731  (dL/dx of ||x - x_target||^2)
    torch.cuda.synchronize()
    copy_gbs, read_gbs = stream_rates()
    log(f"reference rates: device copy {copy_gbs:.0f} GB/s, read-only sum {read_gbs:.0f} GB/s")

    sec, infos, x, ainfos, lam = timed_solves(P, rp, ci, va, bt, prm, args.steps, args.warmup,
                                              adjoint=grad_of, label="fp64")
    last, alast = infos[-1], ainfos[-1]
    fwd_s = sum(i["solve_ms"] for i in infos) * 1e-3 / len(infos)
    adj_s = sec - fwd_s
    log(f"fp64: {sec:.3f} s per forward+adjoint (forward {fwd_s:.3f} s), outer={last['outer_iters']} "
        f"inner={last['total_inner']} true_rel_res={last['true_rel_residual']:.3e}; adjoint "
        f"outer={alast['outer_iters']} true_rel_res={alast['true_rel_residual']:.3e}")
    for inf, what in ((last, "forward"), (alast, "adjoint")):
        if not inf["converged"] or not inf["true_rel_residual"] <= tol * (1 + 1e-6):
            raise RuntimeError(f"FP64 {what} solve did not reach tol: {inf['true_rel_residual']}")

    avg_s, alg, sk, launches = fused_rate(infos, A, t, m, zeta, False)
    own, nd = own_bytes(infos, A, t, m, False)
    achieved = alg / avg_s / 1e9
    log(f"fused spmv+sketch (FP64): {launches} timed launches, mean {avg_s * 1e6:.2f} us, "
        f"{alg / 1e6:.1f} MB algorithmic (+{sk / 1e6:.1f} MB packed sketch) -> {achieved:.0f} GB/s")

    result = {
        "metric": "time-to-1e-8 rel. residual (s) + SpMV/sketch HBM GB/s vs peak, FP64 vs mixed",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"varcoef_convdiff3d_256^3 7-point upwind, n={A.n}, nnz={A.nnz}, "
                                f"kappa log-uniform [0.1,10], conv (50,50,50), b~U[-1,1); "
                                f"sGMRES m={m} t={t} s={s} zeta={zeta}; FGMRES tol {tol:g}; "
                                f"one step = FP64 forward + adjoint (A^T solve, dL/dA)"),
                   "n": A.n, "nnz": A.nnz,
                   "forward": {"time_s": fwd_s, "outer_iters": last["outer_iters"],
                               "total_inner": last["total_inner"],
                               "true_rel_residual": last["true_rel_residual"]},
                   "adjoint": {"time_s": adj_s, "outer_iters": alast["outer_iters"],
                               "total_inner": alast["total_inner"],
                               "true_rel_residual": alast["true_rel_residual"]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": PMC_TRAFFIC_BYTES,
                     "target_frac": TARGET_FRAC,
                     "kernel": kernel_label(last, False, 2) + ": fused SpMV + sketch + window "
                               "dots, FP64, forward solve",
                     "bytes_per_launch": alg, "packed_sketch_bytes_per_launch": sk,
                     "own_storage_bytes_per_launch": own, "diagonals": nd,
                     "frac_on_own_storage_bytes": own / avg_s / 1e9 / HBM_PEAK_GBS,
                     "mean_launch_us": avg_s * 1e6, "launches": launches,
                     "measured_copy_gbs": copy_gbs, "measured_read_gbs": read_gbs,
                     "own_storage_rate_of_measured_read": own / avg_s / 1e9 / read_gbs},
    }

    if not args.no_mixed:
        pm = P.SolveParams(**{**prm.__dict__, "precision": "mixed"})
        reps = max(1, min(args.steps, 3))
        msec, minfos, xm, mainfos, lamm = timed_solves(P, rp, ci, va, bt, pm, reps, 1,
                                                       adjoint=grad_of, label="mixed")
        im, iam = minfos[-1], mainfos[-1]
        err = (torch.linalg.norm(xm - x) / torch.linalg.norm(x)).item()
        # (the mixed adjoint's right-hand side is formed from the mixed x)
        lerr = (torch.linalg.norm(lamm - lam) / torch.linalg.norm(lam)).item()
        mavg, malg, msk, ml = fused_rate(minfos, A, t, m, zeta, True)
        mown, _ = own_bytes(minfos, A, t, m, True)
        mfwd = sum(i["solve_ms"] for i in minfos) * 1e-3 / len(minfos)
        result["mixed"] = {
            "time_to_tol_s": msec, "forward_time_s": mfwd, "adjoint_time_s": msec - mfwd,
            "speedup_vs_fp64": sec / msec,
            "forward_speedup_vs_fp64": fwd_s / mfwd,
            "converged": bool(im["converged"] and iam["converged"]),
            "true_rel_residual": im["true_rel_residual"],
            "adjoint_true_rel_residual": iam["true_rel_residual"],
            "outer_iters": im["outer_iters"], "total_inner": im["total_inner"],
            "adjoint_outer_iters": iam["outer_iters"],
            "rel_error_vs_fp64_solution": err, "rel_error_vs_fp64_adjoint": lerr,
            "fused_mean_launch_us": mavg * 1e6, "fused_alg_bytes": malg,
            "fused_alg_gbs": malg / mavg / 1e9, "frac": malg / mavg / 1e9 / HBM_PEAK_GBS,
            "own_storage_bytes": mown, "frac_on_own_storage_bytes": mown / mavg / 1e9 / HBM_PEAK_GBS,
            "packed_sketch_bytes": msk,
            "kernel": kernel_label(im, True, 2),
        }
        log(f"mixed: {msec:.3f} s per forward+adjoint (x{sec / msec:.2f}), outer={im['outer_iters']} "
            f"inner={im['total_inner']} true_rel_res={im['true_rel_residual']:.3e} err={err:.2e} "
            f"adjoint err={lerr:.2e}; fused {mavg * 1e6:.1f} us ({malg / mavg / 1e9:.0f} GB/s)")

    if not args.no_secondary:
        reps = max(1, min(args.steps, 3))
        result["secondary"] = [secondary_row(P, W, torch, 2, reps, cpu=not args.no_cpu),
                               secondary_row(P, W, torch, 3, reps)]

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(A, b, p, last["total_inner"] + alast["total_inner"])

    print(json.dumps(result), flush=True)


def cpu_baseline(A, b, p, total_inner):
    """The oracle on a bounded prefix of the forward solve, one BLAS thread:
    the sketch generation, then one outer step with a forced inner cycle of
    K steps; the per-inner-step time is extrapolated to the GPU run's inner
    steps (forward and adjoint), plus one sketch generation per solve."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    K = 4
    As = A.to_scipy()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        S = oracle.sketch_matrix(A.n, p["s"], p["zeta"], p["seed"])
        t_sketch = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.sfgmres(As, b, m=p["m"], t=p["t"], s=p["s"], zeta=p["zeta"], tol=p["tol"],
                       seed=p["seed"], max_outer=1, forced_k=[K], record_true_residual=False,
                       sketch=lambda w: oracle.apply_sketch(S, w))
        t_step = time.perf_counter() - t0
    per_inner = t_step / K
    value = 2 * t_sketch + per_inner * total_inner
    blas = [d.get("num_threads") for d in threadpool_info()]
    log(f"cpu oracle: sketch {t_sketch:.1f}s, first outer step with k={K} {t_step:.1f}s -> "
        f"extrapolated {value:.0f}s")
    return {"value": value, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"256^3 system, same seed: the oracle's sketch generation ({t_sketch:.1f}s) "
                       f"and its first outer FGMRES step with a forced inner cycle of k={K} "
                       f"({t_step:.1f}s), one thread (scipy SpMV and numpy sketch are single-"
                       f"threaded; BLAS limited to 1); value = 2 sketch generations + the time per "
                       f"inner step x the GPU run's {total_inner} forward+adjoint inner steps "
                       f"(extrapolated)"),
            "host_cpu_count": os.cpu_count(), "blas_threads_default": blas}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no "
              "multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.info or args.workload != 5 or any(getattr(args, k) is not None for k in
                                              ("m", "t", "s", "zeta", "cond_threshold", "outer",
                                               "precisions", "precond", "mid_outer")):
        other_workload(args)
        return
    headline(args)


if __name__ == "__main__":
    main()
