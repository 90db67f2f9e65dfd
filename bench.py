"""Benchmark: time to a 1e-8 relative residual of the sketched-FGMRES solver
on one MI355X, with the fused SpMV+sketch kernel's HBM roofline fraction.

Workload (the default): 3D convection-diffusion, 7-point first-order upwind
stencil on a 128^3 grid (n = 2,097,152, nnz = 14,581,760, CSR FP64,
diffusion 1, convection (50, 50, 50)), b uniform in [-1, 1) from a fixed
seed, x0 = 0; inner sGMRES m = 100, Arnoldi window t = 2, sparse sign sketch
s = 400, zeta = 8; FGMRES to tol 1e-8 in FP64.

One step = one complete solve (every step of the method: initial residual,
inner cycles of fused SpMV+sketch+window dots, sketched QR and decisions,
truncated Arnoldi, z = B y, outer SpMV, Gram-Schmidt, Givens, final iterate
and its true residual).  Inputs are resident in HBM before the timed region.
The same solve in mixed precision (FP32 inner SpMV/sketch input/basis, FP64
sketch accumulation, QR, outer loop) is timed after it and reported with its
speedup and its solution error against the FP64 solution.

Output: one JSON line (rank 0).  ``roofline`` is for the fused inner
SpMV+sketch kernel: algorithmic bytes per launch,
12 nnz + 20 n + 8 n nwin + 12 ceil(zeta/8) n (values and column indices, row
pointers, the input vector, the output vector, the nwin Arnoldi window
vectors its fused dot products read, and the packed sketch columns),
divided by the kernel's mean duration measured with HIP events on the
library's stream over the timed solves (every 7th inner step's launch, the
events being recorded by the launch itself at the kernel's start and end).  ``cpu_baseline`` times the CPU
oracle on the first outer step of the same solve (k_1 inner steps, one
thread) and scales its per-inner-step time to the GPU run's total inner
steps.
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
# HBM bytes per dispatch of the fused kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB), each scaled by the factor measured on a plain device copy
# of known size (bench.py --copy-calibration): FETCH_SIZE x 2.0 + WRITE_SIZE x
# 1.0, averaged over the working dispatches of one FP64 solve.  Valid only for
# the kernel source it was measured on; None whenever that kernel changes.
PMC_TRAFFIC_BYTES = 269046574


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128, help="grid points per axis (128 = the benchmark workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3, 4, 5],
                    help="2 = the benchmark line (128^3); 3 = 1M power-law (FP64 and mixed), "
                         "4 = 512^2 parameterised operator and 5 = 256^3 variable coefficients "
                         "(forward and adjoint): informational timings of the other workloads")
    ap.add_argument("--m", type=int, default=None, help="override the workload's inner cap k_max")
    ap.add_argument("--t", type=int, default=None, help="override the Arnoldi window")
    ap.add_argument("--s", type=int, default=None, help="override the sketch rows")
    ap.add_argument("--zeta", type=int, default=None, help="override the sketch nonzeros per column")
    ap.add_argument("--precisions", default=None, help="comma list of fp64,mixed (other workloads)")
    ap.add_argument("--cond-threshold", type=float, default=None,
                    help="override the C2 condition threshold (other workloads)")
    ap.add_argument("--outer", default=None, choices=["fgmres", "restarted"],
                    help="outer iteration (other workloads): FGMRES or restarted sGMRES")
    ap.add_argument("--adjoint", action="store_true",
                    help="workloads 4 and 5: time the adjoint solve also when --precisions is given")
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
    """Mean duration of the timed working fused launches and their algorithmic
    bytes (matrix, row pointers, x, y, window, packed sketch)."""
    launches = sum(i["spmv_launches"] for i in infos)
    ms = sum(i["spmv_ms"] for i in infos)
    win = sum(window_sum(i["inner_k"], i["stop_reason"], t, m)[0] for i in infos)
    vb = 4 if fp32 else 8
    zg = (zeta + 7) // 8  # packed sketch: groups of 12 bytes per column
    nbytes = (vb + 4) * A.nnz + (4 + 2 * vb) * A.n + vb * A.n * (win / launches) + 12 * zg * A.n
    avg = ms * 1e-3 / launches
    return avg, nbytes


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
        avg, nbytes = fused_rate(infos, A, t, m, zeta, prec == "mixed")
        rec = {"time_to_tol_s": sec, "converged": bool(inf["converged"]),
               "residual_history": [float(v) for v in inf["residual_history"]],
               "true_rel_residual": inf["true_rel_residual"], "outer_iters": inf["outer_iters"],
               "total_inner": inf["total_inner"], "spmv_mean_launch_us": avg * 1e6,
               "spmv_bytes_per_launch": nbytes, "spmv_achieved_gbs": nbytes / avg / 1e9}
        log(f"{prec}: {sec * 1e3:.2f} ms/solve outer={inf['outer_iters']} "
            f"inner={inf['total_inner']} true_rel_res={inf['true_rel_residual']:.3e} "
            f"fused {avg * 1e6:.1f} us ({nbytes / avg / 1e9:.0f} GB/s)")
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no "
              "multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload != 2 or any(getattr(args, k) is not None
                                 for k in ("m", "t", "s", "zeta", "cond_threshold", "outer")):
        other_workload(args)
        return

    import torch
    import paper_2506_18408_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    t0 = time.time()
    N = args.grid
    A = W.convdiff3d(N, 1.0, (50.0, 50.0, 50.0))
    b = W.rhs(A.n, np.random.default_rng([2, 1]), "u11")
    seed = W.sketch_seed(2)
    m, t, s, zeta, tol = 100, 2, 400, 8, 1e-8
    log(f"workload convdiff3d N={N}: n={A.n} nnz={A.nnz} generated in {time.time() - t0:.1f}s")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    bt = torch.from_numpy(b).to(dev)
    prm = P.SolveParams(m=m, t=t, s=s, zeta=zeta, tol=tol, seed=seed, max_outer=100)
    x = torch.empty_like(bt)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        _, info = P.solve(rp, ci, va, bt, params=prm, out=x)
        log(f"warmup {w}: {info['solve_ms']:.1f} ms outer={info['outer_iters']} inner={info['total_inner']}")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    for k in range(args.steps):
        _, info = P.solve(rp, ci, va, bt, params=prm, out=x, profile=PROFILE_STRIDE)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sec = elapsed / args.steps
    last = infos[-1]
    log(f"fp64: {sec * 1e3:.2f} ms/solve, outer={last['outer_iters']} inner={last['total_inner']} "
        f"true_rel_res={last['true_rel_residual']:.3e}")
    if not last["converged"] or not last["true_rel_residual"] <= tol * (1 + 1e-6):
        raise RuntimeError(f"FP64 solve did not reach tol: {last['true_rel_residual']}")

    # fused SpMV+sketch kernel: mean duration of its working launches
    spmv_ms = sum(i["spmv_ms"] for i in infos)
    launches = sum(i["spmv_launches"] for i in infos)
    win = 0
    wl = 0
    for i in infos:
        a_, b_ = window_sum(i["inner_k"], i["stop_reason"], t, m)
        win += a_
        wl += b_
    if wl != launches:
        raise RuntimeError(f"launch count mismatch {wl} vs {launches}")
    avg_s = spmv_ms * 1e-3 / launches
    zg = (zeta + 7) // 8  # packed sketch: groups of 12 bytes per column
    bytes_per_launch = 12 * A.nnz + 20 * A.n + 8 * A.n * (win / launches) + 12 * zg * A.n
    achieved = bytes_per_launch / avg_s / 1e9
    log(f"fused spmv+sketch: {launches} launches, mean {avg_s * 1e6:.2f} us, "
        f"{bytes_per_launch / 1e6:.1f} MB algorithmic -> {achieved:.0f} GB/s")

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
        "config": {"workload": f"convdiff3d_{N}^3 7-point upwind, n={A.n}, nnz={A.nnz}, "
                               f"conv (50,50,50), b~U[-1,1); sGMRES m={m} t={t} s={s} zeta={zeta}; "
                               f"FGMRES tol {tol:g}, FP64",
                   "n": A.n, "nnz": A.nnz, "outer_iters": last["outer_iters"],
                   "total_inner": last["total_inner"],
                   "true_rel_residual": last["true_rel_residual"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": PMC_TRAFFIC_BYTES,
                     "kernel": "k_spmv<double, 1, kModeInner, 2, false> (fused SpMV+sketch+window dots; ZB = ceil(zeta/8) = 1, window 2)",
                     "bytes_per_launch": bytes_per_launch, "mean_launch_us": avg_s * 1e6,
                     "launches": launches},
    }

    if not args.no_mixed:
        pm = P.SolveParams(**{**prm.__dict__, "precision": "mixed"})
        xm = torch.empty_like(bt)
        _, im = P.solve(rp, ci, va, bt, params=pm, out=xm)   # warm-up (also builds the FP32 copy)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        reps = max(1, min(args.steps, 3))
        ims = []
        for _ in range(reps):
            _, im = P.solve(rp, ci, va, bt, params=pm, out=xm, profile=PROFILE_STRIDE)
            ims.append(im)
        torch.cuda.synchronize()
        msec = (time.perf_counter() - tm0) / reps
        err = (torch.linalg.norm(xm - x) / torch.linalg.norm(x)).item()
        ml = sum(i["spmv_launches"] for i in ims)
        mms = sum(i["spmv_ms"] for i in ims)
        mwin = sum(window_sum(i["inner_k"], i["stop_reason"], t, m)[0] for i in ims)
        mbytes = 8 * A.nnz + 12 * A.n + 4 * A.n * (mwin / ml) + 12 * zg * A.n
        mavg = mms * 1e-3 / ml
        result["mixed"] = {
            "time_to_tol_s": msec, "speedup_vs_fp64": sec / msec,
            "converged": bool(im["converged"]), "true_rel_residual": im["true_rel_residual"],
            "outer_iters": im["outer_iters"], "total_inner": im["total_inner"],
            "rel_error_vs_fp64_solution": err,
            "spmv_mean_launch_us": mavg * 1e6, "spmv_bytes_per_launch": mbytes,
            "spmv_achieved_gbs": mbytes / mavg / 1e9,
        }
        log(f"mixed: {msec * 1e3:.2f} ms/solve (x{sec / msec:.2f}), outer={im['outer_iters']} "
            f"inner={im['total_inner']} true_rel_res={im['true_rel_residual']:.3e} err={err:.2e}")

    if not args.no_cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        As = A.to_scipy()
        k1 = int(last["inner_k"][0])
        with threadpool_limits(1):
            tc = time.perf_counter()
            r = oracle.sfgmres(As, b, m=m, t=t, s=s, zeta=zeta, tol=tol, seed=seed, max_outer=1,
                               forced_k=[k1], record_true_residual=False)
            tcpu = time.perf_counter() - tc
        per_inner = tcpu / k1
        result["cpu_baseline"] = {
            "value": per_inner * last["total_inner"], "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"first outer FGMRES step of the same solve (k_1={k1} inner sGMRES steps + "
                       f"one outer step) timed at {tcpu:.1f}s on 1 thread; value = that time per "
                       f"inner step x the GPU run's {last['total_inner']} inner steps (extrapolated)"),
        }
        log(f"cpu oracle: {tcpu:.1f}s for k_1={k1} -> extrapolated {per_inner * last['total_inner']:.1f}s")
        del r

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
