"""Benchmark: CPR-FGMRES solve time to relres 1e-6 at 3.28M DOF, FP32 vs FP64 preconditioner.

One step = one cpr_solve (the whole solve phase: CPR apply with the pressure
V-cycle and the stage-2 sweep, outer products, Gram-Schmidt, Givens, true
residual, and the adaptive-setup decision) on the SPE10-sized synthetic
Jacobian (60x220x85 grid, 2.5% inactive cells, layered log-normal
permeability with sigma 2, kz/kx = 0.1), from x = 0, inputs resident in HBM.
SETUP runs before the timed region and is reported separately.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPR-FGMRES time to relres 1e-6 @3.28M DOF, FP32 vs FP64 precond; p50/p99 lat"
HBM_PEAK_GBS = 8000.0


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(shape_full, gpu_its, n_full):
    """Time the oracle (single thread) on a slab of the same workload and scale.

    The sample is the same generator with nz = 4 (about 51K active cells):
    oracle SETUP + FP64 CPR-FGMRES to 1e-6.  The reported value scales the
    oracle's solve time per iteration per cell to the full grid and to the
    GPU's FP64 iteration count.
    """
    from threadpoolctl import threadpool_limits

    import numpy as np

    from oracle import cpr as ocpr
    from oracle import fgmres as ofg
    from workloads import blackoil as bo

    shape = (shape_full[0], shape_full[1], 4)
    case = bo.case_spe10_like(seed=1100, shape=shape)
    b = bo.rhs(case.ndof, 1101)
    with threadpool_limits(limits=1):
        A = ocpr.Bsr.from_case(case)
        t0 = time.perf_counter()
        B = ocpr.setup(A)
        t1 = time.perf_counter()
        res = ofg.fgmres(lambda v: ocpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
        t2 = time.perf_counter()
    per_it_cell = (t2 - t1) / max(res.iterations, 1) / case.n_b
    est_ms = per_it_cell * n_full * gpu_its * 1e3
    return {
        "value": est_ms,
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle FP64 on the {shape[0]}x{shape[1]}x{shape[2]} slab of the same generator "
                   f"({case.n_b} cells): setup {t1 - t0:.1f} s, solve {t2 - t1:.1f} s, {res.iterations} its; "
                   f"value = solve time per iteration per cell x {n_full} cells x {gpu_its} GPU FP64 its"),
        "cpu": _cpu_name(),
        "os_cpu_count": os.cpu_count(),
    }


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shape", type=int, nargs=3, default=(60, 220, 85))
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solve of one Jacobian is not "
              "sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_01970_amd import Params, Solver
    from paper_2201_01970_amd import _capi as capi
    from workloads import blackoil as bo

    dev = torch.device("cuda:0")
    shape = tuple(args.shape)
    t0 = time.perf_counter()
    case = bo.case_spe10_like(seed=1100, shape=shape)
    b_np = bo.rhs(case.ndof, 1101)
    gen_s = time.perf_counter() - t0
    rp = torch.as_tensor(case.row_ptr, device=dev)
    col = torch.as_tensor(case.col, device=dev)
    vals = torch.as_tensor(case.vals.reshape(-1), device=dev)
    b = torch.as_tensor(b_np, device=dev)
    print(f"[bench] case {shape} n_b={case.n_b} nnz_b={case.nnz_b} dof={case.ndof} gen {gen_s:.1f}s",
          file=sys.stderr, flush=True)

    def run(fp32, steps, warmup, profile=False):
        torch.cuda.synchronize()
        t = time.perf_counter()
        S = Solver(rp, col, vals, Params(precond_fp32=fp32))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        x = torch.zeros_like(b)
        info = None
        for _ in range(warmup):
            x.zero_()
            _, info = S.solve(b, x, tol=args.tol)
        times = []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            t1 = time.perf_counter()
            _, info = S.solve(b, x, tol=args.tol)
            times.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        total_ms = (time.perf_counter() - t_all) * 1e3
        prof = None
        if profile:
            # Kernel-class timing: HIP events recorded on the handle's stream
            # around every launch of the timed classes, over `steps` more solves
            # (events cannot sit inside the captured step graphs, so these solves
            # launch eagerly; the kernels are the same).
            S.profile(True)
            torch.cuda.synchronize()
            t_p = time.perf_counter()
            for _ in range(steps):
                x.zero_()
                S.solve(b, x, tol=args.tol)
            torch.cuda.synchronize()
            prof_total_ms = (time.perf_counter() - t_p) * 1e3
            S.profile(False)
            prof = {k: S.profile_read(k) for k in range(capi.CPR_KSTAT_COUNT)}
            prof["total_ms"] = prof_total_ms
        levels = [S.level_info(l) for l in range(S.level_info(0)["n_levels"])]
        S.close()
        return dict(setup_s=setup_s, times=times, total_ms=total_ms, info=info, prof=prof, levels=levels,
                    x=x)

    r32 = run(True, args.steps, args.warmup, profile=True)
    print(f"[bench] fp32 precond: its={r32['info']['iterations']} relres={r32['info']['relres_true']:.2e} "
          f"median={statistics.median(r32['times']):.2f} ms setup={r32['setup_s']:.1f}s",
          file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run(False, args.steps, args.warmup)
        print(f"[bench] fp64 precond: its={r64['info']['iterations']} relres={r64['info']['relres_true']:.2e} "
              f"median={statistics.median(r64['times']):.2f} ms setup={r64['setup_s']:.1f}s",
              file=sys.stderr, flush=True)

    names = {capi.CPR_KSTAT_SPMV: "bsr_spmv_fp64", capi.CPR_KSTAT_SMOOTH_L0: "pgs_scm_colour_sweep_level0",
             capi.CPR_KSTAT_TRANSFER_L0: "residual_restrict_prolong_level0", capi.CPR_KSTAT_STAGE2: "stage2_block_gs"}
    kernels = {}
    prof_total = r32["prof"].pop("total_ms")
    for k, (n, ms, by) in r32["prof"].items():
        if n == 0:
            continue
        avg_ms = ms / n
        gbs = by / n / (avg_ms * 1e-3) / 1e9
        kernels[names[k]] = {"launches": n, "avg_us": avg_ms * 1e3, "bytes_per_launch": by / n,
                             "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                             "share_of_profiled_solves": ms / prof_total}
    dom = max(kernels, key=lambda k: kernels[k]["share_of_profiled_solves"]) if kernels else None
    roof = None
    if dom:
        d = kernels[dom]
        roof = {"bound": "hbm", "kernel": dom, "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["achieved_GBs"] / HBM_PEAK_GBS, "traffic": None}

    med32 = statistics.median(r32["times"])
    out = {
        "metric": METRIC,
        "value": med32,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["total_ms"] / args.steps,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 preconditioner / f64 FGMRES",
        "data": "synthetic",
        "config": {"workload": f"spe10-like black-oil Jacobian {shape[0]}x{shape[1]}x{shape[2]}, "
                               f"2.5% inactive, layered lognormal sigma=2, kz/kx=0.1",
                   "n_cells": case.n_b, "dof": case.ndof, "nnz_blocks": case.nnz_b, "tol": args.tol,
                   "krylov": "FGMRES(30)", "amg": "RS theta=0.25, coarse<=50, PGS-SCM theta=0.05, 2+2 sweeps",
                   "stage2": "multi-colour block GS"},
        "p50_ms": _pct(r32["times"], 0.5),
        "p99_ms": _pct(r32["times"], 0.99),
        "iterations_fp32": r32["info"]["iterations"],
        "relres_true_fp32": r32["info"]["relres_true"],
        "setup_s_fp32": r32["setup_s"],
        "levels": [lv["n"] for lv in r32["levels"]],
        "colours": [lv["n_colours"] for lv in r32["levels"]],
        "roofline": roof,
        "kernels": kernels,
    }
    if r64:
        med64 = statistics.median(r64["times"])
        out.update({"fp64_ms": med64, "fp64_p99_ms": _pct(r64["times"], 0.99),
                    "iterations_fp64": r64["info"]["iterations"], "relres_true_fp64": r64["info"]["relres_true"],
                    "setup_s_fp64": r64["setup_s"], "speedup_fp32_vs_fp64": med64 / med32})
    if not args.no_cpu_baseline:
        its = r64["info"]["iterations"] if r64 else r32["info"]["iterations"]
        out["cpu_baseline"] = cpu_baseline(shape, its, case.n_b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
