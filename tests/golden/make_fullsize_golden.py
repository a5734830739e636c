"""Write the oracle's reference solve at full size (test infrastructure).

Runs the FP64 CPU oracle -- SETUP, then CPR-FGMRES(30) to relres 1e-6 from
x = 0 (Algorithm "ASCPR-GMRES" with the CPR preconditioner of Algorithm "CPR
method") -- and its float32-preconditioner model on one of the full-size
synthetic workloads, and stores what the GPU parity test compares against:
iteration counts, true relative residuals, the norm of x and x itself at a
seeded sample of unknowns.  Only ``oracle/`` and ``workloads/`` are used.

    python tests/golden/make_fullsize_golden.py spe10      # 3.28M DOF
    python tests/golden/make_fullsize_golden.py channels   # 12M DOF
    python tests/golden/make_fullsize_golden.py spe10 4000 # coarsest level <= 4000 rows

With a second argument the AMG coarsens down to that many rows (the default
is 50) and the file name carries it (oracle_fullsize_spe10_coarse4000.json);
the second argument "ua" selects the paper's aggregation AMG with the
AMLI-cycle (coarsest 10000 rows; oracle_fullsize_spe10_ua.json), "bilu" the
block ILU(0) second stage with the default AMG (oracle_fullsize_spe10_bilu.json).

Single-threaded (BLAS limited to one thread), so the recorded wall times are
the oracle's one-core times on the machine that ran the script.
"""
from __future__ import annotations

import dataclasses
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cpr, fgmres  # noqa: E402
from workloads import blackoil as bo  # noqa: E402

N_SAMPLE = 20000


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def sample_dofs(ndof, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(ndof, size=min(N_SAMPLE, ndof), replace=False)
    return np.sort(np.concatenate([idx, [0, ndof - 1]])).astype(np.int64)


def main(which, coarse_max=None):
    from threadpoolctl import threadpool_limits

    from oracle import amg

    if which == "spe10":
        case = bo.case_spe10_like(seed=1100)
        b = bo.rhs(case.ndof, 1101)
        desc = "spe10-like 60x220x85, 2.5% inactive (seed 1100, RHS 1101)"
    elif which == "channels":
        case = bo.case_channels(seed=1400)
        b = bo.rhs(case.ndof, 1401)
        desc = "channelised 200x200x100 (seed 1400, RHS 1401)"
    else:
        raise SystemExit(f"unknown workload {which}")
    second_stage = "bilu" if coarse_max == "bilu" else "bgs"
    if coarse_max == "ua":
        from oracle import uaamg

        amg_params = uaamg.UaParams()
    elif coarse_max == "bilu":
        amg_params = amg.AmgParams()
    else:
        amg_params = amg.AmgParams() if coarse_max is None else amg.AmgParams(coarse_max=coarse_max)
    out = {"workload": desc, "n_b": int(case.n_b), "nnz_b": int(case.nnz_b), "tol": 1e-6, "restart": 30,
           "coarse_max": int(amg_params.coarse_max), "amg": type(amg_params).__name__,
           "second_stage": second_stage}
    print(f"[golden] {desc}: n_b={case.n_b} nnz_b={case.nnz_b}", flush=True)
    with threadpool_limits(limits=1):
        A = cpr.Bsr.from_case(case)
        B64 = None
        for name, dt in (("fp64", np.float64), ("fp32_model", np.float32)):
            t0 = time.perf_counter()
            if B64 is None:
                B = B64 = cpr.setup(A, amg_params, dtype=dt, second_stage=second_stage)
            else:  # the float32 model applies the same SETUP products in float32
                B = dataclasses.replace(B64, dtype=dt)
            t1 = time.perf_counter()
            print(f"[golden] {name} setup {t1 - t0:.1f} s, levels {B.amg.n_levels}", flush=True)
            res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
            t2 = time.perf_counter()
            print(f"[golden] {name} solve {t2 - t1:.1f} s, its {res.iterations}, relres {res.relres_true:.3e}",
                  flush=True)
            rec = {"iterations": int(res.iterations), "relres_true": float(res.relres_true),
                   "relres_est": float(res.relres_est), "converged": bool(res.converged),
                   "history": [float(h) for h in res.history], "setup_s": t1 - t0, "solve_s": t2 - t1,
                   "n_levels": int(B.amg.n_levels)}
            if name == "fp64":
                idx = sample_dofs(case.ndof, 7)
                rec["x_norm"] = float(np.linalg.norm(res.x))
                rec["sample_dof"] = idx.tolist()
                rec["sample_x"] = [float(v) for v in res.x[idx]]
                rec["level_sizes"] = [int(L.A.n_rows) for L in B.amg.levels]
            out[name] = rec
    out["cpu"] = _cpu_name()
    out["cores"] = 1
    suffix = "" if coarse_max is None else (f"_{coarse_max}" if coarse_max in ("ua", "bilu") else f"_coarse{coarse_max}")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_fullsize_{which}{suffix}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"[golden] wrote {path}", flush=True)


if __name__ == "__main__":
    arg2 = sys.argv[2] if len(sys.argv) > 2 else None
    main(sys.argv[1] if len(sys.argv) > 1 else "spe10", arg2 if arg2 in (None, "ua", "bilu") else int(arg2))
