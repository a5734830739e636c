"""The adaptive-setup rule and a Newton-sequence driver (oracle; test infrastructure only).

Section 4, Algorithms "ASCPR-GMRES" and "ASCPR": before solving the k-th
Jacobian the preconditioner of step k-1 is reused when k > 1 and the previous
solve took few iterations, otherwise SETUP runs again; a change of matrix size
always forces a new SETUP (the Remark after the algorithm).  Two forms of
"few" are supported:

* mode "mu"     (the paper's rule): reuse iff It^(k-1) <= mu;
* mode "factor" (relative rule):    reuse iff It^(k-1) <= factor * It_ref,
  where It_ref is the iteration count of the first solve after the last SETUP.

With mode "mu" and mu = 0 every step runs SETUP, i.e. plain CPR-GMRES (the
discussion of the choice of mu).  Reusing B keeps every product of SETUP
frozen, including the copy of A used inside the CPR apply; the outer
FGMRES always uses the current A^(k).  Iterations are inner FGMRES steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cpr, fgmres
from .amg import AmgParams


def decide_rebuild(k, it_prev, it_ref, mode="factor", mu=0, factor=1.3, size_changed=False):
    """True when SETUP must run before solve number k (k counts from 1)."""
    if k <= 1 or size_changed:
        return True
    if mode == "mu":
        return not (it_prev <= mu)
    if mode == "factor":
        return not (it_prev <= factor * it_ref)
    if mode == "never":
        return True
    raise ValueError(mode)


@dataclass
class StepReport:
    step: int
    rebuilt: bool
    iterations: int
    relres_true: float
    converged: bool
    x: np.ndarray | None = None  # the step's iterate


def solve_sequence(steps, params: AmgParams | None = None, tol=1e-6, m=30, mode="factor",
                   mu=0, factor=1.3, dtype=np.float64, second_stage="bgs", decoupling="none"):
    """Run ASCPR-FGMRES over an iterable of (A: cpr.Bsr, b) pairs."""
    B = None
    it_prev = it_ref = 0
    reports = []
    n_prev = None
    for k, (A, b) in enumerate(steps, start=1):
        rebuild = decide_rebuild(k, it_prev, it_ref, mode, mu, factor, size_changed=(A.n_b != n_prev))
        if rebuild:
            B = cpr.setup(A, params, dtype, second_stage=second_stage, decoupling=decoupling)
        res = fgmres.fgmres(lambda v, A=A: cpr.bsr_matvec(A, v), B.apply, b, tol=tol, m=m)
        it_prev = res.iterations
        if rebuild:
            it_ref = res.iterations
        n_prev = A.n_b
        reports.append(StepReport(k, rebuild, res.iterations, res.relres_true, res.converged, res.x))
    return reports
