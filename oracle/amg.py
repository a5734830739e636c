"""Pressure AMG hierarchy, PGS-SCM smoother and V-cycle (oracle; test infrastructure only).

* Hierarchy: RS strength + C/F split + interpolation + Galerkin product on
  each level (module ``rs``), a colouring of every non-coarsest level on the
  paper's strong-connection matrix (Section 5.2, eq. (strong-matrix),
  Algorithms VerticesSplitting/VerticesGrouping), and a dense LU with partial
  pivoting on the coarsest level (Section 6 uses a direct coarsest solver).
  Coarsening stops when a level has at most ``coarse_max`` rows, when the
  next level would keep more than 90% of the rows (or none), or at
  ``max_levels`` levels.

* Smoother: Algorithm PGS-SCM.  Colour classes are relaxed in creation
  order; the rows of one colour are updated "in parallel", which is read
  deterministically: every row of colour l sees the values of the earlier
  colours already updated in this sweep and the values its own colour held
  when the colour started (a snapshot).  When the colouring was built with
  theta = 0 no two rows of one colour are coupled (Proposition "Matrix
  diagonalization"), so the sweep is exactly a forward Gauss-Seidel sweep in
  colour-concatenated order.  Pre- and post-smoothing both run the colours
  forward.  Per row: s = b_i, then s = s - a_ij*x_j for every stored j != i
  in stored order, then x_i = s / a_ii.

* PGS-NO (the paper's reference smoother, "parallel GS based on natural
  ordering", run on NT threads in Section 6): the rows in natural order are
  split into ``gs_chunks`` contiguous chunks (sizes differing by at most one,
  the longer ones first); inside a chunk the rows are relaxed in order with
  the newest values of the chunk's own rows, and rows of other chunks are
  read as they were when the sweep started (block Jacobi across chunks,
  Gauss-Seidel inside them).  One chunk is classical forward GS; one row per
  chunk is Jacobi.  Selected with ``smoother="pgs-no"``.

* V-cycle from a zero initial guess: nu1 pre-sweeps, r = b - A x (stored
  order, diagonal included), b_c = R r (row sums from 0 in stored order),
  recursion, x_i = x_i + (sum_J p_iJ e_J) with the sum from 0 in stored
  order, nu2 post-sweeps; the coarsest level is solved with the LU.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import coloring, rs, strength
from .sparse import Csr, matvec, padded, pattern_lists, residual


@dataclass
class AmgParams:
    theta_rs: float = 0.25
    theta_color: float = 0.05
    coarse_max: int = 50
    max_levels: int = 25
    pre_sweeps: int = 2
    post_sweeps: int = 2
    smoother: str = "pgs-scm"   # or "pgs-no"
    gs_chunks: int = 4096       # PGS-NO: chunks per level


@dataclass
class Level:
    A: Csr
    rs_mask: np.ndarray | None = None
    color_mask: np.ndarray | None = None
    colours: list | None = None
    cf: np.ndarray | None = None
    P: Csr | None = None
    R: Csr | None = None
    diag: np.ndarray | None = None


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    lu: tuple | None = None  # scipy lu_factor of the coarsest matrix
    params: AmgParams = field(default_factory=AmgParams)

    @property
    def n_levels(self):
        return len(self.levels)


def build_hierarchy(A0: Csr, params: AmgParams | None = None) -> Hierarchy:
    params = params or AmgParams()
    H = Hierarchy(params=params)
    A = A0
    while True:
        lev = Level(A=A, diag=A.diagonal())
        H.levels.append(lev)
        n = A.n_rows
        if n <= params.coarse_max or len(H.levels) >= params.max_levels:
            break
        rs_mask, (sp, si) = strength.rs_strength(A, params.theta_rs)
        S = pattern_lists(sp, si)
        ST = [[] for _ in range(n)]
        for i in range(n):
            for j in S[i]:
                ST[j].append(i)
        cf = rs.rs_split(n, S, ST)
        nc = int(np.count_nonzero(cf == rs.C))
        if nc == 0 or nc > 0.9 * n:
            break
        P = rs.interpolation(A, rs_mask, cf)
        R, Ac = rs.galerkin(A, P)
        lev.rs_mask, lev.cf, lev.P, lev.R = rs_mask, cf, P, R
        A = Ac
    # colourings for every smoothed (non-coarsest) level
    for lev in H.levels[:-1]:
        cmask, (cp, ci) = strength.color_strength(lev.A, params.theta_color)
        lev.color_mask = cmask
        lev.colours = coloring.vertices_grouping(lev.A.n_rows, pattern_lists(cp, ci))
    H.lu = scipy.linalg.lu_factor(H.levels[-1].A.to_dense())
    return H


def colour_sweep(A: Csr, colours, x, b, diag=None):
    """One PGS-SCM sweep (in place on x), colours in creation order."""
    if diag is None:
        diag = A.diagonal()
    for members in colours:
        rows = np.asarray(members, dtype=np.int64)
        cols, vals, _ = padded(A, rows)
        vals = np.where(cols == rows[:, None], 0.0, vals)  # j != i
        snap = x.copy()
        s = b[rows].astype(x.dtype, copy=True)
        for t in range(cols.shape[1]):
            s = s - vals[:, t].astype(x.dtype) * snap[cols[:, t]]
        x[rows] = s / diag[rows].astype(x.dtype)
    return x


def chunk_bounds(n, n_chunks):
    """PGS-NO chunk boundaries: min(n_chunks, n) contiguous ranges of rows."""
    c = max(1, min(int(n_chunks), n))
    q, r = divmod(n, c)
    bounds = [0]
    for k in range(c):
        bounds.append(bounds[-1] + q + (1 if k < r else 0))
    return bounds


def natural_chunk_sweep(A: Csr, n_chunks, x, b, diag=None):
    """One PGS-NO sweep (in place on x).

    Row t of every chunk is relaxed in the same step (chunks are independent
    given the sweep-start snapshot, so this is the per-chunk sequential loop
    run side by side).  Per row: s = b_i, then s = s - a_ij * xt_j for every
    stored j != i in stored order, with xt_j = x_j when j is in the row's chunk
    (already relaxed when j < i) and the snapshot otherwise; x_i = s / a_ii."""
    if diag is None:
        diag = A.diagonal()
    n = A.n_rows
    bounds = np.asarray(chunk_bounds(n, n_chunks), dtype=np.int64)
    chunk = np.repeat(np.arange(len(bounds) - 1), np.diff(bounds))
    snap = x.copy()
    lo, hi = bounds[:-1], bounds[1:]
    for t in range(int(np.max(hi - lo)) if n else 0):
        rows = (lo + t)[lo + t < hi]
        cols, vals, _ = padded(A, rows)
        vals = np.where(cols == rows[:, None], 0.0, vals)
        s = b[rows].astype(x.dtype, copy=True)
        for k in range(cols.shape[1]):
            c = cols[:, k]
            xt = np.where(chunk[c] == chunk[rows], x[c], snap[c])
            s = s - vals[:, k].astype(x.dtype) * xt
        x[rows] = s / diag[rows].astype(x.dtype)
    return x


def smooth(H: Hierarchy, lev: Level, A: Csr, x, b):
    """One smoothing sweep of the configured kind on level ``lev``."""
    if H.params.smoother == "pgs-no":
        return natural_chunk_sweep(A, H.params.gs_chunks, x, b, lev.diag)
    return colour_sweep(A, lev.colours, x, b, lev.diag)


def vcycle(H: Hierarchy, b, level=0, dtype=np.float64):
    """One V-cycle applied to b on ``level`` from a zero initial guess."""
    lev = H.levels[level]
    if level == H.n_levels - 1:
        e = scipy.linalg.lu_solve(H.lu, b.astype(np.float64))
        return e.astype(dtype)
    p = H.params
    A = lev.A if dtype == np.float64 else _cast(lev.A, dtype)
    x = np.zeros(A.n_rows, dtype=dtype)
    b = b.astype(dtype)
    for _ in range(p.pre_sweeps):
        smooth(H, lev, A, x, b)
    r = residual(A, x, b)
    R = lev.R if dtype == np.float64 else _cast(lev.R, dtype)
    P = lev.P if dtype == np.float64 else _cast(lev.P, dtype)
    bc = matvec(R, r)
    e = vcycle(H, bc, level + 1, dtype)
    x = x + matvec(P, e)
    for _ in range(p.post_sweeps):
        smooth(H, lev, A, x, b)
    return x


def _cast(A: Csr, dtype):
    return Csr(A.n_rows, A.n_cols, A.indptr, A.indices, A.data.astype(dtype))


def operator_complexity(H: Hierarchy):
    return sum(l.A.nnz for l in H.levels) / H.levels[0].A.nnz
