"""Unsmoothed-aggregation AMG with pairwise matching and the nonlinear AMLI-cycle (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6's solver paragraph names the paper's own B_P: unsmoothed
aggregation AMG, aggregates from non-symmetric pairwise matching (NPAIR),
the nonlinear AMLI-cycle, PGS-SCM smoothing, and a direct solver on a
coarsest space of 10000 unknowns.  The paper gives no formulas; this module
writes out the cited methods in their textbook form, with the readings
below fixed so that the device library can reproduce the aggregates exactly.

* Matching (one pass, on a matrix A).  Couplings are read from the symmetric
  part, s_ij = a_ij / 2 + a_ji / 2 for j != i, the half-entry of the
  lower-numbered row added first, a missing entry counting as 0 (the
  non-symmetric variant of pairwise matching).  Row i's strong set is S_i = {j != i : s_ij <
  -beta * max_k(-s_ik)} when that maximum is positive, else empty (beta =
  0.25).  m_i counts the unaggregated rows k with i in S_k.  While rows are
  left: take the unaggregated row i with the smallest m_i (ties: smallest
  index); among the unaggregated j in S_i take the one with the most
  negative s_ij (ties: smallest index); {i, j} becomes an aggregate, or {i}
  alone when no such j exists; the rows leave the pool and every m_k with k
  in S_l of a leaving row l drops by one.  Aggregates are numbered in the
  order they are formed.
* NPAIR: ``npair`` (2) successive matching passes per level.  The second
  pass runs on A_1 = P_1^T A P_1 (used only for the matching); the level's
  prolongation is P = P_1 P_2, a 0/1 matrix with one entry per row (row i
  carries a 1 in the column of its aggregate), so aggregates hold at most
  2**npair rows; R = P^T is stored explicitly and A_c = R (A P) in the fixed
  order of ``rs.galerkin`` (the 0/1 weights make every coarse entry a sum of
  fine entries).
* Levels: aggregate until a level has at most ``coarse_max`` rows (the
  paper's 10000), until the next level would keep more than 90% of the rows,
  or at ``max_levels``; every non-coarsest level gets the PGS-SCM colouring
  of eq. (strong-matrix) as in ``amg``; the coarsest level is factored by
  dense LU with partial pivoting.
* Nonlinear AMLI-cycle B_l(b) (Hu, Vassilevski and Xu's analysis of the
  cycle the paper cites; the K-cycle of Notay and Vassilevski): x = 0;
  nu1 PGS-SCM sweeps; r = b - A_l x; b_c = R r; the coarse correction e_c is
  the exact solve when level l+1 is the coarsest, otherwise ``inner`` (2)
  steps of flexible GCR on A_{l+1} e = b_c from e = 0 with B_{l+1} as the
  (changing) preconditioner; x = x + P e_c; nu2 sweeps.  GCR is used rather
  than flexible CG because the decoupled pressure matrices are not
  symmetric.
* Flexible GCR (k = 1, 2, ...): z_k = B(r_{k-1}), w_k = A z_k; for every
  earlier i: beta = (w_k, w_i) / (w_i, w_i), z_k -= beta z_i, w_k -= beta w_i;
  alpha = (r_{k-1}, w_k) / (w_k, w_k); e += alpha z_k; r_k = r_{k-1} -
  alpha w_k.  It stops early if (w_k, w_k) = 0.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import amg, coloring, rs, strength
from .sparse import Csr, matvec, pattern_lists, residual, transpose


@dataclass
class UaParams:
    beta: float = 0.25         # strong-coupling threshold of the matching
    npair: int = 2             # matching passes per level
    coarse_max: int = 10000    # coarsest size (Section 6)
    max_levels: int = 25
    theta_color: float = 0.05  # PGS-SCM colouring threshold, eq. (strong-matrix)
    pre_sweeps: int = 2
    post_sweeps: int = 2
    inner: int = 2             # flexible GCR steps per coarse correction
    smoother: str = "pgs-scm"  # read by amg.smooth
    gs_chunks: int = 4096


def symmetric_strength(A: Csr, beta):
    """S_i of the matching as lists, from s_ij = (a_ij + a_ji) / 2."""
    n = A.n_rows
    s = [dict() for _ in range(n)]
    for i in range(n):
        for p in range(A.indptr[i], A.indptr[i + 1]):
            j = int(A.indices[p])
            if j == i:
                continue
            a = float(A.data[p])
            s[i][j] = s[i].get(j, 0.0) + a / 2.0
            s[j][i] = s[j].get(i, 0.0) + a / 2.0
    S = []
    for i in range(n):
        neg = [-v for v in s[i].values()]
        top = max(neg) if neg else 0.0
        if top > 0.0:
            S.append(sorted(j for j, v in s[i].items() if v < -beta * top))
        else:
            S.append([])
    return S, s


def pairwise_matching(A: Csr, beta):
    """One matching pass: aggregate id of every row, and the aggregate count.

    The row with the smallest m_i is found with a heap of (m_i, i) entries;
    entries whose row left the pool or whose count changed are skipped when
    popped (a fresh entry is pushed on every change)."""
    n = A.n_rows
    S, s = symmetric_strength(A, beta)
    m = np.zeros(n, dtype=np.int64)
    for i in range(n):
        for k in S[i]:
            m[k] += 1
    heap = [(int(m[i]), i) for i in range(n)]
    heapq.heapify(heap)
    agg = np.full(n, -1, dtype=np.int64)
    n_agg = 0
    while heap:
        mi, i = heapq.heappop(heap)
        if agg[i] >= 0 or mi != m[i]:
            continue
        best, best_v = -1, 0.0
        for j in S[i]:
            if agg[j] >= 0:
                continue
            v = s[i][j]
            if best < 0 or v < best_v:
                best, best_v = j, v
        members = [i] if best < 0 else [i, best]
        for l in members:
            agg[l] = n_agg
        for l in members:
            for k in S[l]:
                m[k] -= 1
                if agg[k] < 0:
                    heapq.heappush(heap, (int(m[k]), k))
        n_agg += 1
    return agg, n_agg


def aggregation_matrix(agg, n_agg) -> Csr:
    """The 0/1 prolongation of an aggregation: row i has a 1 in column agg[i]."""
    n = agg.shape[0]
    return Csr(n, int(n_agg), np.arange(n + 1, dtype=np.int64), np.asarray(agg, dtype=np.int64).copy(),
               np.ones(n))


def npair_aggregates(A: Csr, beta, npair):
    """Aggregate of every row after ``npair`` matching passes, and the count."""
    agg = np.arange(A.n_rows, dtype=np.int64)
    n_agg = A.n_rows
    Ak = A
    for _ in range(npair):
        a, na = pairwise_matching(Ak, beta)
        agg = a[agg]
        n_agg = na
        _, Ak = rs.galerkin(Ak, aggregation_matrix(a, na))
    return agg, n_agg


def build_hierarchy(A0: Csr, params: UaParams | None = None) -> amg.Hierarchy:
    params = params or UaParams()
    H = amg.Hierarchy(params=params)
    A = A0
    while True:
        lev = amg.Level(A=A, diag=A.diagonal())
        H.levels.append(lev)
        n = A.n_rows
        if n <= params.coarse_max or len(H.levels) >= params.max_levels:
            break
        agg, n_agg = npair_aggregates(A, params.beta, params.npair)
        if n_agg == 0 or n_agg > 0.9 * n:
            break
        P = aggregation_matrix(agg, n_agg)
        R, Ac = rs.galerkin(A, P)
        lev.P, lev.R = P, R
        lev.agg = agg
        A = Ac
    for lev in H.levels[:-1]:
        cmask, (cp, ci) = strength.color_strength(lev.A, params.theta_color)
        lev.color_mask = cmask
        lev.colours = coloring.vertices_grouping(lev.A.n_rows, pattern_lists(cp, ci))
    H.lu = scipy.linalg.lu_factor(H.levels[-1].A.to_dense())
    return H


def gcr(A: Csr, f, precond, steps):
    """``steps`` flexible GCR steps on A e = f from e = 0 (``precond`` may change
    between calls).  Returns e."""
    e = np.zeros_like(f)
    r = f.copy()
    Z, W, D = [], [], []
    for k in range(steps):
        z = precond(r)
        w = matvec(A, z)
        for zi, wi, di in zip(Z, W, D):
            beta = np.dot(w, wi) / di
            z = z - beta * zi
            w = w - beta * wi
        d = np.dot(w, w)
        if d == 0.0:
            break
        alpha = np.dot(r, w) / d
        e = e + alpha * z
        r = r - alpha * w
        Z.append(z)
        W.append(w)
        D.append(d)
    return e


def kcycle(H: amg.Hierarchy, b, level=0, dtype=np.float64):
    """One nonlinear AMLI-cycle B_level(b) from a zero initial guess."""
    p = H.params
    if level == H.n_levels - 1:
        return scipy.linalg.lu_solve(H.lu, b.astype(np.float64)).astype(dtype)
    lev = H.levels[level]
    A = lev.A if dtype == np.float64 else amg._cast(lev.A, dtype)
    x = np.zeros(A.n_rows, dtype=dtype)
    b = b.astype(dtype)
    for _ in range(p.pre_sweeps):
        amg.smooth(H, lev, A, x, b)
    r = residual(A, x, b)
    R = lev.R if dtype == np.float64 else amg._cast(lev.R, dtype)
    P = lev.P if dtype == np.float64 else amg._cast(lev.P, dtype)
    bc = matvec(R, r)
    if level + 1 == H.n_levels - 1:
        ec = kcycle(H, bc, level + 1, dtype)
    else:
        Ac = H.levels[level + 1].A
        Ac = Ac if dtype == np.float64 else amg._cast(Ac, dtype)
        ec = gcr(Ac, bc, lambda v: kcycle(H, v, level + 1, dtype), p.inner).astype(dtype)
    x = x + matvec(P, ec)
    for _ in range(p.post_sweeps):
        amg.smooth(H, lev, A, x, b)
    return x


def operator_complexity(H: amg.Hierarchy):
    return sum(l.A.nnz for l in H.levels) / H.levels[0].A.nnz


def aggregates_of(P: Csr):
    """Aggregate id of every row of a 0/1 aggregation prolongation."""
    return np.asarray(P.indices, dtype=np.int64)


__all__ = ["UaParams", "symmetric_strength", "pairwise_matching", "aggregation_matrix", "npair_aggregates",
           "build_hierarchy", "gcr", "kcycle", "operator_complexity", "aggregates_of", "transpose"]
