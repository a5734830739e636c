"""Block ILU(0) second stage with level scheduling (oracle; test infrastructure only).

Section 3.1 names block ILU as the relaxation operator R of eq. (CPR), and
Section 6 computes it "based on level scheduling" (citing Saad, *Iterative
Methods for Sparse Linear Systems*, 2nd ed.).  Written out here from the
textbook definitions:

* Factorisation (ILU(0), IKJ form, on 3x3 blocks, natural row order, no fill:
  the factors keep exactly the stored block pattern of A).  For each row i in
  ascending order, for each stored k < i in ascending order:
      L_ik  = A_ik U_kk^{-1}
      A_ij -= L_ik U_kj   for every stored j > k of row k that is also
                          stored in row i,
  where row k is already final.  Row i then holds L_ik (k < i), U_ii (the
  updated diagonal block) and U_ij (j > i).  U_ii^{-1} is the inverse of the
  3x3 block by LU with partial pivoting (LAPACK through numpy.linalg.inv).
  The product L_ik U_kj of two blocks is an ordinary 3x3 matrix product
  (numpy.matmul), A_ik U_kk^{-1} likewise.
* Solve (L U) d = r with L unit lower block triangular:
      y_i = r_i - sum_{k < i} L_ik y_k            (forward, ascending i)
      d_i = U_ii^{-1} (y_i - sum_{j > i} U_ij d_j)  (backward, descending i)
  Each block product is summed in stored block order, component by component
  (column 0, 1, 2 of the block), one product at a time, as in
  ``cpr.bsr_residual``; U_ii^{-1} t is summed from 0 over columns 0, 1, 2.
* Level scheduling: the forward level of row i is 0 when row i has no stored
  k < i, else 1 + the largest forward level among them; the backward level
  uses the stored j > i.  Rows of one level depend only on rows of earlier
  levels, so they can be processed in parallel; every row's arithmetic is the
  same as in the sequential loop, so the result does not depend on the
  schedule.  The sequential loops below define the result; the level sets are
  returned for checking and for the device schedule.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BiluFactors:
    row_ptr: np.ndarray
    col: np.ndarray
    LU: np.ndarray       # [nnz, 3, 3]: L_ik for k < i, U_ij for j >= i (U_ii updated diagonal)
    Uinv: np.ndarray     # [n, 3, 3]: inverse of U_ii
    diag_pos: np.ndarray  # position of block (i, i) in row i

    @property
    def n_b(self):
        return int(self.row_ptr.shape[0] - 1)

    def cast(self, dtype):
        return BiluFactors(self.row_ptr, self.col, self.LU.astype(dtype), self.Uinv.astype(dtype), self.diag_pos)


def bilu0(A) -> BiluFactors:
    """Block ILU(0) of a 3x3-block matrix with sorted columns and stored diagonals."""
    n = A.n_b
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    LU = np.array(A.vals, dtype=np.float64, copy=True)
    Uinv = np.empty((n, 3, 3))
    diag_pos = np.empty(n, dtype=np.int64)
    for i in range(n):
        a, b = rp[i], rp[i + 1]
        pos_in_row = {int(col[p]): p for p in range(a, b)}
        diag_pos[i] = pos_in_row[i]
        for p in range(a, b):
            k = int(col[p])
            if k >= i:
                break
            LU[p] = LU[p] @ Uinv[k]
            for q in range(rp[k], rp[k + 1]):
                j = int(col[q])
                if j <= k:
                    continue
                t = pos_in_row.get(j)
                if t is not None:
                    LU[t] = LU[t] - LU[p] @ LU[q]
        Uinv[i] = np.linalg.inv(LU[diag_pos[i]])
    return BiluFactors(rp, col, LU, Uinv, diag_pos)


def forward_levels(row_ptr, col):
    """Level of each row in the forward (lower) solve."""
    n = len(row_ptr) - 1
    lev = np.zeros(n, dtype=np.int64)
    for i in range(n):
        m = -1
        for p in range(row_ptr[i], row_ptr[i + 1]):
            k = col[p]
            if k < i:
                m = max(m, lev[k])
        lev[i] = m + 1
    return lev


def backward_levels(row_ptr, col):
    """Level of each row in the backward (upper) solve."""
    n = len(row_ptr) - 1
    lev = np.zeros(n, dtype=np.int64)
    for i in range(n - 1, -1, -1):
        m = -1
        for p in range(row_ptr[i], row_ptr[i + 1]):
            j = col[p]
            if j > i:
                m = max(m, lev[j])
        lev[i] = m + 1
    return lev


def _block_sub(t, blk, v):
    """t - blk v, one product at a time: for each row r, columns 0, 1, 2."""
    for r in range(3):
        for c in range(3):
            t[r] = t[r] - blk[r, c] * v[c]
    return t


def solve(F: BiluFactors, r):
    """d = (L U)^{-1} r, the forward then the backward substitution."""
    dt = F.LU.dtype
    n = F.n_b
    r3 = np.asarray(r, dtype=dt).reshape(-1, 3)
    y = np.zeros((n, 3), dtype=dt)
    for i in range(n):
        t = r3[i].copy()
        for p in range(F.row_ptr[i], F.row_ptr[i + 1]):
            k = F.col[p]
            if k >= i:
                break
            t = _block_sub(t, F.LU[p], y[k])
        y[i] = t
    d = np.zeros((n, 3), dtype=dt)
    for i in range(n - 1, -1, -1):
        t = y[i].copy()
        for p in range(F.diag_pos[i] + 1, F.row_ptr[i + 1]):
            t = _block_sub(t, F.LU[p], d[F.col[p]])
        out = np.zeros(3, dtype=dt)
        for rr in range(3):
            for c in range(3):
                out[rr] = out[rr] + F.Uinv[i, rr, c] * t[c]
        d[i] = out
    return d.reshape(-1)


def solve_by_levels(F: BiluFactors, r, flev=None, blev=None):
    """``solve`` executed level by level (all rows of a level at once).

    Every row performs the same operations in the same order as in ``solve``
    (the rows it reads are final before its level starts), so the result is
    identical bit for bit; this is the schedule the device runs."""
    dt = F.LU.dtype
    n = F.n_b
    if flev is None:
        flev = forward_levels(F.row_ptr, F.col)
    if blev is None:
        blev = backward_levels(F.row_ptr, F.col)
    r3 = np.asarray(r, dtype=dt).reshape(-1, 3)
    y = np.zeros((n, 3), dtype=dt)
    for lv in range(int(flev.max()) + 1 if n else 0):
        rows = np.nonzero(flev == lv)[0]
        t = r3[rows].copy()
        w = int(np.max(F.diag_pos[rows] - F.row_ptr[rows])) if rows.size else 0
        for s in range(w):
            p = F.row_ptr[rows] + s
            on = p < F.diag_pos[rows]
            pp = np.where(on, p, F.diag_pos[rows])
            k = F.col[pp]
            blk = F.LU[pp]
            v = y[k]
            for rr in range(3):
                for c in range(3):
                    t[:, rr] = np.where(on, t[:, rr] - blk[:, rr, c] * v[:, c], t[:, rr])
        y[rows] = t
    d = np.zeros((n, 3), dtype=dt)
    for lv in range(int(blev.max()) + 1 if n else 0):
        rows = np.nonzero(blev == lv)[0]
        t = y[rows].copy()
        w = int(np.max(F.row_ptr[rows + 1] - F.diag_pos[rows] - 1)) if rows.size else 0
        for s in range(w):
            p = F.diag_pos[rows] + 1 + s
            on = p < F.row_ptr[rows + 1]
            pp = np.where(on, p, F.diag_pos[rows])
            j = F.col[pp]
            blk = F.LU[pp]
            v = d[j]
            for rr in range(3):
                for c in range(3):
                    t[:, rr] = np.where(on, t[:, rr] - blk[:, rr, c] * v[:, c], t[:, rr])
        out = np.zeros_like(t)
        Ui = F.Uinv[rows]
        for rr in range(3):
            for c in range(3):
                out[:, rr] = out[:, rr] + Ui[:, rr, c] * t[:, c]
        d[rows] = out
    return d.reshape(-1)
