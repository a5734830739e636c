"""CSR container and row sums taken in stored order (oracle; test infrastructure only).

NumPy's reductions use pairwise summation and BLAS reorders freely, so any
sum whose exact rounding is compared against the device is written here as an
explicit left-to-right loop over the stored entries of each row.  Rows are
padded to a common width with zero values at the end; a zero product added
(or subtracted) leaves a finite partial sum unchanged, so the padding does not
alter the result.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    n_rows: int
    n_cols: int
    indptr: np.ndarray  # int64 [n_rows+1]
    indices: np.ndarray  # int64 [nnz]
    data: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def row(self, i):
        a, b = self.indptr[i], self.indptr[i + 1]
        return self.indices[a:b], self.data[a:b]

    def to_dense(self):
        d = np.zeros((self.n_rows, self.n_cols))
        for i in range(self.n_rows):
            c, v = self.row(i)
            for j, a in zip(c, v):
                d[i, j] += a
        return d

    def diagonal(self):
        dg = np.zeros(self.n_rows)
        for i in range(self.n_rows):
            c, v = self.row(i)
            hit = np.nonzero(c == i)[0]
            if hit.size:
                dg[i] = v[hit[0]]
        return dg


def csr_from_dense(d):
    n, m = d.shape
    indptr = [0]
    indices, data = [], []
    for i in range(n):
        nz = np.nonzero(d[i])[0]
        indices.extend(nz.tolist())
        data.extend(d[i, nz].tolist())
        indptr.append(len(indices))
    return Csr(n, m, np.array(indptr, dtype=np.int64), np.array(indices, dtype=np.int64),
               np.array(data, dtype=np.float64))


def padded(A: Csr, rows=None):
    """Rows (all, or the given subset) as [len, W] column/value arrays, zero-padded."""
    if rows is None:
        rows = np.arange(A.n_rows)
    rows = np.asarray(rows, dtype=np.int64)
    start = A.indptr[rows]
    length = A.indptr[rows + 1] - start
    W = int(length.max()) if rows.size else 0
    t = np.arange(W)[None, :]
    valid = t < length[:, None]
    pos = np.where(valid, start[:, None] + t, 0)
    cols = np.where(valid, A.indices[pos] if A.nnz else 0, 0)
    vals = np.where(valid, A.data[pos] if A.nnz else 0.0, 0.0)
    return cols, vals, valid


def residual(A: Csr, x, b):
    """r_i = b_i - sum_j a_ij x_j, subtracting products one by one in stored order."""
    cols, vals, _ = padded(A)
    s = np.array(b, dtype=vals.dtype, copy=True)
    for t in range(cols.shape[1]):
        s = s - vals[:, t] * x[cols[:, t]]
    return s


def matvec(A: Csr, x):
    """y_i = sum_j a_ij x_j accumulated from 0 in stored order."""
    cols, vals, _ = padded(A)
    s = np.zeros(A.n_rows, dtype=vals.dtype)
    for t in range(cols.shape[1]):
        s = s + vals[:, t] * x[cols[:, t]]
    return s


def transpose(A: Csr) -> Csr:
    """Explicit transpose; each row of the result lists its columns ascending."""
    counts = np.bincount(A.indices, minlength=A.n_cols)
    indptr = np.zeros(A.n_cols + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    row_of = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.indptr))
    # a stable sort by column keeps the source rows ascending inside each column
    order = np.argsort(A.indices, kind="stable")
    return Csr(A.n_cols, A.n_rows, indptr, row_of[order], A.data[order].copy())


def pattern_lists(indptr, indices):
    """Row lists of a boolean pattern as Python lists (for the greedy algorithms)."""
    return [indices[indptr[i]:indptr[i + 1]].tolist() for i in range(len(indptr) - 1)]
