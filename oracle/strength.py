"""Strength of connection (oracle; test infrastructure only).

Two different notions are used on every AMG level:

* ``color_strength`` is the paper's matrix of strong connections S(A, theta),
  eq. (strong-matrix) in Section 5.2: S_ij = 1 iff i != j and
  |a_ij| > theta * sum_k |a_ik|.  The sum runs over every stored entry of row
  i, diagonal included, accumulated left to right in stored order.  It drives
  the vertex colouring of the PGS-SCM smoother.

* ``rs_strength`` is the classical Ruge-Stueben strength used for C/F
  coarsening (the paper's own AMG is aggregation based and does not define
  one): j is a strong dependency of i iff j != i and
  -a_ij >= theta * max_{k != i}(-a_ik), provided that maximum is positive;
  otherwise row i has no strong dependencies.

Both return a boolean mask over the stored entries of A (the quantity the
device must reproduce bit for bit) and the pattern as (indptr, indices).
"""
from __future__ import annotations

import numpy as np

from .sparse import Csr, padded


def _mask_to_pattern(A: Csr, mask):
    counts = np.zeros(A.n_rows, dtype=np.int64)
    row_of = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    np.add.at(counts, row_of[mask], 1)
    indptr = np.zeros(A.n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, A.indices[mask].astype(np.int64)


def color_strength(A: Csr, theta: float):
    """eq. (strong-matrix): mask of stored entries with |a_ij| > theta*sum_k |a_ik|."""
    cols, vals, valid = padded(A)
    rowsum = np.zeros(A.n_rows)
    for t in range(cols.shape[1]):
        rowsum = rowsum + np.abs(vals[:, t])
    bound = theta * rowsum
    row_of = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    mask = (np.abs(A.data) > bound[row_of]) & (A.indices != row_of)
    return mask, _mask_to_pattern(A, mask)


def rs_strength(A: Csr, theta: float):
    """Classical RS strength: -a_ij >= theta * max_{k!=i}(-a_ik) when that max > 0."""
    row_of = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    offdiag = A.indices != row_of
    neg = np.where(offdiag, -A.data, -np.inf)
    rowmax = np.full(A.n_rows, -np.inf)
    np.maximum.at(rowmax, row_of, neg)
    bound = theta * rowmax
    mask = offdiag & (rowmax[row_of] > 0.0) & (-A.data >= bound[row_of])
    return mask, _mask_to_pattern(A, mask)
