"""Classical Ruge-Stueben coarsening for the pressure AMG (oracle; test infrastructure only).

The paper names its pressure solver B_P (Section 3.1) but leaves its
construction to an external aggregation AMG (Section 6).  The configuration
reproduced here uses classical RS coarsening instead, so this module writes
out the textbook algorithm (Ruge and Stueben 1987; Briggs, Henson and
McCormick, "A Multigrid Tutorial", 2nd ed., ch. 8) with every tie-break and
summation order fixed, because the device library must reproduce the C/F
split bit for bit.

Conventions (S is the RS strength pattern of ``strength.rs_strength``):

* S_i = strong dependencies of i (row i of S); S^T_i = points that strongly
  depend on i.
* First pass.  Points with S_i and S^T_i both empty are F points with an
  empty interpolation row.  Every other point starts undecided with
  lambda_i = |S^T_i|.  Repeatedly take the undecided point of largest lambda
  (ties: smallest index) while that lambda is positive; it becomes C; each
  undecided j in S^T_i becomes F and, for each such j, every undecided k in
  S_j gets lambda_k += 1; then every undecided j in S_i gets lambda_j -= 1.
  Points still undecided when the largest lambda is 0 are visited in
  ascending order: F if one of their strong dependencies is already C,
  otherwise C.
* Second pass.  F points are visited in ascending order.  For F point i let
  C_i = S_i restricted to C points.  Its strong F dependencies j are visited
  in stored order; j violates the rule when no point of S_j lies in C_i.  The
  first violator becomes a tentative C point (joining C_i); a second violator
  turns i itself into a C point and sends the tentative point back to F.
* Coarse points are numbered in ascending fine index.
"""
from __future__ import annotations

import heapq

import numpy as np

from .sparse import Csr, transpose

U, C, F = 0, 1, 2


def rs_split(n, S, ST):
    """C/F split; S and ST are lists of lists.  Returns int8 array of C(1)/F(2)."""
    state = np.full(n, U, dtype=np.int8)
    lam = np.zeros(n, dtype=np.int64)
    heap = []
    for i in range(n):
        if not S[i] and not ST[i]:
            state[i] = F
        else:
            lam[i] = len(ST[i])
            heap.append((-lam[i], i))
    heapq.heapify(heap)

    while heap:
        neg, i = heapq.heappop(heap)
        if state[i] != U or -neg != lam[i]:
            continue  # stale entry
        if lam[i] == 0:
            break
        state[i] = C
        for j in ST[i]:
            if state[j] == U:
                state[j] = F
                for k in S[j]:
                    if state[k] == U:
                        lam[k] += 1
                        heapq.heappush(heap, (-lam[k], k))
        for j in S[i]:
            if state[j] == U:
                lam[j] -= 1
                heapq.heappush(heap, (-lam[j], j))

    for i in range(n):
        if state[i] == U:
            state[i] = F if any(state[j] == C for j in S[i]) else C

    # second pass
    for i in range(n):
        if state[i] != F:
            continue
        Ci = set(j for j in S[i] if state[j] == C)
        tentative = -1
        for j in S[i]:
            if state[j] != F:
                continue
            if any(k in Ci for k in S[j]):
                continue
            if tentative < 0:
                tentative = j
                state[j] = C
                Ci.add(j)
            else:
                state[tentative] = F
                state[i] = C
                break
    return state


def interpolation(A: Csr, S_mask, state):
    """Classical RS interpolation P (n_fine x n_coarse).

    For a C point i the row is the unit vector of its coarse index.  For an F
    point i with interpolatory set C_i (strong C dependencies, stored order):

        d     = a_ii + sum of a_ij over weak j (j not a strong dependency)
        num_j = a_ij + sum over strong F dependencies m of a_im*a_mj / den_m
        den_m = sum of a_mk over k in C_i (row m, stored order)
        w_ij  = -num_j / d

    A strong F dependency m with den_m == 0 is lumped into d like a weak one.
    Sums run in stored order: d first over the weak entries, then the lumped
    ones in the order the strong F dependencies are met.
    """
    n = A.n_rows
    coarse = np.full(n, -1, dtype=np.int64)
    cpts = np.nonzero(state == C)[0]
    coarse[cpts] = np.arange(cpts.size)
    row_of = np.repeat(np.arange(n), np.diff(A.indptr))
    strong = S_mask
    indptr = [0]
    indices, data = [], []
    for i in range(n):
        a, b = A.indptr[i], A.indptr[i + 1]
        cols, vals, st = A.indices[a:b], A.data[a:b], strong[a:b]
        if state[i] == C:
            indices.append(coarse[i])
            data.append(1.0)
            indptr.append(len(indices))
            continue
        Ci = [j for j, s in zip(cols, st) if s and state[j] == C]
        if not Ci:
            indptr.append(len(indices))
            continue
        Cset = set(Ci)
        d = 0.0
        for j, v in zip(cols, vals):
            if j == i:
                d = v
        for j, v, s in zip(cols, vals, st):
            if j != i and not s:
                d = d + v
        num = {}
        for j, v, s in zip(cols, vals, st):
            if s and state[j] == C:
                num[j] = v
        for m, a_im, s in zip(cols, vals, st):
            if not s or state[m] != F:
                continue
            ma, mb = A.indptr[m], A.indptr[m + 1]
            den = 0.0
            for k, a_mk in zip(A.indices[ma:mb], A.data[ma:mb]):
                if k in Cset:
                    den = den + a_mk
            if den == 0.0:
                d = d + a_im
                continue
            for k, a_mk in zip(A.indices[ma:mb], A.data[ma:mb]):
                if k in Cset:
                    num[k] = num[k] + (a_im * a_mk) / den
        for j in Ci:
            indices.append(coarse[j])
            data.append(-num[j] / d)
        indptr.append(len(indices))
    del row_of
    return Csr(n, int(cpts.size), np.array(indptr, dtype=np.int64),
               np.array(indices, dtype=np.int64), np.array(data, dtype=np.float64))


def spgemm_ordered(A: Csr, B: Csr) -> Csr:
    """C = A B with a fixed order: for row i, for k in row i of A (stored order),
    for j in row k of B (stored order), c_ij = c_ij + a_ik*b_kj (starting at 0.0);
    each result row is then sorted by column.  No entry is dropped."""
    indptr = [0]
    indices, data = [], []
    for i in range(A.n_rows):
        acc = {}
        for p in range(A.indptr[i], A.indptr[i + 1]):
            k, a_ik = A.indices[p], A.data[p]
            for q in range(B.indptr[k], B.indptr[k + 1]):
                j = B.indices[q]
                acc[j] = acc.get(j, 0.0) + a_ik * B.data[q]
        for j in sorted(acc):
            indices.append(j)
            data.append(acc[j])
        indptr.append(len(indices))
    return Csr(A.n_rows, B.n_cols, np.array(indptr, dtype=np.int64),
               np.array(indices, dtype=np.int64), np.array(data, dtype=np.float64))


def galerkin(A: Csr, P: Csr):
    """R = P^T stored explicitly; A_c = R (A P) in the order of ``spgemm_ordered``."""
    R = transpose(P)
    AP = spgemm_ordered(A, P)
    Ac = spgemm_ordered(R, AP)
    return R, Ac
