"""CPR two-stage preconditioner on 3x3-block matrices (oracle; test infrastructure only).

Section 3.1 of the paper defines the preconditioner B through its error
propagation, eq. (CPR):  I - B A = (I - R A)(I - Pi_P B_P Pi_P^T A),  and
applies it with Algorithm "CPR method" (x starts at 0 when B is used as a
preconditioner):

    r  = b - A x
    x  = x + Pi_P B_P Pi_P^T r       (stage 1: pressure AMG)
    r  = b - A x
    x  = x + R r                     (stage 2)

* Pi_P^T takes the pressure unknown (slot 0) of every cell; Pi_P puts a
  pressure vector back in slot 0 with zero saturations.  The pressure matrix
  is A_PP = Pi_P^T A Pi_P, i.e. the (0,0) entries of the stored blocks in the
  stored pattern; no decoupling is applied first.
* B_P is one V-cycle of the AMG in ``amg``.
* R is one forward multi-colour block Gauss-Seidel sweep from zero.  The
  cells are coloured by VerticesGrouping with theta = 0 on the block graph
  (edge i-j iff block (i,j) is stored and has a nonzero entry, i != j), and a
  colour reads the snapshot of its own colour exactly like the scalar
  smoother.  Per cell: t = r_i - sum_{j != i} A_ij d_j (component by
  component, blocks in stored order, columns 0..2), then d_i = D_i^{-1} t with
  D_i^{-1} the inverse of the diagonal block (LU with partial pivoting).
* Block products y_i[r] = sum over blocks in stored order of
  a[r][0]*x0 + a[r][1]*x1 + a[r][2]*x2, added one product at a time.
* ``decoupling`` (for the full system with wells of eq. (Jacobian-system);
  the paper leaves the well and decoupling details out, Section 2.2): a
  block-diagonal W is applied to the
  rows before anything else, and B is built on W A: "quasi-impes" takes
  W_i = I with (0,1) = -D_01/D_11 and (0,2) = -D_02/D_22 (the pressure row
  loses the saturation derivatives of its own diagonal block, using diagonal
  entries only); "abf" (alternate block factorisation) takes W_i = D_i^{-1},
  so W A has identity diagonal blocks.  The preconditioner for A is then
  v -> B_{WA}(W v); the outer FGMRES still works on A.  W is a SETUP product
  (frozen with B).
* ``second_stage="bilu"`` replaces the block-GS sweep by the paper's own R:
  block ILU(0) of A in natural order, applied with level-scheduled
  triangular solves (module ``bilu``).  Its factors are SETUP products, so
  they stay frozen with the rest of B when B is reused.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import amg, bilu, coloring, uaamg
from .sparse import Csr


@dataclass
class Bsr:
    row_ptr: np.ndarray
    col: np.ndarray
    vals: np.ndarray  # [nnz, 3, 3]

    @property
    def n_b(self):
        return int(self.row_ptr.shape[0] - 1)

    @classmethod
    def from_case(cls, case):
        return cls(np.asarray(case.row_ptr, dtype=np.int64), np.asarray(case.col, dtype=np.int64),
                   np.asarray(case.vals, dtype=np.float64))

    def padded(self, rows=None):
        if rows is None:
            rows = np.arange(self.n_b)
        rows = np.asarray(rows, dtype=np.int64)
        start = self.row_ptr[rows]
        length = self.row_ptr[rows + 1] - start
        W = int(length.max()) if rows.size else 0
        t = np.arange(W)[None, :]
        valid = t < length[:, None]
        pos = np.where(valid, start[:, None] + t, 0)
        cols = np.where(valid, self.col[pos], 0)
        vals = np.where(valid[:, :, None, None], self.vals[pos], 0.0)
        return cols, vals, valid

    def to_dense(self):
        n = self.n_b
        d = np.zeros((3 * n, 3 * n))
        for i in range(n):
            for p in range(self.row_ptr[i], self.row_ptr[i + 1]):
                j = self.col[p]
                d[3 * i:3 * i + 3, 3 * j:3 * j + 3] += self.vals[p]
        return d


def bsr_residual(A: Bsr, x, b):
    """r = b - A x with the products subtracted one by one in stored order."""
    cols, vals, _ = A.padded()
    x3 = x.reshape(-1, 3)
    s = b.reshape(-1, 3).astype(x.dtype, copy=True)
    for t in range(cols.shape[1]):
        xj = x3[cols[:, t]]
        blk = vals[:, t].astype(x.dtype)
        for r in range(3):
            for c in range(3):
                s[:, r] = s[:, r] - blk[:, r, c] * xj[:, c]
    return s.reshape(-1)


def bsr_matvec(A: Bsr, x):
    """y = A x accumulated from 0 in stored order (block, then column)."""
    cols, vals, _ = A.padded()
    x3 = x.reshape(-1, 3)
    s = np.zeros((A.n_b, 3), dtype=x.dtype)
    for t in range(cols.shape[1]):
        xj = x3[cols[:, t]]
        blk = vals[:, t].astype(x.dtype)
        for r in range(3):
            for c in range(3):
                s[:, r] = s[:, r] + blk[:, r, c] * xj[:, c]
    return s.reshape(-1)


def pressure_matrix(A: Bsr) -> Csr:
    """A_PP = Pi_P^T A Pi_P: the (0,0) entry of every stored block, same pattern."""
    return Csr(A.n_b, A.n_b, A.row_ptr.copy(), A.col.copy(), A.vals[:, 0, 0].copy())


def restrict_pressure(v):
    return v.reshape(-1, 3)[:, 0].copy()


def prolong_pressure(e):
    z = np.zeros((e.shape[0], 3), dtype=e.dtype)
    z[:, 0] = e
    return z.reshape(-1)


def block_graph(A: Bsr):
    """S_i = {j != i : block (i,j) stored and not all zero}, as lists."""
    S = []
    for i in range(A.n_b):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        S.append([int(j) for j, blk in zip(A.col[a:b], A.vals[a:b]) if j != i and np.any(blk != 0.0)])
    return S


def diag_inverses(A: Bsr):
    """D_i^{-1} for every cell (LAPACK LU with partial pivoting via numpy.linalg.inv)."""
    D = np.empty((A.n_b, 3, 3))
    for i in range(A.n_b):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        hit = np.nonzero(A.col[a:b] == i)[0]
        D[i] = A.vals[a + hit[0]]
    return np.linalg.inv(D)


def block_gs(A: Bsr, colours, Dinv, r):
    """Stage 2: one forward multi-colour block-GS sweep on A d = r from d = 0."""
    dt = r.dtype
    d = np.zeros((A.n_b, 3), dtype=dt)
    r3 = r.reshape(-1, 3)
    for members in colours:
        rows = np.asarray(members, dtype=np.int64)
        cols, vals, _ = A.padded(rows)
        vals = np.where((cols == rows[:, None])[:, :, None, None], 0.0, vals).astype(dt)
        snap = d.copy()
        t3 = r3[rows].copy()
        for t in range(cols.shape[1]):
            dj = snap[cols[:, t]]
            for rr in range(3):
                for c in range(3):
                    t3[:, rr] = t3[:, rr] - vals[:, t, rr, c] * dj[:, c]
        Di = Dinv[rows].astype(dt)
        out = np.zeros_like(t3)
        for rr in range(3):
            for c in range(3):
                out[:, rr] = out[:, rr] + Di[:, rr, c] * t3[:, c]
        d[rows] = out
    return d.reshape(-1)


def decoupling_weights(A: Bsr, kind):
    """W_i per cell for the decoupling ``kind`` ("quasi-impes" or "abf")."""
    D = np.empty((A.n_b, 3, 3))
    for i in range(A.n_b):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        hit = np.nonzero(A.col[a:b] == i)[0]
        D[i] = A.vals[a + hit[0]]
    if kind == "abf":
        return np.linalg.inv(D)
    if kind == "quasi-impes":
        W = np.zeros_like(D)
        W[:, 0, 0] = W[:, 1, 1] = W[:, 2, 2] = 1.0
        W[:, 0, 1] = -D[:, 0, 1] / D[:, 1, 1]
        W[:, 0, 2] = -D[:, 0, 2] / D[:, 2, 2]
        return W
    raise ValueError(kind)


def left_blocks(W, A: Bsr) -> Bsr:
    """W A: every stored block of row i multiplied on the left by W_i, each
    entry sum_m W[r][m] A[m][c] taken from 0 over m = 0, 1, 2."""
    rows = np.repeat(np.arange(A.n_b), np.diff(A.row_ptr))
    Wr = W[rows]
    out = np.zeros_like(A.vals)
    for r in range(3):
        for c in range(3):
            for m in range(3):
                out[:, r, c] = out[:, r, c] + Wr[:, r, m] * A.vals[:, m, c]
    return Bsr(A.row_ptr.copy(), A.col.copy(), out)


def block_gemv(W, v):
    """(W v)_i = W_i v_i, each component summed from 0 over columns 0, 1, 2."""
    v3 = v.reshape(-1, 3)
    out = np.zeros_like(v3)
    for r in range(3):
        for c in range(3):
            out[:, r] = out[:, r] + W[:, r, c] * v3[:, c]
    return out.reshape(-1)


@dataclass
class CprPreconditioner:
    """Everything SETUP produces (frozen while it is reused)."""

    A: Bsr  # the fine matrix as of setup (used inside the CPR apply)
    amg: amg.Hierarchy
    block_colours: list
    Dinv: np.ndarray
    dtype: type = np.float64
    bilu: bilu.BiluFactors | None = None  # set when the second stage is block ILU(0)
    bilu_levels: tuple | None = None      # (forward, backward) level of every row
    W: np.ndarray | None = None           # decoupling weights (B is built on W A)
    cycle: str = "v"                      # "v": RS V-cycle; "amli": UA-AMG nonlinear AMLI-cycle

    def apply(self, v):
        """z = B v (Algorithm CPR method with x = 0)."""
        dt = self.dtype
        v = v.astype(dt)
        if self.W is not None:
            v = block_gemv(self.W.astype(dt), v)
        rp = restrict_pressure(v)
        if self.cycle == "amli":
            e = uaamg.kcycle(self.amg, rp, 0, dt)
        else:
            e = amg.vcycle(self.amg, rp, 0, dt)
        z = prolong_pressure(e.astype(dt))
        Ad = self.A if dt == np.float64 else Bsr(self.A.row_ptr, self.A.col, self.A.vals.astype(dt))
        r = bsr_residual(Ad, z, v)
        if self.bilu is not None:
            F = self.bilu if dt == np.float64 else self.bilu.cast(dt)
            z = z + bilu.solve_by_levels(F, r, *self.bilu_levels)
        else:
            z = z + block_gs(Ad, self.block_colours, self.Dinv, r)
        return z


def setup(A: Bsr, params=None, dtype=np.float64,
          second_stage: str = "bgs", decoupling: str = "none") -> CprPreconditioner:
    """SETUP of B.  params: amg.AmgParams (classical RS AMG, V-cycle; the
    default) or uaamg.UaParams (the paper's UA-AMG with pairwise matching and
    the nonlinear AMLI-cycle); second_stage: "bgs" (multi-colour block
    Gauss-Seidel) or "bilu" (block ILU(0) with level-scheduled solves);
    decoupling: "none", "quasi-impes" or "abf" (B is then built on W A and
    applied to W v)."""
    W = None
    if decoupling != "none":
        W = decoupling_weights(A, decoupling)
        A = left_blocks(W, A)
    cycle = "amli" if isinstance(params, uaamg.UaParams) else "v"
    if cycle == "amli":
        H = uaamg.build_hierarchy(pressure_matrix(A), params)
    else:
        H = amg.build_hierarchy(pressure_matrix(A), params)
    Af = Bsr(A.row_ptr.copy(), A.col.copy(), A.vals.copy())
    if second_stage == "bilu":
        F = bilu.bilu0(Af)
        levels = (bilu.forward_levels(F.row_ptr, F.col), bilu.backward_levels(F.row_ptr, F.col))
        return CprPreconditioner(A=Af, amg=H, block_colours=[], Dinv=F.Uinv, dtype=dtype, bilu=F,
                                 bilu_levels=levels, W=W, cycle=cycle)
    if second_stage != "bgs":
        raise ValueError(second_stage)
    colours = coloring.vertices_grouping(A.n_b, block_graph(A))
    return CprPreconditioner(A=Af, amg=H, block_colours=colours, Dinv=diag_inverses(A), dtype=dtype, W=W,
                             cycle=cycle)
