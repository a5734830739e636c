"""Pins of the oracle's decoupling and of the implicit-well workload.

The full system of the paper's eq. (Jacobian-system) carries the well
unknowns next to the reservoir ones; here each well is an extra 3x3 block row
(workloads.blackoil.add_wells).  Decoupling multiplies the rows by a
block-diagonal W before B is built (oracle.cpr.setup(decoupling=...)).

* ABF: W_i = D_i^{-1}, so every diagonal block of W A is the identity.
* Quasi-IMPES: rows 1 and 2 of W A are those of A, exactly; when the
  saturation part of a diagonal block is diagonal, the pressure row of W D
  is zero in columns 1 and 2 up to the rounding of D_0a / D_aa.
* W A and W v equal the dense products blockdiag(W) A and blockdiag(W) v.
* B_dec = B_{WA} W satisfies eq. (CPR) on W A: I - B_dec A =
  (I - R (W A)) (I - Pi_P B_P Pi_P^T (W A)), with the dense block-GS R and
  V-cycle B_P of W A.
* With wells, the CPR-FGMRES solution equals a dense direct solve within
  cond * tol, for every decoupling; the well rows have zero pressure row sums.
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres
from workloads import blackoil as bo


def _wells_case(shape=(6, 5, 3), seed=3):
    c = bo.case_small(seed=seed, shape=shape)
    return bo.add_wells(c, bo.five_spot(shape), seed + 1)


def _blockdiag(W):
    n = W.shape[0]
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        D[3 * i:3 * i + 3, 3 * i:3 * i + 3] = W[i]
    return D


def test_abf_gives_identity_diagonal_blocks():
    A = cpr.Bsr.from_case(_wells_case())
    WA = cpr.left_blocks(cpr.decoupling_weights(A, "abf"), A)
    for i in range(A.n_b):
        p = A.row_ptr[i] + np.nonzero(A.col[A.row_ptr[i]:A.row_ptr[i + 1]] == i)[0][0]
        assert np.allclose(WA.vals[p], np.eye(3), atol=1e-13, rtol=0)


def test_quasi_impes_rows_and_zeros():
    case = _wells_case(seed=4)
    # make every diagonal block's saturation part diagonal
    rows = np.repeat(np.arange(case.n_b), np.diff(case.row_ptr))
    on = case.col == rows
    case.vals[on, 1, 2] = 0.0
    case.vals[on, 2, 1] = 0.0
    A = cpr.Bsr.from_case(case)
    W = cpr.decoupling_weights(A, "quasi-impes")
    WA = cpr.left_blocks(W, A)
    assert np.array_equal(WA.vals[:, 1:, :], A.vals[:, 1:, :])
    # D_01 - (D_01 / D_11) D_11: zero up to the rounding of the quotient
    eps = np.finfo(float).eps
    for c in (1, 2):
        assert np.all(np.abs(WA.vals[on, 0, c]) <= 4 * eps * np.abs(A.vals[on, 0, c]))


@pytest.mark.parametrize("kind", ["abf", "quasi-impes"])
def test_products_equal_dense(kind):
    A = cpr.Bsr.from_case(_wells_case(seed=5))
    W = cpr.decoupling_weights(A, kind)
    Wd = _blockdiag(W)
    WA = cpr.left_blocks(W, A)
    assert np.allclose(WA.to_dense(), Wd @ A.to_dense(), rtol=0, atol=1e-13 * np.abs(A.to_dense()).max())
    v = np.random.default_rng(6).standard_normal(3 * A.n_b)
    assert np.allclose(cpr.block_gemv(W, v), Wd @ v, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["abf", "quasi-impes"])
def test_cpr_identity_on_the_decoupled_matrix(kind):
    case = _wells_case(shape=(5, 4, 2), seed=7)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, decoupling=kind)
    n = 3 * A.n_b
    Ad = A.to_dense()
    WAd = _blockdiag(B.W) @ Ad
    Bd = np.column_stack([B.apply(e) for e in np.eye(n)])
    # R: the block-GS sweep of W A, assembled column by column
    WA = cpr.left_blocks(B.W, A)
    R = np.column_stack([cpr.block_gs(WA, B.block_colours, B.Dinv, e) for e in np.eye(n)])
    nb = A.n_b
    BP = np.column_stack([amg.vcycle(B.amg, e) for e in np.eye(nb)])
    Pi = np.zeros((n, nb))
    Pi[0::3, :] = np.eye(nb)
    I = np.eye(n)
    lhs = I - Bd @ Ad
    rhs = (I - R @ WAd) @ (I - Pi @ BP @ Pi.T @ WAd)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)


@pytest.mark.parametrize("kind", ["none", "quasi-impes", "abf"])
def test_solve_with_wells_equals_dense(kind):
    case = _wells_case(shape=(7, 6, 4), seed=8)
    A = cpr.Bsr.from_case(case)
    b = bo.rhs(case.ndof, 9)
    B = cpr.setup(A, decoupling=kind)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-10)
    Ad = A.to_dense()
    x = np.linalg.solve(Ad, b)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= np.linalg.cond(Ad) * 1e-10 * np.linalg.norm(x)


def test_well_rows():
    case = _wells_case(seed=10)
    n_cells = case.n_b - 5
    for w in range(5):
        i = n_cells + w
        blk = case.vals[case.row_ptr[i]:case.row_ptr[i + 1]]
        cols = case.col[case.row_ptr[i]:case.row_ptr[i + 1]]
        assert cols[-1] == i and np.all(cols[:-1] < n_cells)
        assert abs(blk[:, 0, 0].sum()) <= 1e-12 * blk[-1, 0, 0]
        assert np.array_equal(blk[-1, 1:, 1:], np.eye(2))
        assert len(cols) - 1 == case.grid[2]  # every layer of the column is active
