"""Pins of the oracle's block ILU(0) second stage (oracle/bilu.py).

* No fill on a block-tridiagonal matrix: ILU(0) is the exact block LU, so the
  solve equals a dense direct solve (Saad, ILU(0) on a matrix whose LU has the
  pattern of A).
* ILU(0) defining property: (L U)_ij = A_ij at every stored block (i, j),
  with L unit lower and U upper assembled densely from the factors; off the
  pattern L U differs from A (the dropped fill) on a 2D grid.
* A block-diagonal matrix: the solve is block Jacobi, D^{-1} r.
* Level sets on a full nx x ny x nz 7-point grid in natural order have the
  closed form i + j + k (forward) and (nx-1-i) + (ny-1-j) + (nz-1-k)
  (backward); on masked grids every dependency sits on an earlier level and
  every row above level 0 has one on the level just before (longest path).
* The sparse triangular solves equal dense solves with the assembled L and U
  (L unit lower triangular; U block upper triangular); the level-by-level
  solve equals the sequential one bit for bit.
* CPR with R = (L U)^{-1}: I - B A = (I - R A)(I - Pi_P B_P Pi_P^T A) on
  dense operators (eq. (CPR)).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import bilu, cpr
from workloads import blackoil as bo


def _rand_bsr(n_b, pattern, rng, dominance=4.0):
    """3x3-block matrix with the given per-row column lists, diagonally dominant blocks."""
    rp = [0]
    col = []
    vals = []
    for i in range(n_b):
        cols = sorted(set(pattern[i]) | {i})
        for j in cols:
            blk = rng.uniform(-1, 1, (3, 3))
            if j == i:
                blk += dominance * len(cols) * np.eye(3)
            col.append(j)
            vals.append(blk)
        rp.append(len(col))
    return cpr.Bsr(np.array(rp), np.array(col), np.array(vals))


def _dense_factors(F):
    n = F.n_b
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(F.row_ptr[i], F.row_ptr[i + 1]):
            j = F.col[p]
            if j < i:
                L[3 * i:3 * i + 3, 3 * j:3 * j + 3] = F.LU[p]
            else:
                U[3 * i:3 * i + 3, 3 * j:3 * j + 3] = F.LU[p]
    return L, U


def _grid_case(shape, seed, mask_frac=0.0):
    rng = np.random.default_rng(seed)
    if mask_frac:
        active = bo.random_mask(shape, rng, mask_frac)
    else:
        active = np.ones(shape[0] * shape[1] * shape[2], dtype=bool)
    perm = bo.perm_iid_lognormal(shape, rng, sigma=1.0)
    faces = bo.make_faces(shape, perm, active, 1.0, rng)
    return bo.assemble(shape, active, faces)


def test_block_tridiagonal_is_exact_lu():
    rng = np.random.default_rng(1)
    n = 40
    A = _rand_bsr(n, [[i - 1, i + 1] if 0 < i < n - 1 else ([1] if i == 0 else [n - 2]) for i in range(n)], rng)
    F = bilu.bilu0(A)
    r = rng.standard_normal(3 * n)
    d = bilu.solve(F, r)
    want = np.linalg.solve(A.to_dense(), r)
    assert np.linalg.norm(d - want) <= 1e-13 * np.linalg.norm(want)


def test_lu_equals_a_on_the_pattern_and_drops_fill():
    case = _grid_case((5, 4, 1), 3)
    A = cpr.Bsr.from_case(case)
    F = bilu.bilu0(A)
    L, U = _dense_factors(F)
    LU = L @ U
    Ad = A.to_dense()
    on = np.zeros_like(Ad, dtype=bool)
    for i in range(A.n_b):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col[p]
            on[3 * i:3 * i + 3, 3 * j:3 * j + 3] = True
    scale = np.abs(Ad).max()
    assert np.max(np.abs(LU - Ad)[on]) <= 1e-13 * scale
    # the 2D five-point pattern produces fill at (i, i-nx+1) that ILU(0) drops
    assert np.max(np.abs(LU - Ad)[~on]) > 1e-6 * scale
    # U_ii^{-1} is the inverse of the diagonal block of U
    for i in range(A.n_b):
        assert np.allclose(F.Uinv[i] @ U[3 * i:3 * i + 3, 3 * i:3 * i + 3], np.eye(3), atol=1e-13)


def test_block_diagonal_is_block_jacobi():
    rng = np.random.default_rng(4)
    n = 25
    A = _rand_bsr(n, [[] for _ in range(n)], rng)
    F = bilu.bilu0(A)
    r = rng.standard_normal(3 * n)
    d = bilu.solve(F, r).reshape(-1, 3)
    for i in range(n):
        assert np.allclose(d[i], np.linalg.solve(A.vals[i], r[3 * i:3 * i + 3]), rtol=1e-13, atol=0)


def test_levels_closed_form_on_full_grid():
    shape = (6, 5, 4)
    case = _grid_case(shape, 5)
    nx, ny, nz = shape
    f = bilu.forward_levels(case.row_ptr, case.col)
    b = bilu.backward_levels(case.row_ptr, case.col)
    c = np.arange(nx * ny * nz)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    assert np.array_equal(f, i + j + k)
    assert np.array_equal(b, (nx - 1 - i) + (ny - 1 - j) + (nz - 1 - k))
    assert f.max() + 1 == nx + ny + nz - 2


@pytest.mark.parametrize("seed", [6, 7])
def test_levels_valid_and_longest_path_on_masked_grid(seed):
    case = _grid_case((9, 7, 5), seed, mask_frac=0.1)
    rp, col = case.row_ptr, case.col
    for lev, lower in ((bilu.forward_levels(rp, col), True), (bilu.backward_levels(rp, col), False)):
        for r in range(case.n_b):
            deps = [c for c in col[rp[r]:rp[r + 1]] if (c < r if lower else c > r)]
            assert all(lev[d] < lev[r] for d in deps)
            if deps:
                assert max(lev[d] for d in deps) == lev[r] - 1
            else:
                assert lev[r] == 0


def test_sparse_solves_equal_dense_triangular_solves():
    case = _grid_case((6, 5, 3), 8, mask_frac=0.1)
    A = cpr.Bsr.from_case(case)
    F = bilu.bilu0(A)
    L, U = _dense_factors(F)
    r = np.random.default_rng(9).standard_normal(case.ndof)
    y = scipy.linalg.solve_triangular(L, r, lower=True, unit_diagonal=True)
    # U is block upper triangular with full 3x3 diagonal blocks: a general dense solve
    want = np.linalg.solve(U, y)
    d = bilu.solve(F, r)
    assert np.linalg.norm(d - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_level_schedule_is_bit_identical(dtype):
    case = bo.case_small()
    A = cpr.Bsr.from_case(case)
    F = bilu.bilu0(A).cast(dtype)
    r = np.random.default_rng(10).standard_normal(case.ndof).astype(dtype)
    assert np.array_equal(bilu.solve(F, r), bilu.solve_by_levels(F, r))


def test_cpr_identity_with_bilu_second_stage():
    case = _grid_case((4, 3, 3), 11)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, second_stage="bilu")
    n = 3 * A.n_b
    Bd = np.column_stack([B.apply(e) for e in np.eye(n)])
    Ad = A.to_dense()
    L, U = _dense_factors(B.bilu)
    R = np.linalg.inv(L @ U)
    # stage 1 operator Pi_P B_P Pi_P^T, assembled column by column
    from oracle import amg

    nb = A.n_b
    BP = np.column_stack([amg.vcycle(B.amg, e) for e in np.eye(nb)])
    Pi = np.zeros((n, nb))
    Pi[0::3, :] = np.eye(nb)
    S1 = Pi @ BP @ Pi.T
    I = np.eye(n)
    lhs = I - Bd @ Ad
    rhs = (I - R @ Ad) @ (I - S1 @ Ad)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)
