"""Pins of the oracle's CPR apply (Section 3.1, eq. (CPR) and Algorithm CPR method).

* Identity: with B assembled column by column from the oracle's apply,
  I - B A equals (I - R A)(I - Pi_P B_P Pi_P^T A), where R is the dense
  forward block Gauss-Seidel operator (D + L)^{-1} in block-colour order and
  B_P the pressure V-cycle operator.
* Special case: with zero pressure/saturation couplings and a direct
  pressure solve (single-level hierarchy), stage 1 solves the pressure block
  exactly and stage 2 leaves it unchanged.
* The block colouring of a 7-point grid has 2 colours (bipartite graph).
* The block residual and product agree with the dense matrix.
"""
import numpy as np

from oracle import amg, cpr
from workloads import blackoil as bo


def _small_case(shape=(4, 3, 3), seed=31, frac=0.0):
    rng = np.random.default_rng(seed)
    perm = bo.perm_iid_lognormal(shape, rng, sigma=1.5)
    active = bo.random_mask(shape, rng, frac)
    case = bo.assemble(shape, active, bo.make_faces(shape, perm, active, 0.5, rng))
    return cpr.Bsr.from_case(case)


def _operator(f, n):
    return np.column_stack([f(np.eye(n)[:, k]) for k in range(n)])


def test_bsr_products_match_dense():
    A = _small_case(shape=(5, 4, 3), frac=0.1)
    d = A.to_dense()
    rng = np.random.default_rng(2)
    x = rng.standard_normal(3 * A.n_b)
    b = rng.standard_normal(3 * A.n_b)
    assert np.allclose(cpr.bsr_matvec(A, x), d @ x, rtol=1e-14, atol=1e-16)
    assert np.allclose(cpr.bsr_residual(A, x, b), b - d @ x, rtol=1e-14, atol=1e-15)


def test_cpr_error_propagation_identity():
    A = _small_case()
    n = 3 * A.n_b
    d = A.to_dense()
    B = cpr.setup(A, amg.AmgParams(coarse_max=8))
    assert B.amg.n_levels >= 2
    Bm = _operator(B.apply, n)
    # dense stage-2 operator: forward block GS in block-colour order
    order = [v for c in B.block_colours for v in c]
    perm = np.concatenate([[3 * v, 3 * v + 1, 3 * v + 2] for v in order])
    Pm = np.eye(n)[perm]
    Ap = Pm @ d @ Pm.T
    M = np.zeros_like(Ap)
    for bi in range(A.n_b):
        M[3 * bi:3 * bi + 3, :3 * bi + 3] = Ap[3 * bi:3 * bi + 3, :3 * bi + 3]
    Rm = Pm.T @ np.linalg.inv(M) @ Pm
    BPm = _operator(lambda v: amg.vcycle(B.amg, v), A.n_b)
    Pi = np.zeros((n, A.n_b))
    Pi[np.arange(0, n, 3), np.arange(A.n_b)] = 1.0
    I = np.eye(n)
    lhs = I - Bm @ d
    rhs_ = (I - Rm @ d) @ (I - Pi @ BPm @ Pi.T @ d)
    assert np.abs(lhs - rhs_).max() < 1e-12 * np.abs(lhs).max()


def test_stage1_exact_on_decoupled_pressure():
    A = _small_case(shape=(5, 3, 2), seed=33)
    v = A.vals.copy()
    v[:, 0, 1:] = 0.0
    v[:, 1:, 0] = 0.0
    A = cpr.Bsr(A.row_ptr, A.col, v)
    B = cpr.setup(A, amg.AmgParams(coarse_max=10 ** 6))
    assert B.amg.n_levels == 1
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal(3 * A.n_b)
    z = B.apply(rhs)
    App = cpr.pressure_matrix(A).to_dense()
    want = np.linalg.solve(App, rhs[0::3])
    assert np.allclose(z[0::3], want, rtol=1e-12, atol=1e-14)


def test_block_colouring_two_colours_on_grid():
    A = _small_case(shape=(7, 6, 4), frac=0.15, seed=34)
    B = cpr.setup(A)
    assert len(B.block_colours) == 2
