"""Pins of the oracle's PGS-SCM colour sweep (Section 5.2, Algorithm PGS-SCM).

* With a theta = 0 colouring, one colour sweep equals a plain sequential
  forward Gauss-Seidel sweep over the rows in colour-concatenated order,
  bit for bit (no two rows of a colour are coupled).
* n singleton colours in natural order give classical Gauss-Seidel, the case
  c = n named in Section 5.1.
* One colour holding every row gives Jacobi (the snapshot reading).
The references below are written as plain per-row loops over the stored
entries, not through the oracle's padded vector code.
"""
import numpy as np
import scipy.linalg

from oracle import amg, coloring, strength
from oracle.cpr import Bsr, pressure_matrix
from oracle.sparse import pattern_lists
from workloads import blackoil as bo


def _gs_rows(A, order, x, b):
    for i in order:
        s = b[i]
        diag = None
        for p in range(A.indptr[i], A.indptr[i + 1]):
            j, a = A.indices[p], A.data[p]
            if j == i:
                diag = a
            else:
                s = s - a * x[j]
        x[i] = s / diag
    return x


def _jacobi(A, x, b):
    old = x.copy()
    for i in range(A.n_rows):
        s = b[i]
        for p in range(A.indptr[i], A.indptr[i + 1]):
            j, a = A.indices[p], A.data[p]
            if j == i:
                diag = a
            else:
                s = s - a * old[j]
        x[i] = s / diag
    return x


def _case_pressure(shape=(9, 7, 4), seed=21):
    case = bo.case_spe10_like(seed=seed, shape=shape, inactive_frac=0.05)
    return pressure_matrix(Bsr.from_case(case))


def test_theta0_sweep_is_sequential_gs_in_colour_order_bitwise():
    A = _case_pressure()
    _, (ip, ix) = strength.color_strength(A, 0.0)
    colours = coloring.vertices_grouping(A.n_rows, pattern_lists(ip, ix))
    rng = np.random.default_rng(1)
    b = rng.standard_normal(A.n_rows)
    x0 = rng.standard_normal(A.n_rows)
    got = amg.colour_sweep(A, colours, x0.copy(), b)
    want = _gs_rows(A, [v for c in colours for v in c], x0.copy(), b)
    assert np.array_equal(got, want)


def test_singleton_colours_are_classical_gs():
    A = _case_pressure(seed=22)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(A.n_rows)
    x0 = rng.standard_normal(A.n_rows)
    got = amg.colour_sweep(A, [[i] for i in range(A.n_rows)], x0.copy(), b)
    want = _gs_rows(A, range(A.n_rows), x0.copy(), b)
    assert np.array_equal(got, want)


def test_single_colour_is_jacobi():
    A = _case_pressure(seed=23)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.n_rows)
    x0 = rng.standard_normal(A.n_rows)
    got = amg.colour_sweep(A, [list(range(A.n_rows))], x0.copy(), b)
    want = _jacobi(A, x0.copy(), b)
    assert np.array_equal(got, want)


def test_theta_positive_sweep_reduces_error_on_spd_pressure():
    A = _case_pressure(seed=24)
    _, (ip, ix) = strength.color_strength(A, 0.05)
    colours = coloring.vertices_grouping(A.n_rows, pattern_lists(ip, ix))
    d = A.to_dense()
    rng = np.random.default_rng(4)
    xs = rng.standard_normal(A.n_rows)
    b = d @ xs
    x = np.zeros(A.n_rows)
    e0 = np.sqrt((xs - x) @ d @ (xs - x))
    for _ in range(3):
        amg.colour_sweep(A, colours, x, b)
    e1 = np.sqrt((xs - x) @ d @ (xs - x))
    assert e1 < e0


# ---- PGS-NO (natural-order chunks; the paper's reference smoother) ----------
def test_pgs_no_one_chunk_is_classical_gs_bitwise():
    A = _case_pressure(seed=25)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A.n_rows)
    x0 = rng.standard_normal(A.n_rows)
    got = amg.natural_chunk_sweep(A, 1, x0.copy(), b)
    want = _gs_rows(A, range(A.n_rows), x0.copy(), b)
    assert np.array_equal(got, want)


def test_pgs_no_one_row_per_chunk_is_jacobi_bitwise():
    A = _case_pressure(seed=26)
    rng = np.random.default_rng(6)
    b = rng.standard_normal(A.n_rows)
    x0 = rng.standard_normal(A.n_rows)
    got = amg.natural_chunk_sweep(A, A.n_rows, x0.copy(), b)
    want = _jacobi(A, x0.copy(), b)
    assert np.array_equal(got, want)


def test_pgs_no_chunk_bounds():
    for n, c in ((10, 3), (10, 10), (10, 40), (1, 5), (4096, 4096), (100003, 4096)):
        bnd = amg.chunk_bounds(n, c)
        sizes = np.diff(bnd)
        assert bnd[0] == 0 and bnd[-1] == n
        assert len(sizes) == min(c, n)
        assert sizes.max() - sizes.min() <= 1 and np.all(sizes[:-1] >= sizes[1:])


def test_pgs_no_is_block_jacobi_with_gs_blocks():
    """x_new = M^{-1} (b - (A - M) x), M = the lower triangle (diagonal
    included) of the chunk-diagonal part of A: the splitting the sweep
    implements, solved densely."""
    A = _case_pressure(seed=27)
    n = A.n_rows
    d = A.to_dense()
    rng = np.random.default_rng(7)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    for chunks in (2, 5, 17):
        bnd = amg.chunk_bounds(n, chunks)
        M = np.zeros_like(d)
        for lo, hi in zip(bnd[:-1], bnd[1:]):
            M[lo:hi, lo:hi] = np.tril(d[lo:hi, lo:hi])
        want = scipy.linalg.solve_triangular(M, b - (d - M) @ x0, lower=True)
        got = amg.natural_chunk_sweep(A, chunks, x0.copy(), b)
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
        # and it is neither plain GS nor Jacobi
        gs = _gs_rows(A, range(n), x0.copy(), b)
        assert np.linalg.norm(got - gs) > 1e-8 * np.linalg.norm(gs)


def test_pgs_no_vcycle_converges_and_drifts_with_chunks():
    """As a smoother inside the V-cycle: a CPR solve converges for any chunk
    count, and the iteration count depends on it (the drift the paper reports
    for PGS-NO as the thread count grows), while PGS-SCM's does not change."""
    from oracle import cpr, fgmres

    case = bo.case_small()
    A = cpr.Bsr.from_case(case)
    b = bo.rhs(case.ndof, 1001)
    its = {}
    for chunks in (1, 64, 2000):
        B = cpr.setup(A, amg.AmgParams(smoother="pgs-no", gs_chunks=chunks))
        res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-8)
        assert res.converged
        its[chunks] = res.iterations
    assert its[1] <= its[2000]
    assert len(set(its.values())) > 1
