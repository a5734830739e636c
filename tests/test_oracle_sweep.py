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
