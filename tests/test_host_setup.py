"""The library's host-side SETUP routines against the oracle, bit for bit (CPU).

The strength patterns fed to both sides come from the oracle; the library's
VerticesGrouping, RS split, interpolation and Galerkin product must then give
exactly the oracle's colours, C/F split, weights and coarse matrix.  Also
checks that the shared library exports every symbol the headers declare.
"""
import os
import re

import numpy as np
import pytest

from oracle import coloring, rs, strength
from oracle.cpr import Bsr, pressure_matrix
from oracle.sparse import pattern_lists
from workloads import blackoil as bo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2201_01970_amd", "libcpr_mi355x.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")


def _declared_symbols():
    names = set()
    for h in ("cpr.h", "cpr_inspect.h", "cpr_serve.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cpr_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    import ctypes

    lib = ctypes.CDLL(LIB)
    names = _declared_symbols()
    assert len(names) >= 20
    for name in sorted(names):
        assert hasattr(lib, name), name
    from paper_2201_01970_amd import _capi

    assert set(_capi.SIGNATURES) == names


def _levels_of(case_shape, seed, theta_rs=0.25):
    """A chain of oracle levels (A, rs mask, S lists, cf, P) of a generated case."""
    from oracle import amg

    case = bo.case_spe10_like(seed=seed, shape=case_shape, inactive_frac=0.05)
    H = amg.build_hierarchy(pressure_matrix(Bsr.from_case(case)), amg.AmgParams(theta_rs=theta_rs))
    return H


def _csr32(A):
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data


def test_grouping_bit_exact():
    from paper_2201_01970_amd import host_grouping

    H = _levels_of((14, 12, 6), 51)
    for lev in H.levels[:-1]:
        for theta in (0.0, 0.05, 0.3):
            _, (ip, ix) = strength.color_strength(lev.A, theta)
            want = coloring.colour_array(lev.A.n_rows, coloring.vertices_grouping(lev.A.n_rows,
                                                                                   pattern_lists(ip, ix)))
            got, nc = host_grouping(ip, ix)
            assert nc == want.max() + 1
            assert np.array_equal(got, want)
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        d = (rng.uniform(size=(n, n)) < rng.uniform(0.02, 0.4))
        np.fill_diagonal(d, False)
        S = [list(np.nonzero(d[i])[0]) for i in range(n)]
        ip = np.concatenate([[0], np.cumsum([len(s) for s in S])])
        ix = np.array([j for s in S for j in s], dtype=np.int64)
        want = coloring.colour_array(n, coloring.vertices_grouping(n, S))
        got, _ = host_grouping(ip, ix)
        assert np.array_equal(got, want)


def test_rs_split_interp_galerkin_bit_exact():
    from paper_2201_01970_amd import host_galerkin, host_interpolation, host_rs_split

    for shape, seed in (((14, 12, 6), 52), ((20, 9, 7), 53)):
        H = _levels_of(shape, seed)
        assert H.n_levels >= 3
        for lev in H.levels[:-1]:
            A = lev.A
            mask, (ip, ix) = strength.rs_strength(A, 0.25)
            cf = host_rs_split(ip, ix)
            assert np.array_equal(cf, lev.cf)
            p_ptr, p_col, p_val, nc = host_interpolation(*_csr32(A), mask.astype(np.uint8), cf)
            assert nc == lev.P.n_cols
            assert np.array_equal(p_ptr, lev.P.indptr)
            assert np.array_equal(p_col, lev.P.indices)
            assert np.array_equal(p_val, lev.P.data)  # bit for bit
            Ac_ptr, Ac_col, Ac_val = host_galerkin(*_csr32(A), p_ptr, p_col, p_val, nc)
            nxt = H.levels[H.levels.index(lev) + 1].A
            assert np.array_equal(Ac_ptr, nxt.indptr)
            assert np.array_equal(Ac_col, nxt.indices)
            assert np.array_equal(Ac_val, nxt.data)


def test_rs_split_random_graphs_bit_exact():
    from paper_2201_01970_amd import host_rs_split

    rng = np.random.default_rng(4)
    for _ in range(300):
        n = int(rng.integers(1, 50))
        d = rng.uniform(size=(n, n)) < rng.uniform(0.02, 0.3)
        np.fill_diagonal(d, False)
        S = [list(np.nonzero(d[i])[0]) for i in range(n)]
        ST = [[] for _ in range(n)]
        for i in range(n):
            for j in S[i]:
                ST[j].append(i)
        want = rs.rs_split(n, S, ST)
        ip = np.concatenate([[0], np.cumsum([len(s) for s in S])])
        ix = np.array([j for s in S for j in s], dtype=np.int64)
        got = host_rs_split(ip, ix)
        assert np.array_equal(got, want)


def test_interpolation_hand_derived_strong_f_neighbours():
    """The library's RS interpolation on the hand-worked case of test_oracle_rs:
    equal to the oracle bit for bit and to the exact rational weights."""
    from paper_2201_01970_amd import host_interpolation
    from test_oracle_rs import hand_case, hand_expected_dense

    A, mask, state = hand_case()
    p_ptr, p_col, p_val, nc = host_interpolation(*_csr32(A), mask.astype(np.uint8), state)
    P = rs.interpolation(A, mask, state)
    assert nc == 3
    assert np.array_equal(p_ptr, P.indptr)
    assert np.array_equal(p_col, P.indices)
    assert np.array_equal(p_val, P.data)
    got = np.zeros((6, 3))
    for i in range(6):
        for k in range(p_ptr[i], p_ptr[i + 1]):
            got[i, p_col[k]] = p_val[k]
    assert np.allclose(got, hand_expected_dense(), rtol=4e-16, atol=0.0)


@pytest.mark.parametrize("shape,wells", [((9, 7, 4), False), ((6, 5, 3), True)], ids=["grid", "wells"])
def test_host_bilu0_matches_oracle(shape, wells):
    """The library's block ILU(0) against the oracle's: the same level sets
    exactly; factors within rounding (both run the IKJ algorithm in the same
    order, but the oracle forms 3x3 products and inverses with NumPy/LAPACK);
    and the oracle's level-scheduled solve on the library's factors equals its
    sequential solve on its own factors within 1e-13."""
    import ctypes as C

    from oracle import bilu
    from paper_2201_01970_amd import _capi

    case = bo.case_spe10_like(seed=77, shape=shape, inactive_frac=0.05)
    if wells:
        case = bo.add_wells(case, bo.five_spot(shape), 78)
    A = Bsr.from_case(case)
    F = bilu.bilu0(A)
    n, nnz = case.n_b, case.nnz_b
    rp = np.ascontiguousarray(case.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(case.col, dtype=np.int32)
    vals = np.ascontiguousarray(case.vals.reshape(-1), dtype=np.float64)
    lu = np.empty(nnz * 9)
    uinv = np.empty(n * 9)
    flev = np.empty(n, dtype=np.int32)
    blev = np.empty(n, dtype=np.int32)
    lib = _capi.lib()
    st = lib.cpr_host_bilu0(n, rp.ctypes.data, col.ctypes.data, vals.ctypes.data, lu.ctypes.data,
                            uinv.ctypes.data, flev.ctypes.data, blev.ctypes.data)
    assert st == 0
    assert np.array_equal(flev, bilu.forward_levels(F.row_ptr, F.col))
    assert np.array_equal(blev, bilu.backward_levels(F.row_ptr, F.col))
    lu = lu.reshape(-1, 3, 3)
    uinv = uinv.reshape(-1, 3, 3)
    scale = np.abs(F.LU).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(lu - F.LU) <= 1e-12 * scale)
    assert np.allclose(uinv, F.Uinv, rtol=1e-12, atol=1e-12 * np.abs(F.Uinv).max())
    Fd = bilu.BiluFactors(F.row_ptr, F.col, lu, uinv, F.diag_pos)
    r = bo.rhs(case.ndof, 79)
    want = bilu.solve(F, r)
    got = bilu.solve_by_levels(Fd, r)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_host_bilu0_reports_singular_pivot():
    from paper_2201_01970_amd import _capi

    case = bo.case_small(seed=5, shape=(3, 3, 2))
    vals = np.array(case.vals, dtype=np.float64)
    rows = np.repeat(np.arange(case.n_b), np.diff(case.row_ptr))
    diag = np.nonzero(case.col == rows)[0]
    vals[diag[0]] = 0.0  # row 0 has no lower neighbour: U_00 = A_00
    n, nnz = case.n_b, case.nnz_b
    rp = np.ascontiguousarray(case.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(case.col, dtype=np.int32)
    flat = np.ascontiguousarray(vals.reshape(-1))
    out = [np.empty(nnz * 9), np.empty(n * 9), np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int32)]
    st = _capi.lib().cpr_host_bilu0(n, rp.ctypes.data, col.ctypes.data, flat.ctypes.data,
                                    *[o.ctypes.data for o in out])
    assert st == _capi.CPR_ERR_SINGULAR_BLOCK


def _host_aggregates(A, beta=0.25, npair=2):
    from paper_2201_01970_amd import _capi

    n = A.n_rows
    ptr, col, val = (np.ascontiguousarray(A.indptr, dtype=np.int32), np.ascontiguousarray(A.indices, dtype=np.int32),
                     np.ascontiguousarray(A.data, dtype=np.float64))
    agg = np.empty(n, dtype=np.int32)
    na = np.zeros(1, dtype=np.int32)
    st = _capi.lib().cpr_host_aggregates(n, ptr.ctypes.data, col.ctypes.data, val.ctypes.data, beta, npair,
                                         agg.ctypes.data, na.ctypes.data)
    assert st == 0
    return agg, int(na[0])


@pytest.mark.parametrize("npair", [1, 2])
@pytest.mark.parametrize("which", ["spe10", "channels", "decoupled", "random"])
def test_host_aggregates_match_oracle(which, npair):
    """The library's pairwise matching gives exactly the oracle's aggregates
    (same pairs, same numbering), on pressure matrices of the generated
    workloads, a quasi-IMPES-decoupled one (non-symmetric, positive entries)
    and random non-symmetric matrices, for one and two passes."""
    from oracle import cpr as ocpr
    from oracle import uaamg
    from oracle.sparse import csr_from_dense

    if which == "spe10":
        A = pressure_matrix(Bsr.from_case(bo.case_spe10_like(seed=91, shape=(14, 12, 6))))
    elif which == "channels":
        A = pressure_matrix(Bsr.from_case(bo.case_channels(seed=92, shape=(16, 16, 6))))
    elif which == "decoupled":
        B = Bsr.from_case(bo.case_small(seed=93, shape=(10, 9, 4)))
        A = pressure_matrix(ocpr.left_blocks(ocpr.decoupling_weights(B, "quasi-impes"), B))
    else:
        rng = np.random.default_rng(94)
        d = rng.standard_normal((60, 60)) * (rng.random((60, 60)) < 0.1)
        np.fill_diagonal(d, 5.0)
        A = csr_from_dense(d)
    want, nw = uaamg.npair_aggregates(A, 0.25, npair)
    got, ng = _host_aggregates(A, 0.25, npair)
    assert ng == nw
    assert np.array_equal(got, want)


def test_host_aggregates_match_oracle_at_block_parallel_size():
    """87,750 pressure rows with 588,528 stored entries: large enough that the
    library's transpose (inside the matching's symmetric part) splits its rows
    into two blocks and the strong sets are built over 42 row chunks.  The
    symmetric merge needs every transposed row in ascending column order, so
    the aggregates equal the oracle's only if the block-parallel transpose
    keeps that order."""
    from oracle import uaamg

    A = pressure_matrix(Bsr.from_case(bo.case_spe10_like(seed=95, shape=(60, 60, 25))))
    assert A.indptr[-1] > 2 * 262144
    want, nw = uaamg.npair_aggregates(A, 0.25, 2)
    got, ng = _host_aggregates(A, 0.25, 2)
    assert ng == nw
    assert np.array_equal(got, want)
