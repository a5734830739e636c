"""Pins of the oracle's classical RS coarsening, interpolation and Galerkin product.

Closed forms: on 1D tridiag(-1, 2, -1) the split takes every odd index
(0-based) as C, interpolation is linear (weights 1/2) and the interior
coarse operator is (1/2) tridiag(-1, 2, -1).  On the 3D 7-point Laplacian
(6, -1) the interior coarse row of a red-black split is 5 on the diagonal,
-1/6 at the six points two steps along an axis and -1/3 at the twelve face
diagonals.  Invariants: every F point with strong dependencies has a strong C
dependency and every strongly coupled F-F pair shares a C point of the
interpolation set; symmetric A gives symmetric A_c; the Galerkin product
agrees with the dense triple product.
"""
import numpy as np

from oracle import rs, strength
from oracle.sparse import csr_from_dense, pattern_lists


def _split(A, theta=0.25):
    mask, (ip, ix) = strength.rs_strength(A, theta)
    S = pattern_lists(ip, ix)
    ST = [[] for _ in range(A.n_rows)]
    for i in range(A.n_rows):
        for j in S[i]:
            ST[j].append(i)
    return mask, S, rs.rs_split(A.n_rows, S, ST)


def _lap1d(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def _lap3d(n):
    N = n ** 3
    d = np.zeros((N, N))
    idx = lambda i, j, k: i + n * (j + n * k)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = idx(i, j, k)
                d[r, r] = 6
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    a, b, c = i + di, j + dj, k + dk
                    if 0 <= a < n and 0 <= b < n and 0 <= c < n:
                        d[r, idx(a, b, c)] = -1
    return d


def test_1d_split_interp_and_coarse_operator():
    n = 15
    A = csr_from_dense(_lap1d(n))
    mask, S, cf = _split(A)
    assert list(np.nonzero(cf == rs.C)[0]) == list(range(1, n, 2))
    P = rs.interpolation(A, mask, cf)
    Pd = P.to_dense()
    for i in range(0, n, 2):  # F points: weights 1/2 to each C neighbour
        nbrs = [j for j in (i - 1, i + 1) if 0 <= j < n]
        for j in nbrs:
            assert Pd[i, (j - 1) // 2] == 0.5
    R, Ac = rs.galerkin(A, P)
    Acd = Ac.to_dense()
    nc = Acd.shape[0]
    for I in range(1, nc - 1):
        assert Acd[I, I] == 1.0 and Acd[I, I - 1] == -0.5 and Acd[I, I + 1] == -0.5


def test_3d_red_black_interior_coarse_stencil():
    n = 7
    d = _lap3d(n)
    A = csr_from_dense(d)
    mask, S, cf = _split(A)
    idx = lambda i, j, k: i + n * (j + n * k)
    # interior parity pattern of the split
    interior = [(i, j, k) for i in range(1, n - 1) for j in range(1, n - 1) for k in range(1, n - 1)]
    par = {(i + j + k) % 2: set() for (i, j, k) in interior}
    for (i, j, k) in interior:
        par[(i + j + k) % 2].add(int(cf[idx(i, j, k)]))
    assert all(len(v) == 1 for v in par.values()) and par[0] != par[1]
    P = rs.interpolation(A, mask, cf)
    R, Ac = rs.galerkin(A, P)
    Pd, Acd = P.to_dense(), Ac.to_dense()
    assert np.allclose(Acd, Pd.T @ d @ Pd, rtol=0, atol=1e-13)
    coarse = -np.ones(n ** 3, dtype=int)
    cpts = np.nonzero(cf == rs.C)[0]
    coarse[cpts] = np.arange(cpts.size)
    c0 = (3, 3, 3) if cf[idx(3, 3, 3)] == rs.C else (3, 3, 2)
    I = coarse[idx(*c0)]
    row = Acd[I]
    assert abs(row[I] - 5.0) < 1e-14
    for ax in range(3):
        for sgn in (-1, 1):
            p = list(c0)
            p[ax] += 2 * sgn
            assert abs(row[coarse[idx(*p)]] + 1 / 6) < 1e-14
    for a1 in range(3):
        for a2 in range(a1 + 1, 3):
            for s1 in (-1, 1):
                for s2 in (-1, 1):
                    p = list(c0)
                    p[a1] += s1
                    p[a2] += s2
                    assert abs(row[coarse[idx(*p)]] + 1 / 3) < 1e-14
    assert abs(row.sum()) < 1e-13


def test_split_invariants_on_random_m_matrices():
    rng = np.random.default_rng(5)
    for trial in range(30):
        n = int(rng.integers(10, 60))
        off = -(rng.uniform(size=(n, n)) < 0.15).astype(float) * rng.uniform(0.1, 1.0, size=(n, n))
        off = off + off.T
        np.fill_diagonal(off, 0)
        d = off + np.diag(-off.sum(axis=1) + rng.uniform(0.01, 0.1, size=n))
        A = csr_from_dense(d)
        mask, S, cf = _split(A)
        assert set(np.unique(cf)) <= {rs.C, rs.F}
        for i in range(n):
            if cf[i] != rs.F or not S[i]:
                continue
            Ci = {j for j in S[i] if cf[j] == rs.C}
            assert Ci, "F point without strong C dependency"
            for j in S[i]:
                if cf[j] == rs.F:
                    assert set(S[j]) & Ci, "strong F-F pair without common C point"
        P = rs.interpolation(A, mask, cf)
        R, Ac = rs.galerkin(A, P)
        Acd = Ac.to_dense()
        Pd = P.to_dense()
        assert np.allclose(Acd, Pd.T @ d @ Pd, rtol=1e-13, atol=1e-14)
        assert np.allclose(Acd, Acd.T, rtol=1e-13, atol=1e-14)
        # interpolation reproduces constants where rows of A sum to ~0 only
        # approximately; check the weights are positive for M-matrices
        assert (P.data > 0).all()


# ---------------------------------------------------------------------------
# Hand-derived classical interpolation with strong F-F couplings.
#
# Six points; the C/F state and the strength pattern are given by hand (the
# interpolation formula is pinned on its own, independent of the split):
#   F = {0, 1, 5}, C = {2, 3, 4} (coarse indices 0, 1, 2).
# Row 0: a00 = 10, a01 = -2 (strong, F), a02 = -3 (strong, C), a03 = -1
#        (strong, C), a04 = -0.5 (weak), a05 = -1.5 (strong, F).
# Row 1: a10 = -1 (strong, F), a11 = 8, a12 = -4, a13 = -2 (strong, C).
# Row 5: a50 = -1 (strong, F), a54 = -2 (strong, C), a55 = 4.
# Rows 2-4 (C points) carry entries that a transposed index would pick up.
#
# Textbook RS interpolation (Briggs, Henson, McCormick, ch. 8):
#   w_ij = -(a_ij + sum_{m strong F} a_im a_mj / sum_{k in C_i} a_mk)
#          / (a_ii + sum_{n weak} a_in)
# with a strong F neighbour that meets no point of C_i lumped into the
# diagonal.  Worked by hand:
#   row 0: C_0 = {2, 3}.  m = 1: denominator a12 + a13 = -6, so
#          num_2 = -3 + (-2)(-4)/(-6) = -13/3, num_3 = -1 + (-2)(-2)/(-6) = -5/3.
#          m = 5 meets neither 2 nor 3 (denominator 0): lumped.
#          d = 10 - 0.5 - 1.5 = 8, so w_02 = 13/24, w_03 = 5/24.
#   row 1: C_1 = {2, 3}.  m = 0: denominator a02 + a03 = -4, so
#          num_2 = -4 + (-1)(-3)/(-4) = -19/4, num_3 = -2 + (-1)(-1)/(-4) = -9/4;
#          d = 8, so w_12 = 19/32, w_13 = 9/32.
#   row 5: C_5 = {4}.  m = 0: denominator a04 = -1/2, so
#          num_4 = -2 + (-1)(-1/2)/(-1/2) = -3; d = 4, so w_54 = 3/4.
# Lumping every strong F neighbour instead (row 0: d = 6) gives w_02 = 1/2;
# reading a_km for a_mk, or summing the denominator over all of row m, also
# changes these weights.
# ---------------------------------------------------------------------------
from fractions import Fraction as Q  # noqa: E402

from oracle.sparse import Csr  # noqa: E402

_HAND_ROWS = {
    0: [(0, 10.0), (1, -2.0), (2, -3.0), (3, -1.0), (4, -0.5), (5, -1.5)],
    1: [(0, -1.0), (1, 8.0), (2, -4.0), (3, -2.0)],
    2: [(0, -1.1), (1, -0.7), (2, 5.0), (4, -1.0)],
    3: [(0, -0.9), (1, -1.3), (3, 6.0)],
    4: [(0, -0.2), (2, -1.5), (4, 3.0), (5, -0.25)],
    5: [(0, -1.0), (4, -2.0), (5, 4.0)],
}
# strong dependencies of the F rows (C rows are never interpolated)
_HAND_STRONG = {0: {1, 2, 3, 5}, 1: {0, 2, 3}, 5: {0, 4}}
_HAND_STATE = [rs.F, rs.F, rs.C, rs.C, rs.C, rs.F]
_HAND_P = {  # row -> {coarse column: exact weight}
    0: {0: Q(13, 24), 1: Q(5, 24)},
    1: {0: Q(19, 32), 1: Q(9, 32)},
    2: {0: Q(1)},
    3: {1: Q(1)},
    4: {2: Q(1)},
    5: {2: Q(3, 4)},
}


def hand_case():
    """The hand-built matrix, its strength mask and C/F state (also used by the C++ check)."""
    indptr, indices, data, mask = [0], [], [], []
    for i in range(6):
        for j, v in _HAND_ROWS[i]:
            indices.append(j)
            data.append(v)
            mask.append(j in _HAND_STRONG.get(i, set()))
        indptr.append(len(indices))
    A = Csr(6, 6, np.array(indptr, dtype=np.int64), np.array(indices, dtype=np.int64),
            np.array(data, dtype=np.float64))
    return A, np.array(mask, dtype=bool), np.array(_HAND_STATE, dtype=np.int8)


def hand_expected_dense():
    P = np.zeros((6, 3))
    for i, row in _HAND_P.items():
        for J, w in row.items():
            P[i, J] = float(w)
    return P


def test_interpolation_strong_f_neighbours_hand_derived():
    A, mask, state = hand_case()
    # the hand-given strength pattern is what classical RS strength gives at 0.25
    rs_mask, _ = strength.rs_strength(A, 0.25)
    for i in (0, 1, 5):
        a, b = A.indptr[i], A.indptr[i + 1]
        assert list(rs_mask[a:b]) == list(mask[a:b])
    P = rs.interpolation(A, mask, state)
    assert P.n_cols == 3
    want = hand_expected_dense()
    got = P.to_dense()
    assert np.allclose(got, want, rtol=4e-16, atol=0.0), (got, want)
    # every weight within one rounding of the exact rational
    for i, row in _HAND_P.items():
        for J, w in row.items():
            assert abs(Q(got[i, J]) - w) <= abs(w) * Q(1, 2 ** 51)
