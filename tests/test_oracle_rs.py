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
