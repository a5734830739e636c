"""Pins of the oracle's UA-AMG (pairwise matching, NPAIR, nonlinear AMLI-cycle).

Section 6 names the paper's B_P: unsmoothed aggregation with non-symmetric
pairwise matching and the nonlinear AMLI-cycle.  The pins:
* 1D Laplacian (closed form): one pass pairs {2k, 2k+1}, two passes give
  {4k..4k+3}, and the coarse matrix is again tridiag(-1, 2, -1), exactly;
* anisotropic 2D grid: pairs follow the strong direction;
* random matrices (brute force): the aggregates partition the rows, pairs
  are strongly coupled by the dense symmetric-part rule, every pair is led
  by a row whose partner is its most negative free strong coupling, and a
  singleton's strong neighbours were all aggregated before it;
* Galerkin product with the 0/1 prolongation equals the dense P^T A P on
  integer matrices exactly, and keeps zero row sums;
* flexible GCR: one step with the exact inverse, n steps with the identity,
  monotone residuals and r_k orthogonal to A z_k;
* the AMLI-cycle on a two-level hierarchy is the V-cycle, bit for bit; on
  3D Poisson its FGMRES converges fast and two GCR steps never need more
  outer iterations than one;
* CPR with UA-AMG: dense direct solves on small black-oil grids.
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres, uaamg
from oracle.sparse import csr_from_dense
from workloads import blackoil as bo


def _tridiag(n):
    return np.diag(2.0 * np.ones(n)) + np.diag(-np.ones(n - 1), 1) + np.diag(-np.ones(n - 1), -1)


def test_1d_pairs_quadruples_and_coarse_operator():
    n = 32
    A = csr_from_dense(_tridiag(n))
    agg, na = uaamg.pairwise_matching(A, 0.25)
    assert na == n // 2 and np.array_equal(agg, np.arange(n) // 2)
    agg2, na2 = uaamg.npair_aggregates(A, 0.25, 2)
    assert na2 == n // 4 and np.array_equal(agg2, np.arange(n) // 4)
    H = uaamg.build_hierarchy(A, uaamg.UaParams(coarse_max=4))
    assert [L.A.n_rows for L in H.levels] == [32, 8, 2]
    assert np.array_equal(H.levels[1].A.to_dense(), _tridiag(8))


def _grid2d(nx, ny, wx, wy):
    n = nx * ny
    d = np.zeros((n, n))
    for j in range(ny):
        for i in range(nx):
            r = i + nx * j
            for di, dj, w in ((1, 0, wx), (-1, 0, wx), (0, 1, wy), (0, -1, wy)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    d[r, ii + nx * jj] = -w
                    d[r, r] += w
            d[r, r] += 1e-3
    return d


def test_anisotropic_pairs_follow_the_strong_direction():
    nx, ny = 8, 6
    A = csr_from_dense(_grid2d(nx, ny, 1.0, 0.01))
    agg, na = uaamg.pairwise_matching(A, 0.25)
    for a in range(na):
        rows = np.nonzero(agg == a)[0]
        assert rows.size <= 2
        if rows.size == 2:
            assert rows[1] - rows[0] == 1 and rows[0] // nx == rows[1] // nx
    assert na == nx * ny // 2


def _random_matrix(rng, n, density, symmetric):
    d = np.zeros((n, n))
    mask = rng.random((n, n)) < density
    vals = -rng.random((n, n))
    d[mask] = vals[mask]
    if symmetric:
        d = np.triu(d, 1)
        d = d + d.T
    np.fill_diagonal(d, 0.0)
    # a few positive couplings, which are never strong
    pos = rng.random((n, n)) < density / 5
    d[pos & (d == 0.0)] = 0.1
    np.fill_diagonal(d, -d.sum(axis=1) + 1.0)
    return d


@pytest.mark.parametrize("seed", range(12))
def test_matching_invariants_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 40
    d = _random_matrix(rng, n, 0.12, symmetric=seed % 2 == 0)
    A = csr_from_dense(d)
    beta = 0.25
    agg, na = uaamg.pairwise_matching(A, beta)
    # dense symmetric-part strength, written independently
    s = (d + d.T) / 2.0
    S = []
    for i in range(n):
        off = [(-s[i, j], j) for j in range(n) if j != i and (d[i, j] != 0.0 or d[j, i] != 0.0)]
        top = max((v for v, _ in off), default=0.0)
        S.append({j for v, j in off if top > 0.0 and s[i, j] < -beta * top})
    assert sorted(np.unique(agg)) == list(range(na))
    for a in range(na):
        rows = [int(r) for r in np.nonzero(agg == a)[0]]
        assert len(rows) in (1, 2)
        if len(rows) == 1:
            i = rows[0]
            assert all(agg[j] < a for j in S[i])
            continue
        ok = False
        for i, j in (rows, rows[::-1]):
            if j not in S[i]:
                continue
            free = [k for k in S[i] if agg[k] >= a]
            best = min(free, key=lambda k: (s[i, k], k))
            ok = ok or best == j
        assert ok, (a, rows)


def test_galerkin_with_aggregation_is_exact_on_integers():
    rng = np.random.default_rng(3)
    n = 30
    d = np.round(_random_matrix(rng, n, 0.2, symmetric=False) * 8)
    np.fill_diagonal(d, 0.0)
    np.fill_diagonal(d, -d.sum(axis=1))  # zero row sums
    A = csr_from_dense(d)
    agg, na = uaamg.npair_aggregates(A, 0.25, 2)
    P = uaamg.aggregation_matrix(agg, na)
    R, Ac = uaamg.rs.galerkin(A, P)
    Pd = P.to_dense()
    assert np.array_equal(Ac.to_dense(), Pd.T @ d @ Pd)
    assert np.all(Ac.to_dense().sum(axis=1) == 0.0)
    assert np.array_equal(R.to_dense(), Pd.T)


def test_gcr_pins():
    rng = np.random.default_rng(5)
    n = 12
    d = rng.standard_normal((n, n)) + n * np.eye(n)
    A = csr_from_dense(d)
    f = rng.standard_normal(n)
    exact = np.linalg.solve(d, f)
    e1 = uaamg.gcr(A, f, lambda r: np.linalg.solve(d, r), 1)
    assert np.linalg.norm(e1 - exact) <= 1e-12 * np.linalg.norm(exact)
    en = uaamg.gcr(A, f, lambda r: r.copy(), n)
    assert np.linalg.norm(en - exact) <= 1e-9 * np.linalg.norm(exact)
    prev = np.linalg.norm(f)
    for k in range(1, n):
        e = uaamg.gcr(A, f, lambda r: r.copy(), k)
        r = f - d @ e
        assert np.linalg.norm(r) <= prev * (1 + 1e-13)
        prev = np.linalg.norm(r)
        # the last search direction w = A z is orthogonal to the new residual
        ek1 = uaamg.gcr(A, f, lambda r: r.copy(), k - 1)
        w = d @ (e - ek1)
        assert abs(np.dot(r, w)) <= 1e-6 * np.linalg.norm(r) * np.linalg.norm(w) + 1e-300


def _poisson3d(m):
    n = m ** 3
    d = np.zeros((n, n))
    for k in range(m):
        for j in range(m):
            for i in range(m):
                r = i + m * (j + m * k)
                d[r, r] = 6.0
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < m and 0 <= jj < m and 0 <= kk < m:
                        d[r, ii + m * (jj + m * kk)] = -1.0
    return d


def test_two_level_amli_is_the_v_cycle():
    A = csr_from_dense(_poisson3d(6))
    H = uaamg.build_hierarchy(A, uaamg.UaParams(coarse_max=60))
    assert H.n_levels == 2
    b = np.random.default_rng(2).standard_normal(A.n_rows)
    assert np.array_equal(uaamg.kcycle(H, b), amg.vcycle(H, b))


def test_amli_cycle_converges_on_3d_poisson():
    d = _poisson3d(12)
    A = csr_from_dense(d)
    b = np.random.default_rng(4).standard_normal(A.n_rows)
    its = {}
    for inner in (1, 2):
        H = uaamg.build_hierarchy(A, uaamg.UaParams(coarse_max=30, inner=inner))
        assert H.n_levels >= 4
        res = fgmres.fgmres(lambda v: d @ v, lambda v: uaamg.kcycle(H, v), b, tol=1e-8)
        assert res.converged
        assert np.linalg.norm(b - d @ res.x) <= 1e-8 * np.linalg.norm(b) * 1.01
        its[inner] = res.iterations
    assert its[2] <= its[1]
    assert its[2] <= 15


@pytest.mark.parametrize("shape", [(6, 6, 3), (10, 10, 4)])
def test_cpr_with_uaamg_matches_dense_solve(shape):
    case = bo.case_small(seed=17, shape=shape)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, uaamg.UaParams(coarse_max=10))
    assert B.amg.n_levels >= 2
    b = bo.rhs(case.ndof, 18)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-8)
    dense = A.to_dense()
    x = np.linalg.solve(dense, b)
    cond = np.linalg.cond(dense)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= cond * 1e-8 * np.linalg.norm(x)
