"""Pins of the oracle's strength-of-connection routines.

The paper's strong-connection matrix, eq. (strong-matrix) of Section 5.2, and
the classical RS strength are recomputed by brute force on dense matrices with
exactly rounded sums (math.fsum) and compared entry by entry; special cases
fix theta = 0 and theta >= 1.
"""
import math

import numpy as np

from oracle import strength
from oracle.sparse import csr_from_dense


def _random_sparse(rng, n, density=0.3):
    d = rng.standard_normal((n, n)) * (rng.uniform(size=(n, n)) < density)
    d[np.arange(n), np.arange(n)] = rng.uniform(1, 5, size=n)
    return d


def test_color_strength_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(40):
        d = _random_sparse(rng, 30)
        A = csr_from_dense(d)
        theta = [0.0, 0.01, 0.05, 0.1, 0.3][trial % 5]
        mask, (ip, ix) = strength.color_strength(A, theta)
        for i in range(30):
            bound = theta * math.fsum(abs(v) for v in d[i])
            want = sorted(j for j in range(30) if j != i and d[i, j] != 0 and abs(d[i, j]) > bound)
            assert list(ix[ip[i]:ip[i + 1]]) == want


def test_color_strength_special_cases():
    rng = np.random.default_rng(8)
    d = _random_sparse(rng, 25)
    A = csr_from_dense(d)
    mask0, _ = strength.color_strength(A, 0.0)
    row_of = np.repeat(np.arange(25), np.diff(A.indptr))
    assert np.array_equal(mask0, (A.indices != row_of) & (A.data != 0))
    for th in (1.0, 1.5):
        mask1, _ = strength.color_strength(A, th)
        assert not mask1.any()


def test_rs_strength_brute_force():
    rng = np.random.default_rng(9)
    for trial in range(40):
        d = _random_sparse(rng, 30)
        A = csr_from_dense(d)
        theta = [0.25, 0.1, 0.5, 0.0][trial % 4]
        mask, (ip, ix) = strength.rs_strength(A, theta)
        for i in range(30):
            neg = [-d[i, k] for k in range(30) if k != i and d[i, k] != 0]
            mx = max(neg) if neg else -math.inf
            want = []
            if mx > 0:
                want = [j for j in range(30) if j != i and d[i, j] != 0 and -d[i, j] >= theta * mx]
            assert list(ix[ip[i]:ip[i + 1]]) == want


def test_rs_strength_constant_poisson_all_neighbours_strong():
    n = 6
    idx = lambda i, j, k: i + n * (j + n * k)
    N = n ** 3
    d = np.zeros((N, N))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = idx(i, j, k)
                d[r, r] = 6
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    a, b_, c = i + di, j + dj, k + dk
                    if 0 <= a < n and 0 <= b_ < n and 0 <= c < n:
                        d[r, idx(a, b_, c)] = -1
    A = csr_from_dense(d)
    mask, _ = strength.rs_strength(A, 0.25)
    row_of = np.repeat(np.arange(N), np.diff(A.indptr))
    assert np.array_equal(mask, A.indices != row_of)
