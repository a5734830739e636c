"""Pins of the oracle's FGMRES (Section 4, Algorithm ASCPR-GMRES).

* B = I and m >= N: converges within N steps to the LAPACK solution.
* B = A^{-1}: one step.
* The Givens estimate is non-increasing within a cycle and matches the true
  residual at the end.
* With a fixed linear B, the flexible iterate equals the printed right-
  preconditioned GMRES iterate x0 + B(P_m y_m), written out here separately.
* Happy breakdown: b in a 1-dimensional invariant subspace stops at j = 1.
"""
import numpy as np

from oracle import fgmres


def _rand_nonsym(rng, n, shift=4.0):
    return rng.standard_normal((n, n)) + shift * np.eye(n)


def test_identity_precond_full_space_matches_lapack():
    rng = np.random.default_rng(1)
    n = 25
    A = _rand_nonsym(rng, n)
    b = rng.standard_normal(n)
    res = fgmres.fgmres(lambda v: A @ v, lambda v: v.copy(), b, tol=1e-13, m=n)
    assert res.iterations <= n
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-10 * np.linalg.cond(A)


def test_exact_inverse_one_step():
    rng = np.random.default_rng(2)
    n = 30
    A = _rand_nonsym(rng, n)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(n)
    res = fgmres.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-10)
    assert res.iterations == 1 and res.converged


def test_estimate_monotone_and_true_residual():
    rng = np.random.default_rng(3)
    n = 200
    A = _rand_nonsym(rng, n, shift=12.0)
    b = rng.standard_normal(n)
    res = fgmres.fgmres(lambda v: A @ v, lambda v: v.copy(), b, tol=1e-8, m=60)
    h = res.history
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
    assert res.converged
    rel = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert abs(rel - res.relres_est) <= 1e-6 * rel + 1e-14


def _right_pgmres(A, B, b, m, tol):
    """Printed form: x_m = x0 + B (P_m y_m), one cycle only."""
    n = b.shape[0]
    r0 = b.copy()
    beta = np.linalg.norm(r0)
    P = [r0 / beta]
    Hb = np.zeros((m + 1, m))
    for j in range(m):
        pbar = A @ (B @ P[j])
        for i in range(j + 1):
            Hb[i, j] = pbar @ P[i]
        pt = pbar - sum(Hb[i, j] * P[i] for i in range(j + 1))
        Hb[j + 1, j] = np.linalg.norm(pt)
        P.append(pt / Hb[j + 1, j])
    e1 = np.zeros(m + 1)
    e1[0] = beta
    y = np.linalg.lstsq(Hb, e1, rcond=None)[0]
    return B @ (np.column_stack(P[:m]) @ y)


def test_flexible_equals_right_preconditioned_for_fixed_b():
    rng = np.random.default_rng(4)
    n = 80
    A = _rand_nonsym(rng, n, shift=6.0)
    Bm = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n)
    m = 6
    res = fgmres.fgmres(lambda v: A @ v, lambda v: Bm @ v, b, tol=1e-30, m=m, max_restarts=1)
    want = _right_pgmres(A, Bm, b, m, 0.0)
    assert np.linalg.norm(res.x - want) / np.linalg.norm(want) < 1e-12


def test_happy_breakdown():
    n = 10
    A = np.diag(np.arange(1.0, n + 1))
    b = np.zeros(n)
    b[3] = 2.0
    res = fgmres.fgmres(lambda v: A @ v, lambda v: v.copy(), b, tol=1e-12)
    assert res.iterations == 1 and res.converged
    assert np.allclose(res.x[3], 0.5)
