"""Pins of the oracle's V-cycle against two-grid theory.

* Exactness: with ideal interpolation (every F point couples only to C
  points, as RS produces on 1D Poisson), the Galerkin coarse operator, an exact
  coarse solve and one post-relaxation that visits F before C, one cycle
  returns the exact solution.  Any dropped term in the restriction,
  interpolation, Galerkin product or coarse solve breaks this.
* Convergence factor: for 1D (n=63) and 3D (8^3) Poisson the asymptotic
  factor of the implemented two-level cycle (power iteration on the error
  propagator I - B A) equals the spectral radius of the two-grid operator
  assembled densely from textbook pieces: forward Gauss-Seidel in colour
  order, S = I - (D+L)^{-1} A, and the coarse correction
  I - P (P^T A P)^{-1} P^T A.
"""
import numpy as np
import scipy.linalg

from oracle import amg, rs
from oracle.sparse import csr_from_dense
from tests.test_oracle_rs import _lap1d, _lap3d


def _two_level(d, colours=None, pre=0, post=1, theta_color=0.0):
    A = csr_from_dense(d)
    p = amg.AmgParams(coarse_max=10 ** 9, theta_color=theta_color, pre_sweeps=pre, post_sweeps=post)
    # level 0 with its split; force a two-level hierarchy
    H = amg.build_hierarchy(A, amg.AmgParams(coarse_max=d.shape[0] // 2 + 1, max_levels=2,
                                             theta_color=theta_color, pre_sweeps=pre, post_sweeps=post))
    assert H.n_levels == 2
    if colours is not None:
        H.levels[0].colours = colours
    H.params = amg.AmgParams(coarse_max=p.coarse_max, max_levels=2, theta_color=theta_color,
                             pre_sweeps=pre, post_sweeps=post)
    return H


def test_ideal_two_grid_is_exact_in_one_cycle_1d():
    n = 63
    d = _lap1d(n)
    H = _two_level(d)
    cf = H.levels[0].cf
    F = [i for i in range(n) if cf[i] == rs.F]
    C = [i for i in range(n) if cf[i] == rs.C]
    H.levels[0].colours = [F, C]
    rng = np.random.default_rng(0)
    xs = rng.standard_normal(n)
    b = d @ xs
    x = amg.vcycle(H, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12


def _dense_gs(d, order):
    Pm = np.eye(d.shape[0])[order]
    Ap = Pm @ d @ Pm.T
    M = np.tril(Ap)
    S = np.eye(d.shape[0]) - np.linalg.solve(M, Ap)
    return Pm.T @ S @ Pm


def _assembled_rate(d, H, pre, post):
    lev = H.levels[0]
    order = [v for c in lev.colours for v in c]
    S = _dense_gs(d, order)
    Pd = lev.P.to_dense()
    Ac = Pd.T @ d @ Pd
    CGC = np.eye(d.shape[0]) - Pd @ np.linalg.solve(Ac, Pd.T @ d)
    E = np.linalg.matrix_power(S, post) @ CGC @ np.linalg.matrix_power(S, pre)
    return max(abs(np.linalg.eigvals(E)))


def _power_rate(d, H, its=200):
    rng = np.random.default_rng(1)
    e = rng.standard_normal(d.shape[0])
    rate = 0.0
    for k in range(its):
        e_new = e - amg.vcycle(H, d @ e)
        rate = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    return rate


def test_two_grid_rate_matches_dense_eigensolve():
    for d, pre, post in ((_lap1d(63) + 0.01 * np.eye(63), 1, 1), (_lap3d(8), 2, 2)):
        H = _two_level(d, pre=pre, post=post)
        rho = _assembled_rate(d, H, pre, post)
        got = _power_rate(d, H)
        assert rho < 1.0
        assert abs(got - rho) < 1e-3, (got, rho)
