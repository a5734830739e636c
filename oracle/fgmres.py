"""Flexible restarted GMRES(m) with right preconditioning (oracle; test infrastructure only).

Follows Algorithm "ASCPR-GMRES" of Section 4 (restarted GMRES, classical
Gram-Schmidt Arnoldi, happy breakdown when h_{j+1,j} = 0, least-squares
problem on the Hessenberg matrix, true residual at every restart) with these
readings:

* flexible form: z_j = B p_j is stored and the update is x = x0 + Z y (with a
  fixed linear B this is the same iterate as the printed x0 + B(P_m y));
* beta of the least-squares problem is the norm of the cycle's starting
  residual (the printed ||p_1|| is 1 by construction);
* convergence is ||r||/||r_0|| < tol with r_0 the residual of the call's
  initial guess; inside a cycle the Givens estimate |g_{j+1}| is checked after
  every step and an early exit is confirmed with the true residual;
* the iteration count is the number of inner Arnoldi steps (one B apply and
  one product with A each), summed over restarts.

The least-squares problem is solved by Givens rotations:
rho = sqrt(h_jj^2 + h_{j+1,j}^2), c = h_jj/rho, s = h_{j+1,j}/rho,
g_{j+1} = -s g_j, g_j = c g_j.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FgmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    relres_true: float
    relres_est: float
    history: list = field(default_factory=list)  # |g_{j+1}|/||r0|| per step


def fgmres(matvec, precond, b, x0=None, tol=1e-6, m=30, max_restarts=100):
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - matvec(x)
    beta0 = float(np.sqrt(np.dot(r, r)))
    if beta0 == 0.0:
        return FgmresResult(x, 0, 0, True, 0.0, 0.0)
    its = 0
    hist = []
    est = 1.0
    for cycle in range(max_restarts):
        rn = float(np.sqrt(np.dot(r, r)))
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / rn
        g[0] = rn
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            its += 1
            h = np.array([np.dot(w, V[i]) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h[i] * V[i]
            hn = float(np.sqrt(np.dot(w, w)))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = float(np.sqrt(H[j, j] * H[j, j] + H[j + 1, j] * H[j + 1, j]))
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            est = abs(g[j + 1]) / beta0
            hist.append(est)
            if hn == 0.0:
                break  # happy breakdown
            V[j + 1] = w / hn
            if est < tol:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            s = g[i]
            for l in range(i + 1, k):
                s = s - H[i, l] * y[l]
            y[i] = s / H[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - matvec(x)
        rel = float(np.sqrt(np.dot(r, r))) / beta0
        if rel < tol:
            return FgmresResult(x, its, cycle, True, rel, est, hist)
    return FgmresResult(x, its, max_restarts - 1, False, rel, est, hist)
