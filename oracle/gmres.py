"""Restarted GMRES with right preconditioning, as used by the oracle.

Sec. 6: GMRES stops on a 1e-8 reduction of the Euclidean norm of the relative residual.
Reading: right preconditioning, so the monitored norm is the true residual
||b - A x||_2 <= rtol ||b||_2, from x0 = 0 unless given; restart length m; "its"
counts Arnoldi steps summed over restarts.  The Arnoldi basis is orthogonalised by
classical Gram-Schmidt applied twice, and the small least-squares problem is reduced by
Givens rotations (textbook GMRES).  At the end of each cycle the true residual is
recomputed; a cycle that reaches the estimate but not the true residual restarts.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, precond=None, x0=None, restart=30, rtol=1e-8, maxit=10000):
    """Return ``(x, info)`` with info = dict(its, restarts, relres, converged)."""
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(N), dict(its=0, restarts=0, relres=0.0, converged=True)
    target = rtol * bnorm
    its = 0
    restarts = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while beta > target and its < maxit:
        V = np.zeros((restart + 1, N))
        Z = np.zeros((restart, N))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = matvec(Z[j])
            # classical Gram-Schmidt, twice
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            # apply the previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= target or hn == 0.0 or its >= maxit:
                break
            V[j + 1] = w / hn
        # x += Z y with H[:k,:k] y = g[:k]
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        restarts += 1
    return x, dict(its=its, restarts=restarts, relres=beta / bnorm, converged=bool(beta <= target))
