"""One semi-implicit backward-Euler step of Problem 3 (Sec. 4) and a time loop.

A step at position X^n: assemble C_f(X^n), form the right-hand side (g1, 0, 0, g2) of
eq. (matrix) from (u^n, X^n), solve for (u, p, X, lam)^{n+1}.  The constraint row
follows the matrix form (u^{n+1} inside C_f), which is how the time discretisation of
Sec. 4 treats the coupling terms (semi-implicitly, at the previous position).

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np

from . import gmres as _gmres


def step(system, u_n, X_n, solver="direct", pc="tri", restart=30, rtol=1e-8, maxit=10000):
    """Return ``(state, info)``; ``state`` is the full unknown vector at n+1."""
    system.set_position(X_n)
    b = system.rhs(u_n, X_n)
    if solver == "direct":
        return system.solve_direct(b), dict(its=0)
    A = system.matrix()
    x, info = _gmres.gmres(lambda v: A @ v, b, precond=lambda r: system.apply_precond(r, pc),
                           restart=restart, rtol=rtol, maxit=maxit)
    return x, info


def time_loop(system, X_of_step, steps, u0=None, **kw):
    """Run ``steps`` steps with prescribed positions ``X_of_step(k)``; u^{k+1} feeds the
    next step.  Returns the list of states."""
    lay = system.lay
    u = np.zeros(2 * lay.N2) if u0 is None else np.array(u0, dtype=np.float64)
    out = []
    for k in range(steps):
        x, _ = step(system, u, X_of_step(k), **kw)
        u = x[:2 * lay.N2].copy()
        out.append(x)
    return out
