"""Newton's method for one time step with the nonlinear solid (Sec. 4, last paragraph: a
nonlinear law P(F) is handled by Newton iterations; Sec. 6: they stop on a 1e-6 reduction of
the Euclidean norm of the relative residual).

The step of Problem 3 with a general law is the nonlinear system G(x) = 0, x = (u, p, X, lam):
  G_u   = A_f u - B^T p + C_f(X^n)^T lam - g1
  G_p   = -B u   (+ p_0 at the pinned node)
  G_X   = R(X) - C_s lam - f_X
  G_lam = C_f(X^n) u - (1/dt) C_s X - g2
that is eq. (matrix) with the product A_s X replaced by the solid residual R(X) of
``oracle.hyper`` (f_X: a load on the solid nodes, zero unless given).  Newton's iteration:
J(x_k) d = -G(x_k), x_{k+1} = x_k + d, with J the matrix of eq. (matrix) whose A_s block is the
tangent K(X_k); it stops when ||G(x_k)|| <= rtol ||G(x_0)||.  The Jacobian systems are solved
by the sparse direct solve (the plain definition), with the refinement of ``system``.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import hyper


def _solid_embed(S, M2):
    """The 2 Ns x 2 Ns matrix M2 placed at the X rows and columns of the full system."""
    lay = S.lay
    nf, ns2 = lay.nf, 2 * lay.Ns
    Z = sp.csr_matrix
    return sp.bmat([[Z((nf, nf)), None, None], [None, M2, None], [None, None, Z((ns2, ns2))]], format="csr")


def residual(S, x, b, gamma=hyper.GAMMA, eta=hyper.ETA):
    """G(x) - with b = (g1, 0, f_X, g2): A x with the solid product replaced, minus b."""
    lay = S.lay
    sl = lay.slices()
    X = np.stack([x[sl["Xx"]], x[sl["Xy"]]], axis=1)
    As2 = sp.block_diag([S.S["As"], S.S["As"]], format="csr")
    Ax = S.matrix() @ x
    nf, ns2 = lay.nf, 2 * lay.Ns
    Ax[nf:nf + ns2] += hyper.residual(S.xy_ref, S.tri, X, gamma, eta) - As2 @ x[nf:nf + ns2]
    return Ax - b


def jacobian(S, x, gamma=hyper.GAMMA, eta=hyper.ETA):
    """J(x): eq. (matrix) with A_s replaced by the tangent K(X)."""
    lay = S.lay
    sl = lay.slices()
    X = np.stack([x[sl["Xx"]], x[sl["Xy"]]], axis=1)
    As2 = sp.block_diag([S.S["As"], S.S["As"]], format="csr")
    K = hyper.tangent(S.xy_ref, S.tri, X, gamma, eta)
    return (S.matrix() + _solid_embed(S, K - As2)).tocsr()


def _solve(J, r, refine=4):
    lu = spla.splu(J.tocsc())
    d = lu.solve(r)
    rn = np.linalg.norm(r - J @ d)
    for _ in range(refine):
        d2 = d + lu.solve(r - J @ d)
        rn2 = np.linalg.norm(r - J @ d2)
        if rn2 >= rn:
            break
        d, rn = d2, rn2
    return d


def rhs(S, u_n, X_n, f_X=None):
    """b = (g1, 0, f_X, g2) of the step (S.rhs plus the load on the X rows)."""
    b = S.rhs(u_n, X_n)
    if f_X is not None:
        lay = S.lay
        b[lay.nf:lay.nf + 2 * lay.Ns] += np.asarray(f_X, dtype=np.float64)
    return b


def newton_step(S, u_n, X_n, x0, f_X=None, gamma=hyper.GAMMA, eta=hyper.ETA, rtol=1e-6, maxit=50):
    """One step from the initial guess x0.  Returns (x, info) with info = dict(nit, res: the
    residual norms ||G(x_k)||, converged)."""
    S.set_position(X_n)
    b = rhs(S, u_n, X_n, f_X)
    x = np.array(x0, dtype=np.float64)
    res = []
    for k in range(maxit + 1):
        G = residual(S, x, b, gamma, eta)
        res.append(float(np.linalg.norm(G)))
        if res[-1] == 0.0 or res[-1] <= rtol * res[0]:
            return x, dict(nit=k, res=res, converged=True)
        if k == maxit:
            break
        x = x + _solve(jacobian(S, x, gamma, eta), -G)
    return x, dict(nit=maxit, res=res, converged=False)
