"""Rows of the system of eq. (matrix) at sampled unknowns, for grids too large to assemble whole.

Sec. 4, eq. (matrix) and the block definitions after it: the operator rows and the right-hand
side (g1, 0, 0, g2) at a chosen set of velocity nodes, pressure nodes and solid nodes.  Each row
is built from the same definitions as the whole-system assembly, restricted to what the row
touches:
* A_f, M_f, B and B^T rows from the element matrices of the fluid triangles around the node
  (``oracle.fluid.rows_Af``, ``rows_B``, ``rows_BT``, with the boundary condition and the
  pressure pin of the whole assembly);
* A_s and C_s rows from the solid triangles around the sampled solid nodes (``oracle.solid``);
* C_f rows (sampled solid nodes) and C_f^T rows (sampled velocity nodes) from the clipping and
  exact integration of ``oracle.coupling`` over the solid triangles that contain the sampled
  solid nodes or whose mapped bounding box meets the support of a sampled velocity node.

Used to certify a solution on grids where the oracle cannot solve the whole system: the
residual b - A x on the sampled rows.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np

from . import coupling, fluid, solid


def sample_rows(n, Xn, tri, ns, rng, n_vel=60, n_p=40, n_s=25, n_under=20):
    """Seeded sample: random velocity nodes plus nodes under mapped solid triangles (non-empty
    C_f^T rows), random pressure nodes plus the pinned node 0, random solid nodes."""
    L = 2 * n + 1
    cen = Xn[tri].mean(axis=1)
    under = [int(round(c[1] * 2 * n)) * L + int(round(c[0] * 2 * n)) for c in cen[rng.choice(len(cen), n_under)]]
    vel = sorted(set(rng.choice(L * L, n_vel, replace=False).tolist()) | set(under))
    prs = sorted(set(rng.choice((n + 1) ** 2, n_p, replace=False).tolist()) | {0})
    sol = sorted(rng.choice(ns, min(n_s, ns), replace=False).tolist())
    return vel, prs, sol


class SampledSystem:
    """The rows of eq. (matrix) at velocity nodes ``vel`` (both components), pressure nodes
    ``prs`` and solid nodes ``sol`` (X and lam rows, both components), for the fluid grid n,
    the solid reference mesh (xy, tri) and the position Xn ([Ns, 2])."""

    def __init__(self, n, xy, tri, Xn, vel, prs, sol, nu=1.0, rho=1.0, dt=0.01, kappa=10.0):
        self.n, self.nu, self.rho, self.dt, self.kappa = n, nu, rho, dt, kappa
        self.xy = np.asarray(xy, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        self.Xn = np.asarray(Xn, dtype=np.float64)
        self.vel, self.prs, self.sol = list(vel), list(prs), list(sol)
        L = 2 * n + 1
        self.N2, self.Np, self.Ns = L * L, (n + 1) ** 2, self.xy.shape[0]
        self.A, self.M = fluid.rows_Af(n, self.vel, nu, rho, dt)
        self.BT = fluid.rows_BT(n, self.vel)
        self.B = fluid.rows_B(n, self.prs)
        n2e = [[] for _ in range(self.Ns)]
        for e, t in enumerate(self.tri):
            for v in t:
                n2e[v].append(e)
        star = sorted({e for l in self.sol for e in n2e[l]})
        P = self.Xn[self.tri]
        lo, hi = P.min(axis=1), P.max(axis=1)
        near = set()
        for r in self.vel:
            I, J = r % L, r // L
            x0, x1 = max(I - 2, 0) / (2 * n), min(I + 2, 2 * n) / (2 * n)
            y0, y1 = max(J - 2, 0) / (2 * n), min(J + 2, 2 * n) / (2 * n)
            hit = np.nonzero((hi[:, 0] >= x0) & (lo[:, 0] <= x1) & (hi[:, 1] >= y0) & (lo[:, 1] <= y1))[0]
            near.update(int(e) for e in hit)
        els = sorted(near | set(star))
        self.Cf = coupling.assemble(self.Xn, self.xy, self.tri[els], n)[0].tocsr() if els else None
        self.CfT = self.Cf.T.tocsr() if self.Cf is not None else None
        S = solid.assemble(self.xy, self.tri[star], kappa) if star else None
        self.As = S["As"].tocsr() if S else None
        self.Cs = S["Ms"].tocsr() if S else None
        self.bnd = fluid.boundary_p2(n)

    def offsets(self):
        N2, Np, Ns = self.N2, self.Np, self.Ns
        return dict(ux=0, uy=N2, p=2 * N2, Xx=2 * N2 + Np, Xy=2 * N2 + Np + Ns, lx=2 * N2 + Np + 2 * Ns,
                    ly=2 * N2 + Np + 3 * Ns)

    def index(self, key):
        """Global index of the row (block, node)."""
        return self.offsets()[key[0]] + key[1]

    def apply(self, x):
        """{(block, node): (A x)_row} on the sampled rows."""
        o = self.offsets()
        N2, Np, Ns = self.N2, self.Np, self.Ns
        ux, uy, p = x[:N2], x[N2:2 * N2], x[2 * N2:2 * N2 + Np]
        Xx, Xy = x[o["Xx"]:o["Xx"] + Ns], x[o["Xy"]:o["Xy"] + Ns]
        lx, ly = x[o["lx"]:o["lx"] + Ns], x[o["ly"]:o["ly"] + Ns]
        out = {}
        for r in self.vel:
            sx = sum(v[0] * ux[c] + v[1] * uy[c] for c, v in self.A[r].items())
            sy = sum(v[2] * ux[c] + v[3] * uy[c] for c, v in self.A[r].items())
            sx -= sum(v[0] * p[c] for c, v in self.BT[r].items())
            sy -= sum(v[1] * p[c] for c, v in self.BT[r].items())
            if self.CfT is not None:
                ct = self.CfT
                cs, vs = ct.indices[ct.indptr[r]:ct.indptr[r + 1]], ct.data[ct.indptr[r]:ct.indptr[r + 1]]
                sx += vs @ lx[cs]
                sy += vs @ ly[cs]
            out[("ux", r)] = sx
            out[("uy", r)] = sy
        for k in self.prs:
            s = -sum(v[0] * ux[c] + v[1] * uy[c] for c, v in self.B[k].items())
            out[("p", k)] = s + (p[0] if k == 0 else 0.0)
        inv_dt = 1.0 / self.dt
        for l in self.sol:
            sl = slice(self.As.indptr[l], self.As.indptr[l + 1])
            cc = self.As.indices[sl]
            out[("Xx", l)] = self.As.data[sl] @ Xx[cc] - self.Cs.data[sl] @ lx[cc]
            out[("Xy", l)] = self.As.data[sl] @ Xy[cc] - self.Cs.data[sl] @ ly[cc]
            cf = self.Cf
            fc, fv = cf.indices[cf.indptr[l]:cf.indptr[l + 1]], cf.data[cf.indptr[l]:cf.indptr[l + 1]]
            out[("lx", l)] = fv @ ux[fc] - inv_dt * (self.Cs.data[sl] @ Xx[cc])
            out[("ly", l)] = fv @ uy[fc] - inv_dt * (self.Cs.data[sl] @ Xy[cc])
        return out

    def rhs(self, u_n):
        """{(block, node): b_row} of (g1, 0, 0, g2): g1 = (rho/dt) M_f u^n with boundary rows and
        entries zero, g2 = -(1/dt) C_s X^n."""
        N2 = self.N2
        out = {}
        for r in self.vel:
            for comp, key in ((0, "ux"), (1, "uy")):
                g = 0.0
                if not self.bnd[r]:
                    g = (self.rho / self.dt) * sum(m * (0.0 if self.bnd[c] else u_n[comp * N2 + c])
                                                   for c, m in self.M[r].items())
                out[(key, r)] = g
        for k in self.prs:
            out[("p", k)] = 0.0
        for l in self.sol:
            sl = slice(self.Cs.indptr[l], self.Cs.indptr[l + 1])
            cc = self.Cs.indices[sl]
            out[("Xx", l)] = 0.0
            out[("Xy", l)] = 0.0
            out[("lx", l)] = -(1.0 / self.dt) * (self.Cs.data[sl] @ self.Xn[cc, 0])
            out[("ly", l)] = -(1.0 / self.dt) * (self.Cs.data[sl] @ self.Xn[cc, 1])
        return out

    def residual(self, x, u_n):
        """{(block, node): b_row - (A x)_row} on the sampled rows."""
        ax = self.apply(x)
        b = self.rhs(u_n)
        return {k: b[k] - ax[k] for k in ax}
