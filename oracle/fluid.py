"""Fluid discretisation of the oracle: P2 velocity / P1 pressure on the triangulated
unit square, and the blocks M_f, K_f, A_f and B of Sec. 4, eq. (matrix).

Numbering (the fluid grid is Cartesian, Sec. 4 on the coupling assembly):
* n x n square cells of side h = 1/n; cell (i, j) is split along its diagonal from
  (i, j) to (i+1, j+1) into T0 = (v00, v10, v11) and T1 = (v00, v11, v01); the global
  triangle id is 2 (j n + i) + t.
* P2 node (I, J), 0 <= I, J <= 2n, sits at (I h/2, J h/2) and has index J (2n+1) + I.
* P1 pressure node (i, j) has index j (n+1) + i.
* The local P2 order on a triangle (a, b, c) is (a, b, c, ab, bc, ca).
* Velocity unknowns are ordered [u_x (N2) | u_y (N2)].

Blocks (Sec. 4): (M_f)_ij = (phi_j, phi_i), (K_f)_ij = a(phi_j, phi_i) with
a(u, v) = nu (eps(u), eps(v)) (Sec. 3, Problem 2), A_f = (rho/dt) M_f + K_f and
B_ki = (div phi_i, psi_k).  Every element matrix is integrated exactly
(``oracle.poly``).  Sparsity patterns are the element-connectivity patterns with
explicit zeros kept and columns sorted.

Boundary conditions (u = 0 on the boundary of the square, Sec. 3 eq. (conditions)) are
imposed by value: every row and column of a boundary velocity unknown is zeroed in A_f
(diagonal set to 1), in B and in C_f.  The pressure (defined up to a constant, L^2_0 in
Problem 3) is pinned at P1 node 0: row 0 of B is zeroed and the (p0, p0) entry of the
global matrix is 1.  Patterns are not changed by either.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp

from . import poly


def sizes(n):
    return dict(N2=(2 * n + 1) ** 2, Np=(n + 1) ** 2, ntri=2 * n * n)


def p2_index(n, I, J):
    return J * (2 * n + 1) + I


def p1_index(n, i, j):
    return j * (n + 1) + i


@functools.lru_cache(maxsize=2)
def triangle_nodes(n):
    """Local-to-global maps (cached; callers must not modify the arrays).

    Returns ``(p2, p1, verts)``: int arrays [2 n^2, 6] (P2 nodes), [2 n^2, 3] (P1 nodes)
    and float [2 n^2, 3, 2] (vertex coordinates), in global triangle order.
    """
    h = 1.0 / n
    p2 = np.zeros((2 * n * n, 6), dtype=np.int64)
    p1 = np.zeros((2 * n * n, 3), dtype=np.int64)
    vx = np.zeros((2 * n * n, 3, 2))
    for j in range(n):
        for i in range(n):
            for t in range(2):
                tid = 2 * (j * n + i) + t
                if t == 0:
                    V = [(i, j), (i + 1, j), (i + 1, j + 1)]
                else:
                    V = [(i, j), (i + 1, j + 1), (i, j + 1)]
                P = [(2 * a, 2 * b) for (a, b) in V]
                M = [((P[0][0] + P[1][0]) // 2, (P[0][1] + P[1][1]) // 2),
                     ((P[1][0] + P[2][0]) // 2, (P[1][1] + P[2][1]) // 2),
                     ((P[2][0] + P[0][0]) // 2, (P[2][1] + P[0][1]) // 2)]
                p2[tid] = [p2_index(n, I, J) for (I, J) in P + M]
                p1[tid] = [p1_index(n, a, b) for (a, b) in V]
                vx[tid] = [(a * h, b * h) for (a, b) in V]
    return p2, p1, vx


def p2_coords(n):
    """Coordinates of the P2 nodes, [N2, 2]."""
    I, J = np.meshgrid(np.arange(2 * n + 1), np.arange(2 * n + 1), indexing="xy")
    return np.stack([I.ravel() * 0.5 / n, J.ravel() * 0.5 / n], axis=1)


def p1_coords(n):
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    return np.stack([i.ravel() / n, j.ravel() / n], axis=1)


def boundary_p2(n):
    """Boolean mask of P2 nodes on the boundary of the unit square."""
    I, J = np.meshgrid(np.arange(2 * n + 1), np.arange(2 * n + 1), indexing="xy")
    return ((I == 0) | (J == 0) | (I == 2 * n) | (J == 2 * n)).ravel()


def element_matrices(p, nu):
    """Exact P2/P1 element matrices on the triangle with vertex coordinates ``p`` (3x2).

    Returns dict with
      M   (6x6)     int phi_j phi_i
      K   (2,2,6,6) K[alpha, beta, i, j] = nu int eps(phi_j e_beta) : eps(phi_i e_alpha)
      B   (2,3,6)   B[alpha, k, i] = int d_alpha phi_i psi_k
      Mp  (3x3)     P1 mass (pressure)
    """
    grads, area = poly.bary_gradients(p)
    area = abs(area)
    phi = poly.p2_basis()
    psi = poly.p1_basis()
    dphi = [poly.gradient(f, grads) for f in phi]        # [i][comp]

    def eps(i, alpha):
        # symmetric gradient of phi_i e_alpha as a 2x2 nested list of polynomials;
        # (grad v)_{k l} = d_l v_k, so row alpha holds grad(phi_i)
        g = [[{}, {}], [{}, {}]]
        for l in range(2):
            g[alpha][l] = dphi[i][l]
        e = [[None, None], [None, None]]
        for k in range(2):
            for l in range(2):
                e[k][l] = poly.scale(poly.add(g[k][l], g[l][k]), 0.5)
        return e

    E = [[eps(i, a) for a in range(2)] for i in range(6)]
    M = np.zeros((6, 6))
    K = np.zeros((2, 2, 6, 6))
    B = np.zeros((2, 3, 6))
    Mp = np.zeros((3, 3))
    for i in range(6):
        for j in range(6):
            M[i, j] = poly.integrate(poly.mul(phi[i], phi[j]), area)
            for a in range(2):
                for b in range(2):
                    s = {}
                    for k in range(2):
                        for l in range(2):
                            s = poly.add(s, poly.mul(E[j][b][k][l], E[i][a][k][l]))
                    K[a, b, i, j] = nu * poly.integrate(s, area)
    for a in range(2):
        for k in range(3):
            for i in range(6):
                B[a, k, i] = poly.integrate(poly.mul(dphi[i][a], psi[k]), area)
    for k in range(3):
        for l in range(3):
            Mp[k, l] = poly.integrate(poly.mul(psi[k], psi[l]), area)
    return dict(M=M, K=K, B=B, Mp=Mp, area=area)


def _assemble(rows_g, cols_g, local, nrows, ncols):
    """Sum element matrices ``local`` (per element type) into CSR with the
    element-connectivity pattern (explicit zeros kept, sorted columns)."""
    R, C, V = [], [], []
    for rg, cg, loc in zip(rows_g, cols_g, local):
        ne = rg.shape[0]
        R.append(np.repeat(rg[:, :, None], cg.shape[1], axis=2).ravel())
        C.append(np.repeat(cg[:, None, :], rg.shape[1], axis=1).ravel())
        V.append(np.broadcast_to(loc, (ne,) + loc.shape).ravel())
    R = np.concatenate(R)
    C = np.concatenate(C)
    V = np.concatenate(V)
    key = R * ncols + C
    uk, inv = np.unique(key, return_inverse=True)
    vals = np.zeros(uk.shape[0])
    np.add.at(vals, inv, V)
    rr = uk // ncols
    cc = uk % ncols
    indptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(indptr, rr + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.csr_matrix((vals, cc.astype(np.int64), indptr), shape=(nrows, ncols))


def assemble(n, nu=1.0, rho=1.0, dt=0.01):
    """Assemble the fluid blocks on the n x n grid.

    Returns a dict:
      Mf              scalar P2 mass (N2 x N2), no boundary condition
      K               dict {(alpha, beta): N2 x N2} of the eps:eps form, no BC
      Bx, By          Np x N2 blocks of B (B = [Bx | By]), no BC
      Mp              P1 pressure mass (Np x Np)
      Af              A_f = (rho/dt) M_f + K_f on [u_x | u_y] (2 N2 x 2 N2), BC applied
      Bbc             B (Np x 2 N2) with boundary columns and row 0 zeroed (pin)
      bnd             boolean mask of boundary P2 nodes
      Af_blocks       dict {(alpha, beta): N2 x N2} of A_f with the BC applied
    """
    p2, p1, vx = triangle_nodes(n)
    N2, Np = (2 * n + 1) ** 2, (n + 1) ** 2
    el = [element_matrices(vx[t], nu) for t in (0, 1)]     # T0 and T1 of cell (0, 0)
    types = [np.arange(0, 2 * n * n, 2), np.arange(1, 2 * n * n, 2)]
    g2 = [p2[ty] for ty in types]
    g1 = [p1[ty] for ty in types]
    Mf = _assemble(g2, g2, [e["M"] for e in el], N2, N2)
    K = {(a, b): _assemble(g2, g2, [e["K"][a, b] for e in el], N2, N2)
         for a in range(2) for b in range(2)}
    Bx = _assemble(g1, g2, [e["B"][0] for e in el], Np, N2)
    By = _assemble(g1, g2, [e["B"][1] for e in el], Np, N2)
    Mp = _assemble(g1, g1, [e["Mp"] for e in el], Np, Np)
    bnd = boundary_p2(n)

    blocks = {}
    for a in range(2):
        for b in range(2):
            A = K[(a, b)].copy()
            if a == b:
                # same pattern: M_f and K_f are both on the P2-P2 connectivity pattern
                A.data = A.data + (rho / dt) * Mf.data
            blocks[(a, b)] = apply_dirichlet(A, bnd, a == b)
    Af = sp.bmat([[blocks[(0, 0)], blocks[(0, 1)]], [blocks[(1, 0)], blocks[(1, 1)]]], format="csr")
    Bxb = mask_columns(Bx, bnd)
    Byb = mask_columns(By, bnd)
    Bxb = zero_row(Bxb, 0)
    Byb = zero_row(Byb, 0)
    Bbc = sp.hstack([Bxb, Byb], format="csr")
    return dict(n=n, N2=N2, Np=Np, Mf=Mf, K=K, Bx=Bx, By=By, Mp=Mp, Af=Af, Af_blocks=blocks,
                Bbc=Bbc, Bx_bc=Bxb, By_bc=Byb, bnd=bnd, nu=nu, rho=rho, dt=dt)


def apply_dirichlet(A, bnd, diag_block):
    """Zero rows and columns of boundary nodes by value; 1 on the diagonal of a
    diagonal block.  The pattern is unchanged."""
    A = A.tocsr().copy()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    hit = bnd[rows] | bnd[cols]
    A.data[hit] = 0.0
    if diag_block:
        A.data[hit & (rows == cols)] = 1.0
    return A


def mask_columns(A, bnd):
    A = A.tocsr().copy()
    A.data[bnd[A.indices]] = 0.0
    return A


def zero_row(A, r):
    A = A.tocsr().copy()
    A.data[A.indptr[r]:A.indptr[r + 1]] = 0.0
    return A


def _adjacent(n, I, J):
    """Triangles (global id, local P2 index of node (I, J)) containing P2 node (I, J)."""
    out = []
    for cj in range(max(0, (J - 1) // 2), min(n - 1, J // 2) + 1):
        for ci in range(max(0, (I - 1) // 2), min(n - 1, I // 2) + 1):
            for t in (0, 1):
                V = [(ci, cj), (ci + 1, cj), (ci + 1, cj + 1)] if t == 0 else \
                    [(ci, cj), (ci + 1, cj + 1), (ci, cj + 1)]
                P = [(2 * a, 2 * b) for (a, b) in V]
                M = [((P[0][0] + P[1][0]) // 2, (P[0][1] + P[1][1]) // 2),
                     ((P[1][0] + P[2][0]) // 2, (P[1][1] + P[2][1]) // 2),
                     ((P[2][0] + P[0][0]) // 2, (P[2][1] + P[0][1]) // 2)]
                nodes = P + M
                if (I, J) in nodes:
                    out.append((2 * (cj * n + ci) + t, nodes.index((I, J)), nodes, V))
    return out


def rows_Af(n, nodes, nu=1.0, rho=1.0, dt=0.01):
    """Rows of A_f (with the boundary condition) at the given P2 nodes, by summing the
    element matrices of the triangles around each node: {node: {col: (xx, xy, yx, yy)}}.
    Also the rows of M_f (no boundary condition): {node: {col: m}}.  For spot checks of
    grids too large to assemble whole."""
    h = 1.0 / n
    el = [element_matrices(np.array([(0, 0), (h, 0), (h, h)]), nu),
          element_matrices(np.array([(0, 0), (h, h), (0, h)]), nu)]
    L = 2 * n + 1
    bnd = lambda I, J: I == 0 or J == 0 or I == 2 * n or J == 2 * n
    A, Mrows = {}, {}
    for r in nodes:
        I, J = r % L, r // L
        row, mrow = {}, {}
        for (T, a, P2, _) in _adjacent(n, I, J):
            e = el[T & 1]
            for b, (I2, J2) in enumerate(P2):
                c = J2 * L + I2
                v = row.setdefault(c, [0.0, 0.0, 0.0, 0.0])
                v[0] += e["K"][0, 0][a, b]
                v[1] += e["K"][0, 1][a, b]
                v[2] += e["K"][1, 0][a, b]
                v[3] += e["K"][1, 1][a, b]
                mrow[c] = mrow.get(c, 0.0) + e["M"][a, b]
        for c in row:
            if bnd(I, J) or bnd(c % L, c // L):
                row[c] = (1.0, 0.0, 0.0, 1.0) if c == r else (0.0, 0.0, 0.0, 0.0)
            else:
                v = row[c]
                row[c] = (v[0] + (rho / dt) * mrow[c], v[1], v[2], v[3] + (rho / dt) * mrow[c])
        A[r] = dict(sorted(row.items()))
        Mrows[r] = dict(sorted(mrow.items()))
    return A, Mrows


def rows_B(n, p1nodes):
    """Rows of B (boundary columns and row 0 zeroed) at P1 nodes: {k: {col: (bx, by)}}."""
    h = 1.0 / n
    el = [element_matrices(np.array([(0, 0), (h, 0), (h, h)]), 1.0),
          element_matrices(np.array([(0, 0), (h, h), (0, h)]), 1.0)]
    L, L1 = 2 * n + 1, n + 1
    out = {}
    for k in p1nodes:
        i, j = k % L1, k // L1
        row = {}
        for (T, a, P2, _) in _adjacent(n, 2 * i, 2 * j):
            e = el[T & 1]
            for b, (I2, J2) in enumerate(P2):
                c = J2 * L + I2
                v = row.setdefault(c, [0.0, 0.0])
                v[0] += e["B"][0, a, b]
                v[1] += e["B"][1, a, b]
        for c in row:
            I2, J2 = c % L, c // L
            if k == 0 or I2 == 0 or J2 == 0 or I2 == 2 * n or J2 == 2 * n:
                row[c] = (0.0, 0.0)
            else:
                row[c] = tuple(row[c])
        out[k] = dict(sorted(row.items()))
    return out


def rows_BT(n, p2nodes):
    """Rows of B^T (boundary rows and column 0 zeroed) at P2 nodes: {r: {p1 col: (bx, by)}}."""
    h = 1.0 / n
    el = [element_matrices(np.array([(0, 0), (h, 0), (h, h)]), 1.0),
          element_matrices(np.array([(0, 0), (h, h), (0, h)]), 1.0)]
    L, L1 = 2 * n + 1, n + 1
    out = {}
    for r in p2nodes:
        I, J = r % L, r // L
        row = {}
        for (T, a, P2, V) in _adjacent(n, I, J):
            e = el[T & 1]
            for kk, (vi, vj) in enumerate(V):
                c = vj * L1 + vi
                v = row.setdefault(c, [0.0, 0.0])
                v[0] += e["B"][0, kk, a]
                v[1] += e["B"][1, kk, a]
        rb = I == 0 or J == 0 or I == 2 * n or J == 2 * n
        out[r] = {c: ((0.0, 0.0) if (rb or c == 0) else tuple(v)) for c, v in sorted(row.items())}
    return out
