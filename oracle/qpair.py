"""The paper's own element pair (Sec. 4, the discrete spaces): Q2 velocity and discontinuous P1
pressure on the n x n grid of squares, and a Q1 solid (X and lam bilinear on a quadrilateral
mesh of the reference body, S_h = Lambda_h), with the blocks of eq. (matrix).

Numbering and readings (the paper fixes the spaces, not these details):
* Q2 node (I, J), 0 <= I, J <= 2n, sits at (I h/2, J h/2) with index J (2n+1) + I (the same
  lattice as the triangle pair's P2 nodes).  Cell (i, j) holds the nodes (2i + a, 2j + b),
  a, b in {0, 1, 2}, local index a + 3 b; its basis is the tensor product of the quadratic
  Lagrange polynomials at 0, 1/2, 1 of (x - x_i)/h and (y - y_j)/h.
* Pressure: on cell (i, j) (index k = j n + i) the unknowns 3k, 3k + 1, 3k + 2 are the
  coefficients of 1, (x - x_c)/h and (y - y_c)/h, (x_c, y_c) the cell centre.  The pressure
  is pinned at unknown 0 (the constant on cell 0), as the triangle pair pins P1 node 0.
* A_f = (rho/dt) M_f + nu (eps(u), eps(v)), B_ki = (div phi_i, psi_k), M_p = (psi_l, psi_k):
  element integrals by the 3 x 3 Gauss rule on the square, exact for these integrands
  (degree <= 4 in each variable).  Dirichlet rows/columns and the pin as in ``oracle.fluid``.
* Solid quadrilaterals (a, b, c, d) are counter-clockwise; on each, s(xi, eta) = sum_a N_a s_a
  with the bilinear N_a of the unit square; A_s = kappa (grad N_j, grad N_i) and
  C_s = (N_j, N_i) by the 2 x 2 Gauss rule in (xi, eta) (exact on parallelograms).
* C_f(X^n)_lj = sum_E int_E N_l(s) phi_j(X^n(s)) ds.  X^n is bilinear on E, so X^n(E) is the
  quadrilateral of the mapped vertices; its intersection with a fluid cell is clipped as in
  the triangle pair (``oracle.coupling``: x >= x_i, x <= x_{i+1}, y >= y_j, y <= y_{j+1}, no
  diagonal) and kept iff its fan area exceeds 5e-11 h^2.  With x = X^n(s) the integral over a
  piece q is
      int_q N_l(xi(x)) phi_j(x) J_s(xi(x)) / J_X(xi(x)) dx,
  xi(x) the inverse of the bilinear map of E, J_s and J_X the Jacobian determinants of the
  reference and the current bilinear map.  This integrand is not a polynomial when X^n is not
  affine on E; the reading taken is a composite rule: the fan of q from its vertex 0, and on
  each fan triangle (A, B, C) the conical product of 4 x 4 Gauss-Legendre points
  x = A + u (B - A) + u v (C - B) with weight 2 |ABC| u w_u w_v, which is exact for
  polynomials of degree <= 6 and so for every entry when X^n is affine on E (degree 2 + 4).
  xi(x) by Newton's method from the centre of the unit square, to a step below 1e-15.
* Mapped quadrilaterals must be strictly convex, counter-clockwise and inside [0, 1]^2.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fluid as tfluid
from .coupling import MeshError, cell_range, clip_axis, fan_area
from .system import FSISystem, Layout


def sizes(n):
    return dict(N2=(2 * n + 1) ** 2, Np=3 * n * n, ncell=n * n)


def gauss01(k):
    """k-point Gauss-Legendre points and weights on [0, 1]."""
    g, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (g + 1.0), 0.5 * w


def lagrange2(t):
    """Quadratic Lagrange basis at 0, 1/2, 1 and its derivative at the points ``t``:
    two arrays [3, len(t)]."""
    t = np.asarray(t, dtype=np.float64)
    v = np.stack([2.0 * (t - 0.5) * (t - 1.0), 4.0 * t * (1.0 - t), 2.0 * t * (t - 0.5)])
    d = np.stack([4.0 * t - 3.0, 4.0 - 8.0 * t, 4.0 * t - 1.0])
    return v, d


def bilinear(xi, eta):
    """N_a (a = 0..3 for the corners (0,0), (1,0), (1,1), (0,1)) and its derivatives."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    N = np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
    Nx = np.stack([-(1 - eta), 1 - eta, eta, -eta])
    Ne = np.stack([-(1 - xi), -xi, xi, 1 - xi])
    return N, Nx, Ne


# ---------------------------------------------------------------- fluid
def element_matrices(h, nu):
    """Q2 / P1-disc element matrices of a square cell of side h (every cell is the same).

    M (9x9), K (2,2,9,9) with K[alpha, beta, i, j] = nu int eps(phi_j e_beta) : eps(phi_i e_alpha),
    B (2,3,9) with B[alpha, k, i] = int d_alpha phi_i psi_k, Mp (3x3)."""
    t, w = gauss01(3)
    V, D = lagrange2(t)
    npt = 9
    phi = np.zeros((9, npt))
    gx = np.zeros((9, npt))
    gy = np.zeros((9, npt))
    W = np.zeros(npt)
    psi = np.zeros((3, npt))
    for q in range(3):
        for p in range(3):
            g = p + 3 * q
            W[g] = w[p] * w[q] * h * h
            psi[:, g] = [1.0, t[p] - 0.5, t[q] - 0.5]
            for b in range(3):
                for a in range(3):
                    loc = a + 3 * b
                    phi[loc, g] = V[a, p] * V[b, q]
                    gx[loc, g] = D[a, p] * V[b, q] / h
                    gy[loc, g] = V[a, p] * D[b, q] / h

    def eps(i, comp):
        G = np.zeros((2, 2, npt))       # (grad v)_{kl} = d_l v_k: row comp holds grad phi_i
        G[comp, 0] = gx[i]
        G[comp, 1] = gy[i]
        return 0.5 * (G + G.transpose(1, 0, 2))

    E = [[eps(i, a) for a in range(2)] for i in range(9)]
    M = (phi * W) @ phi.T
    K = np.zeros((2, 2, 9, 9))
    for al in range(2):
        for be in range(2):
            for i in range(9):
                for j in range(9):
                    K[al, be, i, j] = nu * np.sum(W * np.sum(E[j][be] * E[i][al], axis=(0, 1)))
    B = np.zeros((2, 3, 9))
    for k in range(3):
        B[0, k] = (gx * psi[k] * W).sum(axis=1)
        B[1, k] = (gy * psi[k] * W).sum(axis=1)
    Mp = (psi * W) @ psi.T
    return dict(M=M, K=K, B=B, Mp=Mp)


def cell_nodes(n):
    """Q2 nodes [n^2, 9] (local order a + 3 b) and pressure unknowns [n^2, 3] of every cell."""
    L = 2 * n + 1
    q2 = np.zeros((n * n, 9), dtype=np.int64)
    pk = np.zeros((n * n, 3), dtype=np.int64)
    for j in range(n):
        for i in range(n):
            k = j * n + i
            q2[k] = [(2 * j + b) * L + 2 * i + a for b in range(3) for a in range(3)]
            pk[k] = [3 * k, 3 * k + 1, 3 * k + 2]
    return q2, pk


def assemble_fluid(n, nu=1.0, rho=1.0, dt=0.01):
    """The fluid blocks of the Q2 / P1-disc pair, in the dict layout of ``oracle.fluid.assemble``."""
    h = 1.0 / n
    N2, Np = (2 * n + 1) ** 2, 3 * n * n
    el = element_matrices(h, nu)
    q2, pk = cell_nodes(n)
    Mf = tfluid._assemble([q2], [q2], [el["M"]], N2, N2)
    K = {(a, b): tfluid._assemble([q2], [q2], [el["K"][a, b]], N2, N2) for a in range(2) for b in range(2)}
    Bx = tfluid._assemble([pk], [q2], [el["B"][0]], Np, N2)
    By = tfluid._assemble([pk], [q2], [el["B"][1]], Np, N2)
    Mp = tfluid._assemble([pk], [pk], [el["Mp"]], Np, Np)
    bnd = tfluid.boundary_p2(n)
    blocks = {}
    for a in range(2):
        for b in range(2):
            A = K[(a, b)].copy()
            if a == b:
                A.data = A.data + (rho / dt) * Mf.data
            blocks[(a, b)] = tfluid.apply_dirichlet(A, bnd, a == b)
    Af = sp.bmat([[blocks[(0, 0)], blocks[(0, 1)]], [blocks[(1, 0)], blocks[(1, 1)]]], format="csr")
    Bxb = tfluid.zero_row(tfluid.mask_columns(Bx, bnd), 0)
    Byb = tfluid.zero_row(tfluid.mask_columns(By, bnd), 0)
    Bbc = sp.hstack([Bxb, Byb], format="csr")
    # integrals of the pressure basis functions (h^2 for the constants, 0 for the slopes)
    p_weights = np.tile([h * h, 0.0, 0.0], n * n)
    return dict(n=n, N2=N2, Np=Np, Mf=Mf, K=K, Bx=Bx, By=By, Mp=Mp, Af=Af, Af_blocks=blocks, Bbc=Bbc,
                Bx_bc=Bxb, By_bc=Byb, bnd=bnd, nu=nu, rho=rho, dt=dt, p_weights=p_weights)


def pressure_interpolant(n, f, fx, fy):
    """P1-disc unknowns of a linear function f (gradient (fx, fy)): per cell the value at the
    centre and h times the gradient."""
    h = 1.0 / n
    out = np.zeros(3 * n * n)
    for j in range(n):
        for i in range(n):
            k = j * n + i
            out[3 * k:3 * k + 3] = [f((i + 0.5) * h, (j + 0.5) * h), fx * h, fy * h]
    return out


# ---------------------------------------------------------------- solid
def assemble_solid(xy, quad, kappa=10.0):
    """Q1 stiffness and mass on the reference quadrilaterals (2 x 2 Gauss rule in (xi, eta)):
    dict with Ks, Ms (= C_s), As (= kappa Ks), areas; the connectivity pattern with explicit
    zeros kept and sorted columns."""
    ns = xy.shape[0]
    t, w = gauss01(2)
    R, C, VK, VM = [], [], [], []
    areas = np.zeros(quad.shape[0])
    for e, qv in enumerate(quad):
        S = xy[qv]
        Ke = np.zeros((4, 4))
        Me = np.zeros((4, 4))
        for p in range(2):
            for q in range(2):
                N, Nx, Ne = bilinear(t[p], t[q])
                J = np.array([[Nx @ S[:, 0], Ne @ S[:, 0]], [Nx @ S[:, 1], Ne @ S[:, 1]]])
                det = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
                if not det > 0.0:
                    raise ValueError(f"solid reference quadrilateral {e} is degenerate or clockwise")
                G = np.linalg.solve(J.T, np.stack([Nx, Ne]))     # [2, 4]: grad_s N_a
                ww = w[p] * w[q] * det
                Ke += ww * (G.T @ G)
                Me += ww * np.outer(N, N)
                areas[e] += ww
        for a in range(4):
            for b in range(4):
                R.append(qv[a])
                C.append(qv[b])
                VK.append(Ke[a, b])
                VM.append(Me[a, b])
    R = np.asarray(R, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    uk, inv = np.unique(R * ns + C, return_inverse=True)
    vk = np.zeros(uk.shape[0])
    vm = np.zeros(uk.shape[0])
    np.add.at(vk, inv, np.asarray(VK))
    np.add.at(vm, inv, np.asarray(VM))
    rows, cols = uk // ns, uk % ns
    indptr = np.zeros(ns + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    Ks = sp.csr_matrix((vk, cols, indptr), shape=(ns, ns))
    Ms = sp.csr_matrix((vm, cols, indptr), shape=(ns, ns))
    As = Ks.copy()
    As.data = kappa * As.data
    return dict(Ks=Ks, Ms=Ms, As=As, areas=areas)


# ---------------------------------------------------------------- coupling
def check_map(Xn, quad):
    """Every mapped quadrilateral strictly convex, counter-clockwise and inside [0, 1]^2."""
    for e, qv in enumerate(quad):
        P = Xn[qv]
        if (P < 0.0).any() or (P > 1.0).any():
            raise MeshError(f"solid quadrilateral {e} leaves the fluid domain under X^n")
        for k in range(4):
            a, b, c = P[k - 1], P[k], P[(k + 1) % 4]
            if not (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]) > 0.0:
                raise MeshError(f"solid quadrilateral {e} is not convex and counter-clockwise under X^n")


def cell_piece(P, n, i, j):
    """The intersection polygon of the mapped quadrilateral P (4 CCW points) with cell (i, j),
    or None when it is not kept."""
    h = 1.0 / n
    pts = [tuple(p) for p in P]
    pts = clip_axis(pts, 0, i / n, True)
    pts = clip_axis(pts, 0, (i + 1) / n, False)
    pts = clip_axis(pts, 1, j / n, True)
    pts = clip_axis(pts, 1, (j + 1) / n, False)
    if len(pts) >= 3 and fan_area(pts) > 5e-11 * h * h:
        return pts
    return None


def intersections(Xn, quad, n, brute_force=False):
    """[(E, cell, polygon)]: by quadrilateral, then cell (j major, i minor); ``brute_force``
    tests every cell instead of the bounding box's."""
    check_map(Xn, quad)
    out = []
    for e, qv in enumerate(quad):
        P = [tuple(Xn[k]) for k in qv]
        i0, i1, j0, j1 = (0, n - 1, 0, n - 1) if brute_force else cell_range(P, n)
        for j in range(j0, j1 + 1):
            for i in range(i0, i1 + 1):
                q = cell_piece(P, n, i, j)
                if q is not None:
                    out.append((e, j * n + i, q))
    return out


def inverse_bilinear(P, x, y):
    """(xi, eta) with sum_a N_a(xi, eta) P_a = (x, y), by Newton's method from (1/2, 1/2)."""
    xi = np.full_like(x, 0.5)
    eta = np.full_like(x, 0.5)
    for _ in range(60):
        N, Nx, Ne = bilinear(xi, eta)
        fx = P[:, 0] @ N - x
        fy = P[:, 1] @ N - y
        a, b = P[:, 0] @ Nx, P[:, 0] @ Ne
        c, d = P[:, 1] @ Nx, P[:, 1] @ Ne
        det = a * d - b * c
        dxi = (d * fx - b * fy) / det
        deta = (a * fy - c * fx) / det
        xi = xi - dxi
        eta = eta - deta
        if max(np.abs(dxi).max(), np.abs(deta).max()) <= 1e-15:
            break
    return xi, eta


def jacobian(P, xi, eta):
    _, Nx, Ne = bilinear(xi, eta)
    return (P[:, 0] @ Nx) * (P[:, 1] @ Ne) - (P[:, 0] @ Ne) * (P[:, 1] @ Nx)


def piece_matrix(P, S, q, i, j, n, k=4, split=0):
    """4 x 9 matrix int_q N_a(xi(x)) phi_b(x) J_s / J_X dx over polygon ``q`` in cell (i, j):
    the fan from vertex 0, the conical product of k x k Gauss-Legendre points on each fan
    triangle (``split`` > 0: each fan triangle cut into 4^split similar ones first, for checks)."""
    u, wu = gauss01(k)
    U, Vv = np.meshgrid(u, u, indexing="ij")
    U, Vv = U.ravel(), Vv.ravel()
    Wt = np.outer(wu, wu).ravel()
    L = np.zeros((4, 9))
    tris = [(np.asarray(q[0]), np.asarray(q[m]), np.asarray(q[m + 1])) for m in range(1, len(q) - 1)]
    for _ in range(split):
        nxt = []
        for A, B, C in tris:
            ab, bc, ca = 0.5 * (A + B), 0.5 * (B + C), 0.5 * (C + A)
            nxt += [(A, ab, ca), (ab, B, bc), (ca, bc, C), (bc, ca, ab)]
        tris = nxt
    for A, B, C in tris:
        two = (B[0] - A[0]) * (C[1] - A[1]) - (C[0] - A[0]) * (B[1] - A[1])
        x = A[0] + U * (B[0] - A[0]) + U * Vv * (C[0] - B[0])
        y = A[1] + U * (B[1] - A[1]) + U * Vv * (C[1] - B[1])
        w = Wt * U * two
        xi, eta = inverse_bilinear(P, x, y)
        N, _, _ = bilinear(xi, eta)
        ratio = jacobian(S, xi, eta) / jacobian(P, xi, eta)
        Vx, _ = lagrange2(x * n - i)
        Vy, _ = lagrange2(y * n - j)
        phi = np.stack([Vx[a] * Vy[b] for b in range(3) for a in range(3)])
        L += np.einsum("ap,bp,p->ab", N, phi, w * ratio)
    return L


def assemble_coupling(Xn, xy_ref, quad, n, brute_force=False, k=4, split=0):
    """C_f(X^n) as a scalar (Ns x N2) CSR matrix with Dirichlet columns zeroed, and the piece
    list [(E, cell)]."""
    N2 = (2 * n + 1) ** 2
    ns = xy_ref.shape[0]
    q2, _ = cell_nodes(n)
    bnd = tfluid.boundary_p2(n)
    pieces = intersections(Xn, quad, n, brute_force=brute_force)
    R, C, V = [], [], []
    for (e, cell, q) in pieces:
        qv = quad[e]
        L = piece_matrix(Xn[qv], xy_ref[qv], q, cell % n, cell // n, n, k=k, split=split)
        for a in range(4):
            for b in range(9):
                R.append(qv[a])
                C.append(q2[cell, b])
                V.append(L[a, b])
    if not R:
        return sp.csr_matrix((ns, N2)), []
    R = np.asarray(R, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    uk, inv = np.unique(R * N2 + C, return_inverse=True)
    vals = np.zeros(uk.shape[0])
    np.add.at(vals, inv, np.asarray(V))
    rows, cols = uk // N2, uk % N2
    indptr = np.zeros(ns + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    vals[bnd[cols]] = 0.0
    return sp.csr_matrix((vals, cols, indptr), shape=(ns, N2)), [(e, c) for (e, c, _) in pieces]


# ---------------------------------------------------------------- the system
class QSystem(FSISystem):
    """eq. (matrix) with the Q2 / P1-disc fluid and the Q1 solid; the unknown vector, the
    super-blocks, the direct solve and the block preconditioners are those of ``FSISystem``."""

    def __init__(self, n, xy_ref, quad, nu=1.0, rho=1.0, kappa=10.0, dt=0.01):
        self.n = n
        self.xy_ref = np.asarray(xy_ref, dtype=np.float64)
        self.tri = np.asarray(quad, dtype=np.int64)   # the solid elements (quadrilaterals)
        self.nu, self.rho, self.kappa, self.dt = nu, rho, kappa, dt
        self.F = assemble_fluid(n, nu=nu, rho=rho, dt=dt)
        self.S = assemble_solid(self.xy_ref, self.tri, kappa=kappa)
        self.lay = Layout(self.F["N2"], self.F["Np"], self.xy_ref.shape[0])
        self.Cf = None
        self.pieces = None
        self._lu11 = None
        self._lu22 = None

    @classmethod
    def from_workload(cls, wl):
        xy, quad = wl.solid_mesh()
        return cls(wl.n, xy, quad, nu=wl.nu, rho=wl.rho, kappa=wl.kappa, dt=wl.dt)

    def set_position(self, Xn):
        self.Xn = np.asarray(Xn, dtype=np.float64)
        self.Cf, self.pieces = assemble_coupling(self.Xn, self.xy_ref, self.tri, self.n)
        self._lu11 = None
        return self.Cf
