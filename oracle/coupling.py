"""Coupling matrix C_f(X^n) of the oracle.

Sec. 4 (block definitions after eq. (matrix)):
  (C_f)_lj = (chi_l, phi_j(X^n))_B = sum_E int_E chi_l(s) phi_j(X^n(s)) ds.
The solid map X^n is P1, hence affine on every solid triangle E, and the change of
variables x = X^n(s) gives
  int_E chi_l phi_j(X^n) ds = (|E| / |X^n(E)|) int_{X^n(E)} lam_l(x) phi_j(x) dx,
where lam_l are the barycentric coordinates of the mapped triangle X^n(E).  The paper
integrates exactly by intersecting X^n(E) with the fluid elements: candidates come from
the bounding box of X^n(E) on the Cartesian fluid grid, the intersections are computed by
Sutherland-Hodgman clipping (Sec. 4, the paragraph on the coupling assembly), and each
intersection polygon is integrated exactly.  The integrand lam_l * phi_j is a cubic on
each piece.

Reading of the degenerate cases (the paper is silent; the HIP path follows the same
reading so that both produce the same intersection list bit for bit):
* The mapped triangle (CCW) is clipped against x >= x_i, x <= x_{i+1}, y >= y_j,
  y <= y_{j+1} (in that order), with x_i = i / n, y_j = j / n; the result is split by
  the cell diagonal f = (x - x_i) - (y - y_j): f >= 0 is the triangle T0 = (v00, v10, v11),
  -f >= 0 the triangle T1 = (v00, v11, v01).
* Against each half-plane g >= 0 a vertex v is kept iff g(v) >= 0; a crossing point
  a + t (b - a), t = g(a) / (g(a) - g(b)), is emitted only when g(a), g(b) have strictly
  opposite signs; on an axis line the clipped coordinate is set to the line value.
* A piece is kept iff its fan (shoelace) area from vertex 0 exceeds 5e-11 * h * h
  (1e-10 of a fluid triangle's area).
* Candidate cells: i in [floor(xmin * n), floor(xmax * n)] and the same for j, clamped
  to [0, n-1].  Pieces are listed by solid triangle, then cell (j major, i minor), then
  fluid triangle t = 0, 1.
* Columns of Dirichlet velocity nodes are kept in the pattern and zeroed by value.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fluid, poly, quadrature


class MeshError(ValueError):
    """X^n maps a solid triangle to a degenerate/inverted triangle or outside the square."""


def _cross(ax, ay, bx, by):
    return ax * by - bx * ay


def signed_area(P):
    (x0, y0), (x1, y1), (x2, y2) = P
    return 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))


def clip_axis(poly_pts, axis, c, keep_ge):
    """Sutherland-Hodgman clip of a polygon (list of (x, y)) against one axis line.

    ``axis`` 0 is x, 1 is y; ``keep_ge`` keeps coordinate >= c, otherwise <= c."""
    out = []
    m = len(poly_pts)
    for k in range(m):
        a = poly_pts[k]
        b = poly_pts[(k + 1) % m]
        fa = (a[axis] - c) if keep_ge else (c - a[axis])
        fb = (b[axis] - c) if keep_ge else (c - b[axis])
        if fa >= 0.0:
            out.append(a)
        if (fa > 0.0 and fb < 0.0) or (fa < 0.0 and fb > 0.0):
            t = fa / (fa - fb)
            if axis == 0:
                out.append((c, a[1] + t * (b[1] - a[1])))
            else:
                out.append((a[0] + t * (b[0] - a[0]), c))
    return out


def clip_diagonal(poly_pts, xi, yj, upper):
    """Clip against the cell diagonal: keep (x - xi) - (y - yj) >= 0 (lower-right
    triangle T0) or, with ``upper``, (y - yj) - (x - xi) >= 0 (upper-left T1)."""
    out = []
    m = len(poly_pts)
    for k in range(m):
        a = poly_pts[k]
        b = poly_pts[(k + 1) % m]
        if upper:
            fa = (a[1] - yj) - (a[0] - xi)
            fb = (b[1] - yj) - (b[0] - xi)
        else:
            fa = (a[0] - xi) - (a[1] - yj)
            fb = (b[0] - xi) - (b[1] - yj)
        if fa >= 0.0:
            out.append(a)
        if (fa > 0.0 and fb < 0.0) or (fa < 0.0 and fb > 0.0):
            t = fa / (fa - fb)
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    return out


def fan_area(pts):
    """Shoelace area of a polygon as a fan from vertex 0 (accumulated in order)."""
    if len(pts) < 3:
        return 0.0
    x0, y0 = pts[0]
    s = 0.0
    for k in range(1, len(pts) - 1):
        s += (pts[k][0] - x0) * (pts[k + 1][1] - y0) - (pts[k + 1][0] - x0) * (pts[k][1] - y0)
    return 0.5 * s


def cell_pieces(P, n, i, j):
    """Clip the mapped triangle P (3 CCW points) with fluid cell (i, j).

    Returns a list of (t, polygon) for the two fluid triangles t = 0, 1 whose piece
    is kept (area above the threshold)."""
    h = 1.0 / n
    tau = 5e-11 * h * h
    xi, xi1 = i / n, (i + 1) / n
    yj, yj1 = j / n, (j + 1) / n
    pts = [tuple(p) for p in P]
    pts = clip_axis(pts, 0, xi, True)
    pts = clip_axis(pts, 0, xi1, False)
    pts = clip_axis(pts, 1, yj, True)
    pts = clip_axis(pts, 1, yj1, False)
    out = []
    if len(pts) < 3:
        return out
    for t in (0, 1):
        q = clip_diagonal(pts, xi, yj, upper=(t == 1))
        if len(q) >= 3 and fan_area(q) > tau:
            out.append((t, q))
    return out


def cell_range(P, n):
    xs = [p[0] for p in P]
    ys = [p[1] for p in P]
    i0 = min(max(int(math.floor(min(xs) * n)), 0), n - 1)
    i1 = min(max(int(math.floor(max(xs) * n)), 0), n - 1)
    j0 = min(max(int(math.floor(min(ys) * n)), 0), n - 1)
    j1 = min(max(int(math.floor(max(ys) * n)), 0), n - 1)
    return i0, i1, j0, j1


def check_map(Xn, tri):
    """Validity of X^n: every mapped triangle has positive area and lies in [0,1]^2."""
    for e, t in enumerate(tri):
        P = Xn[t]
        if not signed_area(P) > 0.0:
            raise MeshError(f"solid triangle {e} is degenerate or inverted under X^n")
        if (P < 0.0).any() or (P > 1.0).any():
            raise MeshError(f"solid triangle {e} leaves the fluid domain under X^n")


def intersections(Xn, tri, n, brute_force=False):
    """The list of intersection pieces [(E, T, polygon)] in the canonical order.

    ``brute_force`` tests every fluid cell for every solid triangle (the paper's nested
    loop); otherwise only the cells of the bounding box are tested."""
    check_map(Xn, tri)
    out = []
    for e, t in enumerate(tri):
        P = [tuple(Xn[k]) for k in t]
        if brute_force:
            i0, i1, j0, j1 = 0, n - 1, 0, n - 1
        else:
            i0, i1, j0, j1 = cell_range(P, n)
        for j in range(j0, j1 + 1):
            for i in range(i0, i1 + 1):
                for (tt, q) in cell_pieces(P, n, i, j):
                    out.append((e, 2 * (j * n + i) + tt, q))
    return out


def _bary(P, x, y):
    """Barycentric coordinates of (x, y) in triangle P."""
    (x0, y0), (x1, y1), (x2, y2) = P
    d = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    l0 = ((x1 - x) * (y2 - y) - (x2 - x) * (y1 - y)) / d
    l1 = ((x2 - x) * (y0 - y) - (x0 - x) * (y2 - y)) / d
    l2 = ((x0 - x) * (y1 - y) - (x1 - x) * (y0 - y)) / d
    return l0, l1, l2


_P2 = poly.p2_basis()


def piece_matrix(Pmapped, Tverts, q):
    """3x6 matrix int_piece lam_l(x) phi_j(x) dx over polygon ``q`` (fan of triangles
    from vertex 0, each integrated with the degree-3 rule of ``oracle.quadrature``)."""
    pts, wts = quadrature.cubic_rule()
    L = np.zeros((3, 6))
    x0, y0 = q[0]
    for k in range(1, len(q) - 1):
        tri_pts = [q[0], q[k], q[k + 1]]
        a = fan_area(tri_pts)
        for (b0, b1, b2), w in zip(pts, wts):
            x = b0 * tri_pts[0][0] + b1 * tri_pts[1][0] + b2 * tri_pts[2][0]
            y = b0 * tri_pts[0][1] + b1 * tri_pts[1][1] + b2 * tri_pts[2][1]
            lam = _bary(Pmapped, x, y)
            mu = _bary(Tverts, x, y)
            phi = [poly.evaluate(f, *mu) for f in _P2]
            for l in range(3):
                for jj in range(6):
                    L[l, jj] += w * a * lam[l] * phi[jj]
    return L


def assemble(Xn, xy_ref, tri, n, brute_force=False):
    """C_f(X^n) as a scalar (Ns x N2) CSR matrix with Dirichlet columns zeroed.

    Returns ``(Cf, pieces)`` where ``pieces`` is the list of (E, T) pairs."""
    N2 = (2 * n + 1) ** 2
    ns = xy_ref.shape[0]
    p2, _, vx = fluid.triangle_nodes(n)
    bnd = fluid.boundary_p2(n)
    pieces = intersections(Xn, tri, n, brute_force=brute_force)
    R, C, V = [], [], []
    for (e, T, q) in pieces:
        t = tri[e]
        Pm = [tuple(Xn[k]) for k in t]
        ratio = signed_area(xy_ref[t]) / signed_area(Pm)
        L = ratio * piece_matrix(Pm, [tuple(v) for v in vx[T]], q)
        for l in range(3):
            for jj in range(6):
                R.append(t[l])
                C.append(p2[T, jj])
                V.append(L[l, jj])
    if not R:
        Cf = sp.csr_matrix((ns, N2))
    else:
        R = np.asarray(R, dtype=np.int64)
        C = np.asarray(C, dtype=np.int64)
        key = R * N2 + C
        uk, inv = np.unique(key, return_inverse=True)
        vals = np.zeros(uk.shape[0])
        np.add.at(vals, inv, np.asarray(V))
        rows = uk // N2
        cols = uk % N2
        indptr = np.zeros(ns + 1, dtype=np.int64)
        np.add.at(indptr, rows + 1, 1)
        indptr = np.cumsum(indptr)
        vals[bnd[cols]] = 0.0
        Cf = sp.csr_matrix((vals, cols, indptr), shape=(ns, N2))
    return Cf, [(e, T) for (e, T, _) in pieces]
