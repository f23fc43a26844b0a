"""Quadrature rules on triangles used by the oracle.

* ``cubic_rule``: the 7-point rule with the three vertices (weight 1/20), the three
  edge midpoints (2/15) and the centroid (9/20), times the area.  All weights are
  positive and the rule is exact for polynomials of degree <= 3, which is the degree
  of the coupling integrand chi_l * phi_j (P1 times P2) on a piece of an intersection
  (the paper's "exact quadrature rule", Sec. 4).
* ``conical_rule(k)``: Stroud's conical product of Gauss-Legendre rules
  (Duffy collapse) with k x k Gauss-Legendre points, exact to degree 2k-2; used for the manufactured
  solution (non-polynomial data) and for checks.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np

# barycentric points and weights (weights sum to 1; multiply by the area)
CUBIC_POINTS = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0),
                (0.5, 0.5, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5),
                (1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0)]
CUBIC_WEIGHTS = [1.0 / 20.0] * 3 + [2.0 / 15.0] * 3 + [9.0 / 20.0]


def cubic_rule():
    return list(CUBIC_POINTS), list(CUBIC_WEIGHTS)


def conical_rule(k: int):
    """Barycentric points/weights (weights sum to 1) exact to degree 2k-2 on a triangle."""
    # map the square [0,1]^2 onto the triangle: x = u, y = v (1 - u); Jacobian (1 - u)
    gu, wu = np.polynomial.legendre.leggauss(k)
    gv, wv = np.polynomial.legendre.leggauss(k)
    pts, wts = [], []
    for a, wa in zip(gu, wu):
        u = 0.5 * (a + 1.0)
        for b, wb in zip(gv, wv):
            v = 0.5 * (b + 1.0)
            x = u
            y = v * (1.0 - u)
            # reference triangle (0,0),(1,0),(0,1): area 1/2
            w = 0.25 * wa * wb * (1.0 - u) * 2.0
            pts.append((1.0 - x - y, x, y))
            wts.append(w)
    return pts, wts
