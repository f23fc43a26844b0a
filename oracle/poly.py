"""Polynomials in the barycentric coordinates of a triangle, integrated exactly.

A polynomial is a dict ``{(a, b, c): coeff}`` standing for
sum coeff * l1^a * l2^b * l3^c.  The exact integral over a triangle T uses the
classical formula  int_T l1^a l2^b l3^c = 2|T| a! b! c! / (a+b+c+2)!.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

from math import factorial


def mono(a, b, c, coeff=1.0):
    return {(a, b, c): float(coeff)}


def add(p, q, s=1.0):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0.0) + s * v
    return out


def mul(p, q):
    out = {}
    for (a, b, c), u in p.items():
        for (d, e, f), v in q.items():
            k = (a + d, b + e, c + f)
            out[k] = out.get(k, 0.0) + u * v
    return out


def scale(p, s):
    return {k: s * v for k, v in p.items()}


def diff(p, k):
    """Partial derivative with respect to l_{k+1} (k = 0, 1, 2)."""
    out = {}
    for e, v in p.items():
        if e[k] == 0:
            continue
        e2 = list(e)
        e2[k] -= 1
        out[tuple(e2)] = out.get(tuple(e2), 0.0) + v * e[k]
    return out


def integrate(p, area):
    """Exact integral over a triangle of area ``area``."""
    s = 0.0
    for (a, b, c), v in p.items():
        s += v * 2.0 * area * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
    return s


def evaluate(p, l1, l2, l3):
    s = 0.0
    for (a, b, c), v in p.items():
        s += v * (l1 ** a) * (l2 ** b) * (l3 ** c)
    return s


L = [mono(1, 0, 0), mono(0, 1, 0), mono(0, 0, 1)]


def p1_basis():
    """P1 basis: the barycentric coordinates themselves."""
    return [dict(l) for l in L]


def p2_basis():
    """P2 basis in the local order (a, b, c, ab, bc, ca): vertex l(2l-1), edge 4 l l'."""
    v = [add(scale(mul(l, l), 2.0), l, -1.0) for l in L]
    e = [scale(mul(L[0], L[1]), 4.0), scale(mul(L[1], L[2]), 4.0), scale(mul(L[2], L[0]), 4.0)]
    return v + e


def bary_gradients(p):
    """Gradients of l1, l2, l3 and the signed area of triangle ``p`` (3x2)."""
    (x1, y1), (x2, y2), (x3, y3) = p
    d = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1)   # twice the signed area
    g = [((y2 - y3) / d, (x3 - x2) / d),
         ((y3 - y1) / d, (x1 - x3) / d),
         ((y1 - y2) / d, (x2 - x1) / d)]
    return g, 0.5 * d


def gradient(p_poly, grads):
    """Physical gradient of a barycentric polynomial: list of two polynomials (d/dx, d/dy)."""
    out = []
    for comp in range(2):
        acc = {}
        for k in range(3):
            acc = add(acc, diff(p_poly, k), grads[k][comp])
        out.append(acc)
    return out
