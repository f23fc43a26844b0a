"""Nonlinear solid of the oracle: the hyperelastic law of the paper's second test and the
solid residual and tangent it gives on P1 triangles.

Sec. 3: a hyperelastic solid has an energy density W(F) with the first Piola-Kirchhoff stress
P(F) = dW/dF, and elastic energy E(X) = int_B W(F) ds, F = grad_s X.  Sec. 6.2 (nonlinear
solid model) takes the isotropic exponential density
    W(F) = (gamma / (2 eta)) exp(eta [tr(F^T F) - 2]),   gamma = 1.333, eta = 9.242.
Differentiating with |F|^2 = tr(F^T F):
    P(F) = gamma e(F) F,                         e(F) = exp(eta (|F|^2 - 2)),
    dP_ab / dF_cd = gamma e(F) (delta_ac delta_bd + 2 eta F_ab F_cd).
As eta -> 0 the law tends to the linear one, P = gamma F (kappa = gamma).

The discrete solid row of the fully discrete problem (Sec. 4) is (P(F_h), grad_s Y_h)_B -
(lam_h, Y_h)_B = 0.  With X_h P1 on triangles, F is constant on each triangle E and, with G_i
the (constant) gradient of the P1 basis function chi_i on E,
    R(X)_{i,a} = sum_E |E| P_ab(F_E) G_{i,b}            (the residual, 2 Ns entries),
    K(X)_{(i,a),(j,c)} = sum_E |E| dP_ab/dF_cd(F_E) G_{i,b} G_{j,d}
                       = sum_E |E| gamma e(F_E) [ (G_i . G_j) delta_ac + 2 eta (F_E G_i)_a (F_E G_j)_c ]
(the tangent, the Jacobian dR/dX used by Newton's method, Sec. 4 last paragraph).  Vectors are
laid out [x (Ns) | y (Ns)] as everywhere in the oracle.

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import poly

GAMMA = 1.333      # Sec. 6.2
ETA = 9.242        # Sec. 6.2


def W(F, gamma=GAMMA, eta=ETA):
    """Energy density (gamma / (2 eta)) exp(eta (tr F^T F - 2)); eta = 0 gives its limit
    gamma / 2 (|F|^2 - 2) + const, the linear law's density (up to the constant)."""
    t = float(np.sum(F * F)) - 2.0
    if eta == 0.0:
        return 0.5 * gamma * t
    return (gamma / (2.0 * eta)) * np.exp(eta * t)


def P(F, gamma=GAMMA, eta=ETA):
    """First Piola-Kirchhoff stress dW/dF = gamma exp(eta (|F|^2 - 2)) F."""
    return gamma * np.exp(eta * (float(np.sum(F * F)) - 2.0)) * F


def dPdF(F, gamma=GAMMA, eta=ETA):
    """The tangent tensor D[a, b, c, d] = dP_ab / dF_cd."""
    e = gamma * np.exp(eta * (float(np.sum(F * F)) - 2.0))
    I = np.eye(2)
    return e * (np.einsum("ac,bd->abcd", I, I) + 2.0 * eta * np.einsum("ab,cd->abcd", F, F))


def _element(xy_ref, tri_e, X):
    """Reference gradients G (3 x 2) of the P1 basis on E, |E|, and F_E = sum_i X_i G_i^T."""
    G, area = poly.bary_gradients(xy_ref[tri_e])
    G = np.asarray(G, dtype=np.float64)
    F = np.zeros((2, 2))
    for i in range(3):
        F += np.outer(X[tri_e[i]], G[i])
    return G, area, F


def energy(xy_ref, tri, X, gamma=GAMMA, eta=ETA):
    """E(X) = sum_E |E| W(F_E), X [Ns, 2] (Sec. 3, the elastic potential energy)."""
    total = 0.0
    for t in tri:
        _, area, F = _element(xy_ref, t, X)
        total += area * W(F, gamma, eta)
    return total


def residual(xy_ref, tri, X, gamma=GAMMA, eta=ETA):
    """R(X) = (P(F_h), grad chi_i)_B per node and component, [x | y] (2 Ns)."""
    ns = xy_ref.shape[0]
    R = np.zeros((ns, 2))
    for t in tri:
        G, area, F = _element(xy_ref, t, X)
        Pe = P(F, gamma, eta)
        for i in range(3):
            R[t[i]] += area * (Pe @ G[i])
    return np.concatenate([R[:, 0], R[:, 1]])


def tangent(xy_ref, tri, X, gamma=GAMMA, eta=ETA):
    """K(X) = dR/dX (2 Ns x 2 Ns, [x | y] ordering), assembled from the element tangents
    |E| D(F_E)_{abcd} G_{i,b} G_{j,d}."""
    ns = xy_ref.shape[0]
    rows, cols, vals = [], [], []
    for t in tri:
        G, area, F = _element(xy_ref, t, X)
        D = dPdF(F, gamma, eta)
        Ke = area * np.einsum("abcd,ib,jd->iajc", D, G, G)   # [i, a, j, c]
        for i in range(3):
            for a in range(2):
                for j in range(3):
                    for c in range(2):
                        rows.append(a * ns + t[i])
                        cols.append(c * ns + t[j])
                        vals.append(Ke[i, a, j, c])
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * ns, 2 * ns))
