"""Solid blocks of the oracle: P1 stiffness and mass on the solid reference mesh.

Sec. 4, eq. (matrix) and the block definitions after it, for the linear law
P(F) = kappa F:
  (A_s)_ij = kappa (grad chi_j, grad chi_i)_B,   (C_s)_lj = (chi_l, chi_j)_B.
X and lambda are both P1 on the same mesh (S_h = Lambda_h, Sec. 4), and every block acts
on the two components separately (block diagonal over x and y); the scalar matrices are
returned here.  The integrals are exact (``oracle.poly``).

Test infrastructure (FP64 oracle); see ``oracle/__init__.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import poly


def element_matrices(p):
    """Exact P1 stiffness (3x3) and mass (3x3) on triangle ``p`` (3x2, CCW)."""
    grads, area = poly.bary_gradients(p)
    if area <= 0.0:
        raise ValueError("solid reference triangle is degenerate or clockwise")
    phi = poly.p1_basis()
    K = np.zeros((3, 3))
    M = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            K[i, j] = area * (grads[i][0] * grads[j][0] + grads[i][1] * grads[j][1])
            M[i, j] = poly.integrate(poly.mul(phi[i], phi[j]), area)
    return K, M, area


def assemble(xy, tri, kappa=10.0):
    """Return dict with Ks (P1 stiffness), Ms (= C_s), As (= kappa Ks), areas.

    Both matrices share the P1 connectivity pattern (explicit zeros kept, sorted
    columns)."""
    ns = xy.shape[0]
    R, C, VK, VM = [], [], [], []
    areas = np.zeros(tri.shape[0])
    for e, t in enumerate(tri):
        K, M, a = element_matrices(xy[t])
        areas[e] = a
        for i in range(3):
            for j in range(3):
                R.append(t[i])
                C.append(t[j])
                VK.append(K[i, j])
                VM.append(M[i, j])
    R = np.asarray(R, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    key = R * ns + C
    uk, inv = np.unique(key, return_inverse=True)
    vk = np.zeros(uk.shape[0])
    vm = np.zeros(uk.shape[0])
    np.add.at(vk, inv, np.asarray(VK))
    np.add.at(vm, inv, np.asarray(VM))
    rows = uk // ns
    cols = uk % ns
    indptr = np.zeros(ns + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    Ks = sp.csr_matrix((vk, cols, indptr), shape=(ns, ns))
    Ms = sp.csr_matrix((vm, cols, indptr), shape=(ns, ns))
    As = sp.csr_matrix((kappa * vk, cols, indptr), shape=(ns, ns))
    return dict(Ks=Ks, Ms=Ms, As=As, areas=areas, kappa=kappa)
