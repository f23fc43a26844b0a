"""Pins of the oracle's finite-element blocks against facts fixed by the mathematics.

CPU only.  Each test checks the oracle against something other than itself: numerical
quadrature from a library rule, closed-form integrals of specific fields, brute-force
counts, and invariants of the bilinear forms of Sec. 4, eq. (matrix).
"""
import itertools

import numpy as np
import pytest

from oracle import fluid, poly, quadrature, solid
from paper_2301_10041_amd import inputs


def _gauss_triangle(P, f, k=8):
    """Integrate f(x, y) over triangle P with a Gauss-Legendre product rule (Duffy)."""
    g, w = np.polynomial.legendre.leggauss(k)
    u = 0.5 * (g + 1.0)
    wu = 0.5 * w
    P = np.asarray(P, dtype=float)
    J = abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    s = 0.0
    for a, wa in zip(u, wu):
        for b, wb in zip(u, wu):
            r, t = a, b * (1 - a)
            x = P[0] + r * (P[1] - P[0]) + t * (P[2] - P[0])
            s += wa * wb * (1 - a) * f(x[0], x[1])
    return s * J


def test_barycentric_integrals_against_library_quadrature():
    rng = np.random.default_rng(1)
    for _ in range(5):
        P = rng.uniform(-1, 1, (3, 2))
        grads, area = poly.bary_gradients(P)
        A = abs(area)
        for a, b, c in itertools.product(range(4), repeat=3):
            if a + b + c > 4:
                continue

            def f(x, y):
                # barycentric coordinates by solving the affine system
                T = np.array([[P[0, 0], P[1, 0], P[2, 0]], [P[0, 1], P[1, 1], P[2, 1]], [1, 1, 1]])
                l = np.linalg.solve(T, np.array([x, y, 1.0]))
                return l[0] ** a * l[1] ** b * l[2] ** c
            ref = _gauss_triangle(P, f, k=6)
            assert poly.integrate(poly.mono(a, b, c), A) == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_cubic_rule_exact_to_degree_3_and_not_4():
    rng = np.random.default_rng(2)
    pts, wts = quadrature.cubic_rule()
    assert sum(wts) == pytest.approx(1.0, abs=1e-15)
    assert min(wts) > 0
    P = rng.uniform(0, 1, (3, 2))
    A = abs(poly.bary_gradients(P)[1])
    for a, b in itertools.product(range(5), repeat=2):
        if a + b > 4:
            continue
        f = lambda x, y: x ** a * y ** b
        ref = _gauss_triangle(P, f, k=6)
        q = sum(w * f(*(l0 * P[0] + l1 * P[1] + l2 * P[2])) for (l0, l1, l2), w in zip(pts, wts)) * A
        if a + b <= 3:
            assert q == pytest.approx(ref, rel=1e-13, abs=1e-15)
    # degree 4 is not integrated exactly (the rule is exactly cubic)
    f = lambda x, y: x ** 4
    ref = _gauss_triangle(P, f, k=6)
    q = sum(w * f(*(l0 * P[0] + l1 * P[1] + l2 * P[2])) for (l0, l1, l2), w in zip(pts, wts)) * A
    assert abs(q - ref) > 1e-8 * abs(ref)


def test_p2_basis_is_nodal_and_a_partition_of_unity():
    nodes = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0.5, 0.5, 0), (0, 0.5, 0.5), (0.5, 0, 0.5)]
    B = poly.p2_basis()
    for i, f in enumerate(B):
        for j, nd in enumerate(nodes):
            assert poly.evaluate(f, *nd) == pytest.approx(1.0 if i == j else 0.0, abs=1e-15)
    for l in [(0.2, 0.3, 0.5), (0.7, 0.1, 0.2)]:
        assert sum(poly.evaluate(f, *l) for f in B) == pytest.approx(1.0, abs=1e-15)


def _brute_pattern_counts(n):
    p2, p1, _ = fluid.triangle_nodes(n)
    s22, s12 = set(), set()
    for t in range(p2.shape[0]):
        for a in p2[t]:
            for b in p2[t]:
                s22.add((a, b))
        for a in p1[t]:
            for b in p2[t]:
                s12.add((a, b))
    return len(s22), len(s12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_pattern_sizes_closed_form_and_brute_force(n):
    F = fluid.assemble(n)
    z22, z12 = _brute_pattern_counts(n)
    assert F["Mf"].nnz == z22 == 46 * n * n + 16 * n + 1
    assert F["Bx"].nnz == z12 == 19 * n * n + 10 * n + 1
    for key in F["K"]:
        assert F["K"][key].nnz == z22
    # sorted columns
    for A in (F["Mf"], F["Bx"], F["Af"]):
        for r in range(A.shape[0]):
            c = A.indices[A.indptr[r]:A.indptr[r + 1]]
            assert np.all(np.diff(c) > 0)


@pytest.fixture(scope="module")
def F8():
    return fluid.assemble(8, nu=1.0, rho=1.0, dt=0.01)


def _interp(n, f):
    X = fluid.p2_coords(n)
    return f(X[:, 0], X[:, 1])


def test_mass_matrix_sums(F8):
    n = 8
    M = F8["Mf"]
    assert M.sum() == pytest.approx(1.0, abs=1e-14)          # |Omega| = 1
    rs = np.asarray(M.sum(axis=1)).ravel()
    I, J = np.meshgrid(np.arange(2 * n + 1), np.arange(2 * n + 1), indexing="xy")
    vertex = ((I % 2 == 0) & (J % 2 == 0)).ravel()
    assert np.abs(rs[vertex]).max() < 1e-16                  # vertex functions integrate to 0
    # an edge function integrates to |T|/3 on each of its (1 or 2) triangles
    p2, _, _ = fluid.triangle_nodes(n)
    count = np.zeros(M.shape[0])
    for t in range(p2.shape[0]):
        for k in p2[t, 3:]:
            count[k] += 1
    h = 1.0 / n
    assert np.allclose(rs[~vertex], count[~vertex] * (h * h / 2) / 3, rtol=1e-13, atol=0)
    assert abs(M - M.T).max() < 1e-17
    assert np.linalg.eigvalsh(M.toarray()).min() > 0


def test_stiffness_kernel_rigid_motions_and_energy(F8):
    n = 8
    K = F8["K"]

    def Kmul(ux, uy):
        return (K[(0, 0)] @ ux + K[(0, 1)] @ uy, K[(1, 0)] @ ux + K[(1, 1)] @ uy)

    one = np.ones(K[(0, 0)].shape[0])
    zero = np.zeros_like(one)
    for (ux, uy) in ((one, zero), (zero, one), (-_interp(n, lambda x, y: y), _interp(n, lambda x, y: x))):
        a, b = Kmul(ux, uy)
        assert np.abs(a).max() < 1e-12 and np.abs(b).max() < 1e-12
    # interior rows vanish for any linear field (eps(u) constant)
    ux = _interp(n, lambda x, y: 0.3 * x - 1.7 * y + 0.2)
    uy = _interp(n, lambda x, y: 2.1 * x + 0.4 * y)
    a, b = Kmul(ux, uy)
    bnd = fluid.boundary_p2(n)
    assert np.abs(a[~bnd]).max() < 1e-12 and np.abs(b[~bnd]).max() < 1e-12
    # energy of u = (x^2, x y): eps = [[2x, y/2], [y/2, x]], int eps:eps = 11/6 (nu = 1)
    ux = _interp(n, lambda x, y: x * x)
    uy = _interp(n, lambda x, y: x * y)
    a, b = Kmul(ux, uy)
    assert ux @ a + uy @ b == pytest.approx(11.0 / 6.0, rel=1e-12)
    # symmetric, cross blocks transposes of each other
    assert abs(K[(0, 1)] - K[(1, 0)].T).max() < 1e-15


def test_divergence_block(F8):
    n = 8
    Bx, By, Mp = F8["Bx"], F8["By"], F8["Mp"]
    bnd = fluid.boundary_p2(n)
    ones = np.ones(Bx.shape[0])
    assert np.abs((Bx.T @ ones)[~bnd]).max() < 1e-14         # B^T applied to constant pressure
    assert np.abs((By.T @ ones)[~bnd]).max() < 1e-14
    # u = curl(psi) of a cubic psi is an exactly divergence-free P2 field
    psi_y = lambda x, y: 2 * x * y + x * x - 3 * y * y       # psi = x y^2 + x^2 y - y^3
    psi_x = lambda x, y: y * y + 2 * x * y
    ux = _interp(n, psi_y)
    uy = _interp(n, lambda x, y: -psi_x(x, y))
    assert np.abs(Bx @ ux + By @ uy).max() < 1e-14
    # div (x, 0) = 1: B I_h(x, 0) = M_p 1
    ux = _interp(n, lambda x, y: x)
    assert np.allclose(Bx @ ux, Mp @ np.ones(Mp.shape[0]), rtol=0, atol=1e-15)
    assert Mp.sum() == pytest.approx(1.0, abs=1e-14)


def test_dirichlet_and_pin_by_value(F8):
    n = 8
    F = F8
    bnd = F["bnd"]
    N2 = F["N2"]
    Af = F["Af"].tocoo()
    full_bnd = np.concatenate([bnd, bnd])
    hit = full_bnd[Af.row] | full_bnd[Af.col]
    assert np.all(Af.data[hit & (Af.row != Af.col)] == 0.0)
    assert np.all(Af.data[hit & (Af.row == Af.col)] == 1.0)
    B = F["Bbc"].tocsr()
    assert np.all(B[0].data == 0.0)
    Bc = B.tocoo()
    assert np.all(Bc.data[full_bnd[Bc.col]] == 0.0)
    assert F["Af"].nnz == 4 * (46 * n * n + 16 * n + 1)
    assert N2 == (2 * n + 1) ** 2


def test_solid_blocks():
    xy, tri = inputs.ring_disk(4, (0.5, 0.5), 0.2)
    assert tri.shape[0] == 6 * 16 and xy.shape[0] == 3 * 16 + 3 * 4 + 1
    S = solid.assemble(xy, tri, kappa=10.0)
    area = S["areas"].sum()
    ones = np.ones(xy.shape[0])
    assert np.abs(S["As"] @ ones).max() < 1e-12
    assert ones @ (S["Ms"] @ ones) == pytest.approx(area, rel=1e-14)
    e = xy[:, 0] @ (S["As"] @ xy[:, 0]) + xy[:, 1] @ (S["As"] @ xy[:, 1])
    assert e == pytest.approx(10.0 * 2.0 * area, rel=1e-12)
    # Wathen: eig(D^{-1} M) in [1/2, 2] for P1 triangles
    M = S["Ms"].toarray()
    d = np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(M / np.outer(d, d))
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= 2.0 + 1e-12
    with pytest.raises(ValueError):
        solid.assemble(xy, tri[:, ::-1], kappa=1.0)


def test_ring_mesh_counts_and_orientation():
    for m in (1, 2, 6, 13):
        xy, tri = inputs.ring_disk(m)
        assert tri.shape[0] == 6 * m * m
        assert xy.shape[0] == 3 * m * m + 3 * m + 1
        P = xy[tri]
        d = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1])
        assert (d > 0).all()
        # the triangles tile the inscribed polygon: total area = sum over rings
        assert np.unique(np.sort(tri, axis=1), axis=0).shape[0] == tri.shape[0]


@pytest.mark.parametrize("n", [3, 8])
def test_row_assembly_equals_full_assembly(n):
    """The oracle's row-by-row assembly (used for spot checks of grids too large to
    assemble whole) reproduces the full assembly: same columns, same values."""
    F = fluid.assemble(n, nu=0.7, rho=1.3, dt=0.05)
    N2, Np = F["N2"], F["Np"]
    A, M = fluid.rows_Af(n, range(N2), 0.7, 1.3, 0.05)
    for k, key in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        B = F["Af_blocks"][key].tocsr()
        for r in range(N2):
            cols = B.indices[B.indptr[r]:B.indptr[r + 1]]
            assert list(cols) == list(A[r])
            assert np.allclose(B.data[B.indptr[r]:B.indptr[r + 1]], [A[r][c][k] for c in cols], rtol=0, atol=1e-13)
    Mf = F["Mf"].tocsr()
    for r in range(N2):
        cols = Mf.indices[Mf.indptr[r]:Mf.indptr[r + 1]]
        assert np.allclose(Mf.data[Mf.indptr[r]:Mf.indptr[r + 1]], [M[r][c] for c in cols], rtol=0, atol=1e-16)
    Bx, By = F["Bx_bc"].tocsr(), F["By_bc"].tocsr()
    for k, row in fluid.rows_B(n, range(Np)).items():
        assert list(Bx.indices[Bx.indptr[k]:Bx.indptr[k + 1]]) == list(row)
        for c, v in row.items():
            assert abs(Bx[k, c] - v[0]) < 1e-15 and abs(By[k, c] - v[1]) < 1e-15
    BxT = Bx.T.tocsr()
    BxT.sort_indices()
    for r, row in fluid.rows_BT(n, range(N2)).items():
        assert list(BxT.indices[BxT.indptr[r]:BxT.indptr[r + 1]]) == list(row)
