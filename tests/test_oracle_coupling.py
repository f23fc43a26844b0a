"""Pins of the oracle's coupling matrix C_f(X^n) (Sec. 4, the assembly of the coupling
term by clipping the mapped solid triangles with the Cartesian fluid mesh).

The checks use facts fixed by the mathematics: area coverage of the pieces, the P2
partition of unity, exactness on interpolated quadratics (integrated independently on the
solid mesh), the matching-mesh special case with closed-form P1 x P2 moments, and the
paper's own all-pairs search against the bounding-box search.  CPU only.
"""
import numpy as np
import pytest

from oracle import coupling, fluid, poly, solid
from paper_2301_10041_amd import inputs


def _disk(n=16, m=4, c=(0.5, 0.5), r=0.2, axes=None):
    xy, tri = inputs.ring_disk(m, c, r, axes)
    return xy, tri


def test_brute_force_equals_bucketed_bitwise():
    for (n, m, c, r) in [(8, 2, (0.5, 0.5), 0.2), (8, 3, (0.43, 0.61), 0.17), (16, 2, (0.5, 0.5), 0.25)]:
        xy, tri = _disk(n, m, c, r)
        a = coupling.intersections(xy, tri, n, brute_force=False)
        b = coupling.intersections(xy, tri, n, brute_force=True)
        assert [(e, t) for e, t, _ in a] == [(e, t) for e, t, _ in b]
        for (_, _, p), (_, _, q) in zip(a, b):
            assert p == q


def test_pieces_cover_each_mapped_triangle():
    n = 16
    xy, tri = _disk(n, 5, (0.47, 0.52), 0.21)
    X = inputs.rotation(xy, (0.5, 0.5), 0.3)
    pieces = coupling.intersections(X, tri, n)
    tot = np.zeros(tri.shape[0])
    for e, T, q in pieces:
        tot[e] += coupling.fan_area(q)
    for e, t in enumerate(tri):
        assert tot[e] == pytest.approx(coupling.signed_area(X[t]), rel=1e-12)


def test_piece_inside_its_fluid_triangle():
    n = 8
    xy, tri = _disk(n, 3, (0.51, 0.47), 0.3)
    _, _, vx = fluid.triangle_nodes(n)
    for e, T, q in coupling.intersections(xy, tri, n):
        V = vx[T]
        for (x, y) in q:
            l = np.linalg.solve(np.array([[V[0, 0], V[1, 0], V[2, 0]], [V[0, 1], V[1, 1], V[2, 1]], [1, 1, 1]]),
                                np.array([x, y, 1.0]))
            assert l.min() > -1e-12


def _solid_integral(xy, tri, Xn, q):
    """int_B chi_l q(X^n(s)) ds for a quadratic q(x, y) = sum c_ab x^a y^b, integrated
    exactly on the solid mesh (X^n affine on each triangle)."""
    out = np.zeros(xy.shape[0])
    L = poly.p1_basis()
    for t in tri:
        _, area = poly.bary_gradients(xy[t])
        Xx = poly.add(poly.add(poly.scale(L[0], Xn[t[0], 0]), poly.scale(L[1], Xn[t[1], 0])), poly.scale(L[2], Xn[t[2], 0]))
        Xy = poly.add(poly.add(poly.scale(L[0], Xn[t[0], 1]), poly.scale(L[1], Xn[t[1], 1])), poly.scale(L[2], Xn[t[2], 1]))
        Q = {}
        for (a, b), c in q.items():
            term = {(0, 0, 0): c}
            for _ in range(a):
                term = poly.mul(term, Xx)
            for _ in range(b):
                term = poly.mul(term, Xy)
            Q = poly.add(Q, term)
        for k in range(3):
            out[t[k]] += poly.integrate(poly.mul(L[k], Q), abs(area))
    return out


def test_partition_of_unity_and_quadratic_exactness():
    n = 16
    xy, tri = _disk(n, 4, (0.5, 0.5), 0.2)
    X = inputs.rotation(xy, (0.5, 0.5), 0.37)
    X[:, 0] = 0.5 + 1.1 * (X[:, 0] - 0.5)            # a non-rigid, still affine-per-element map
    Cf, _ = coupling.assemble(X, xy, tri, n)
    Ms = solid.assemble(xy, tri)["Ms"]
    P = fluid.p2_coords(n)
    ones = np.ones(P.shape[0])
    # C_f 1 = C_s 1 row by row (the P2 functions sum to one)
    assert np.allclose(Cf @ ones, Ms @ np.ones(xy.shape[0]), rtol=1e-12, atol=1e-16)
    # C_f I_h(x) = C_s X_x, C_f I_h(y) = C_s X_y
    assert np.allclose(Cf @ P[:, 0], Ms @ X[:, 0], rtol=1e-12, atol=1e-16)
    assert np.allclose(Cf @ P[:, 1], Ms @ X[:, 1], rtol=1e-12, atol=1e-16)
    # C_f I_h(q) = int_B chi_l q(X^n) for quadratics q
    for q in ({(2, 0): 1.0}, {(1, 1): 1.0}, {(0, 2): 1.0, (1, 0): -0.3}):
        vals = sum(c * P[:, 0] ** a * P[:, 1] ** b for (a, b), c in q.items())
        ref = _solid_integral(xy, tri, X, q)
        assert np.allclose(Cf @ vals, ref, rtol=1e-11, atol=1e-15)


def test_matching_mesh_gives_mixed_mass_matrix():
    """Solid = fluid triangles, X = identity: exactly the diagonal pairs survive (the
    edge-touching neighbours have zero-area pieces) and C_f is the P1 x P2 mass matrix
    with closed-form entries |T|/30 (same vertex), -|T|/60 (other vertex), 2|T|/15
    (edge through the vertex) and |T|/15 (opposite edge)."""
    n = 8
    h = 1.0 / n
    p2, p1, vx = fluid.triangle_nodes(n)
    cells = [(3, 3), (4, 3), (3, 4), (4, 4)]
    Ts = [2 * (j * n + i) + t for (i, j) in cells for t in (0, 1)]
    # solid nodes = P1 nodes of these triangles (renumbered), same coordinates
    verts = sorted(set(int(v) for T in Ts for v in p1[T]))
    ren = {v: k for k, v in enumerate(verts)}
    xy = fluid.p1_coords(n)[verts]
    tri = np.array([[ren[int(v)] for v in p1[T]] for T in Ts], dtype=np.int32)
    Cf, pieces = coupling.assemble(xy, xy, tri, n)
    assert pieces == [(e, T) for e, T in enumerate(Ts)]
    A = h * h / 2
    ref = np.zeros(Cf.shape)
    for e, T in enumerate(Ts):
        for l in range(3):
            for jj in range(6):
                if jj < 3:
                    v = A / 30 if jj == l else -A / 60
                else:
                    a, b = [(0, 1), (1, 2), (2, 0)][jj - 3]
                    v = 2 * A / 15 if l in (a, b) else A / 15
                ref[tri[e, l], p2[T, jj]] += v
    assert np.allclose(Cf.toarray(), ref, rtol=0, atol=1e-17)


def test_translation_by_whole_cells_shifts_columns():
    n = 16
    h = 1.0 / n
    xy, tri = _disk(n, 3, (0.4, 0.45), 0.15)
    Cf0, pc0 = coupling.assemble(xy, xy, tri, n)
    X1 = xy.copy()
    X1[:, 0] += 2 * h
    X1[:, 1] += h
    Cf1, pc1 = coupling.assemble(X1, xy, tri, n)
    shift_T = 2 * (1 * n + 2)
    assert [(e, T + shift_T) for e, T in pc0] == pc1
    shift_col = 2 * (2 * n + 1) + 4           # (I, J) -> (I + 4, J + 2)
    for r in range(Cf0.shape[0]):
        c0 = Cf0.indices[Cf0.indptr[r]:Cf0.indptr[r + 1]]
        c1 = Cf1.indices[Cf1.indptr[r]:Cf1.indptr[r + 1]]
        assert np.array_equal(c0 + shift_col, c1)
        assert np.allclose(Cf0.data[Cf0.indptr[r]:Cf0.indptr[r + 1]], Cf1.data[Cf1.indptr[r]:Cf1.indptr[r + 1]],
                           rtol=1e-11, atol=1e-17)


def test_invalid_positions_rejected():
    n = 8
    xy, tri = _disk(n, 2, (0.5, 0.5), 0.2)
    bad = xy.copy()
    bad[:, 0] = 1.0 - bad[:, 0]                          # mirror: every triangle inverted
    with pytest.raises(coupling.MeshError):
        coupling.assemble(bad, xy, tri, n)
    out = xy.copy()
    out[:, 0] += 0.4                                     # pushed through x = 1
    with pytest.raises(coupling.MeshError):
        coupling.assemble(out, xy, tri, n)


def test_dirichlet_columns_zeroed_but_kept():
    n = 8
    xy, tri = inputs.ring_disk(2, (0.12, 0.5), 0.1)      # touches the cells along x = 0
    Cf, _ = coupling.assemble(xy, xy, tri, n)
    bnd = fluid.boundary_p2(n)
    hit = bnd[Cf.indices]
    assert hit.any()
    assert np.all(Cf.data[hit] == 0.0)
