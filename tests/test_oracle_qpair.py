"""Pins of the oracle's Q2 / P1-disc fluid, Q1 solid and their coupling (Sec. 4, the paper's
element pair) against closed forms, invariants and independent integrations."""
import numpy as np
import pytest

from oracle import fluid as tfluid
from oracle import gmres, qpair
from paper_2301_10041_amd import inputs


def mono(a, b):
    """int over the unit square of x^a y^b."""
    return 1.0 / ((a + 1) * (b + 1))


def q2_values(n, f):
    xy = tfluid.p2_coords(n)
    return f(xy[:, 0], xy[:, 1])


@pytest.fixture(scope="module")
def F4():
    return qpair.assemble_fluid(4, nu=0.7, rho=1.3, dt=0.05)


def test_q2_mass_closed_forms(F4):
    M = F4["Mf"]
    one = np.ones(M.shape[0])
    assert abs(one @ M @ one - 1.0) < 1e-14
    u = q2_values(4, lambda x, y: x * x * y)
    v = q2_values(4, lambda x, y: x * y * y)
    assert abs(v @ M @ u - mono(3, 3)) < 1e-14
    w = q2_values(4, lambda x, y: x * x * y * y)     # biquadratic: reproduced by Q2
    assert abs(w @ M @ w - mono(4, 4)) < 1e-14


def test_q2_eps_form_closed_form(F4):
    """V^T K U = nu int eps(U) : eps(V) for U = (y^2, x y), V = (x^2, x^2 y):
    eps(U) = [[0, 3y/2], [3y/2, x]], eps(V) = [[2x, xy], [xy, x^2]], so the integrand is 3 x y^2 + x^3."""
    K = F4["K"]
    N2 = F4["N2"]
    Ux, Uy = q2_values(4, lambda x, y: y * y), q2_values(4, lambda x, y: x * y)
    Vx, Vy = q2_values(4, lambda x, y: x * x), q2_values(4, lambda x, y: x * x * y)
    val = Vx @ K[(0, 0)] @ Ux + Vx @ K[(0, 1)] @ Uy + Vy @ K[(1, 0)] @ Ux + Vy @ K[(1, 1)] @ Uy
    assert abs(val - 0.7 * (3 * mono(1, 2) + mono(3, 0))) < 1e-13
    # rigid motions have no strain
    one, x, y = np.ones(N2), q2_values(4, lambda x, y: x), q2_values(4, lambda x, y: y)
    for (a, b) in ((one, 0 * one), (0 * one, one), (-y, x)):
        r = np.concatenate([K[(0, 0)] @ a + K[(0, 1)] @ b, K[(1, 0)] @ a + K[(1, 1)] @ b])
        assert np.abs(r).max() < 1e-13


def test_p1disc_divergence_and_mass(F4):
    """p^T B U = int p div U and p^T M_p p = int p^2 for p = 1 + 2x - y, U = (x^2 y, y^2)."""
    p = qpair.pressure_interpolant(4, lambda x, y: 1 + 2 * x - y, 2.0, -1.0)
    Ux, Uy = q2_values(4, lambda x, y: x * x * y), q2_values(4, lambda x, y: y * y)
    # (1 + 2x - y)(2xy + 2y)
    exact = (2 * mono(1, 1) + 2 * mono(0, 1) + 4 * mono(2, 1) + 4 * mono(1, 1) - 2 * mono(1, 2)
             - 2 * mono(0, 2))
    assert abs(p @ (F4["Bx"] @ Ux + F4["By"] @ Uy) - exact) < 1e-13
    # (1 + 2x - y)^2 = 1 + 4x^2 + y^2 + 4x - 2y - 4xy
    exact = 1 + 4 * mono(2, 0) + mono(0, 2) + 4 * mono(1, 0) - 2 * mono(0, 1) - 4 * mono(1, 1)
    assert abs(p @ F4["Mp"] @ p - exact) < 1e-14
    # the cell basis 1, (x - x_c)/h, (y - y_c)/h is orthogonal: M_p is diagonal
    el = qpair.element_matrices(0.25, 1.0)
    assert np.abs(el["Mp"] - np.diag(np.diag(el["Mp"]))).max() < 1e-18
    assert np.allclose(np.diag(el["Mp"]), [0.0625, 0.0625 / 12, 0.0625 / 12], rtol=1e-15)


def test_boundary_rows_and_pin(F4):
    bnd = F4["bnd"]
    Bbc = F4["Bbc"].tocsr()
    assert np.all(Bbc.getrow(0).data == 0.0)
    N2 = F4["N2"]
    cols = np.concatenate([np.flatnonzero(bnd), N2 + np.flatnonzero(bnd)])
    assert np.all(Bbc[:, cols].data == 0.0)
    Af = F4["Af"].tocsr()
    for r in np.flatnonzero(bnd)[:5]:
        row = Af.getrow(r)
        assert set(row.data[row.indices != r]) <= {0.0} and Af[r, r] == 1.0


def test_q1_solid_closed_forms():
    xy, quad = inputs.quad_bar(5, 3, 0.3, 0.7, 0.45, 0.55)
    S = qpair.assemble_solid(xy, quad, kappa=2.0)
    one = np.ones(xy.shape[0])
    area = 0.4 * 0.1
    assert abs(one @ S["Ms"] @ one - area) < 1e-15
    assert np.abs(S["Ks"] @ one).max() < 1e-13
    sx, sy = xy[:, 0], xy[:, 1]
    assert abs(sx @ S["Ks"] @ sx - area) < 1e-14
    f = sx * sy    # bilinear: reproduced by Q1 on rectangles; int |grad f|^2 = int (y^2 + x^2)
    a, b, c, d = 0.3, 0.7, 0.45, 0.55
    exact = (b ** 3 - a ** 3) / 3 * (d - c) + (b - a) * (d ** 3 - c ** 3) / 3
    assert abs(f @ S["Ks"] @ f - exact) < 1e-14
    assert np.allclose(S["As"].data, 2.0 * S["Ks"].data)
    # a parallelogram mesh (sheared bar): the 2 x 2 rule stays exact
    xs = xy.copy()
    xs[:, 0] += 0.3 * (xy[:, 1] - 0.45)
    S2 = qpair.assemble_solid(xs, quad)
    assert abs(one @ S2["Ms"] @ one - area) < 1e-15
    assert abs(xs[:, 0] @ S2["Ks"] @ xs[:, 0] - area) < 1e-14


def _s_space_moments(Xn, xy_ref, quad, g):
    """int_B N_l(s) g(X^n(s)) ds per solid node, by 5 x 5 Gauss points in (xi, eta) on every
    quadrilateral: exact when g is a polynomial of degree <= 2 in each of x, y (X^n bilinear)."""
    t, w = qpair.gauss01(5)
    out = np.zeros(xy_ref.shape[0])
    for qv in quad:
        S, P = xy_ref[qv], Xn[qv]
        for p in range(5):
            for q in range(5):
                N, _, _ = qpair.bilinear(t[p], t[q])
                Js = qpair.jacobian(S, np.array([t[p]]), np.array([t[q]]))[0]
                x, y = N @ P[:, 0], N @ P[:, 1]
                out[qv] += w[p] * w[q] * Js * N * g(x, y)
    return out


def _case(pos):
    n = 8
    xy, quad = inputs.quad_bar(5, 2, 0.3, 0.7, 0.45, 0.55)
    if pos == "rotated":
        X = inputs.rotation(xy, (0.5, 0.5), 0.3)
    else:
        X = inputs.bent(xy, 0.05, 0.4, 0.3)
        X[:, 0] += 0.02 * np.sin(7.0 * xy[:, 1])      # and a shear that varies along the bar
    return n, xy, quad, X


@pytest.mark.parametrize("pos", ["rotated", "bent"])
def test_coupling_moments(pos):
    """Q2 reproduces 1, x, y and x^2 y^2, so C_f g = int N_l g(X^n) for these g.  Affine X^n
    (rotation): the composite rule is exact.  Non-affine X^n (bent and sheared): within the
    rule's error, which shrinks with the fan triangles."""
    n, xy, quad, X = _case(pos)
    Cf, pieces = qpair.assemble_coupling(X, xy, quad, n)
    S = qpair.assemble_solid(xy, quad)
    tol = 1e-14 if pos == "rotated" else 2e-8
    for g in (lambda x, y: 1.0 + 0 * x, lambda x, y: x, lambda x, y: y, lambda x, y: x * x * y * y):
        ref = _s_space_moments(X, xy, quad, g)
        got = Cf @ q2_values(n, g)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < tol, (pos, err)
    # C_s rows are the moments of g = 1 and of the coordinates
    assert np.abs(Cf @ np.ones(Cf.shape[1]) - S["Ms"] @ np.ones(xy.shape[0])).max() < (1e-15 if pos == "rotated" else 1e-9)
    # the bounding-box candidates find every piece of the all-pairs search
    _, brute = qpair.assemble_coupling(X, xy, quad, n, brute_force=True)
    assert brute == pieces


def test_coupling_rule_converges_on_a_nonaffine_element():
    """One quadrilateral inside one cell, strongly non-affine: the s-space integral of
    N_a phi_b(X(s)) J_s is a polynomial (exact by Gauss points); the composite rule's error
    falls by more than 2^4 with every split of the fan triangles (a rule exact to degree 6 on
    smooth integrands); this element's corners move by a third of its size, so the default
    rule is within 1e-3 here (the bent bar's moments above are within 2e-8)."""
    n = 4
    xy = np.array([[0.3, 0.3], [0.45, 0.3], [0.45, 0.42], [0.3, 0.42]])
    quad = np.array([[0, 1, 2, 3]])
    X = np.array([[0.28, 0.29], [0.47, 0.3], [0.43, 0.46], [0.3, 0.4]])
    t, w = qpair.gauss01(6)
    ref = np.zeros((4, 9))
    for p in range(6):
        for q in range(6):
            N, _, _ = qpair.bilinear(t[p], t[q])
            Js = qpair.jacobian(xy, np.array([t[p]]), np.array([t[q]]))[0]
            x, y = N @ X[:, 0], N @ X[:, 1]
            Vx, _ = qpair.lagrange2(np.array([x * n - 1]))
            Vy, _ = qpair.lagrange2(np.array([y * n - 1]))
            phi = np.array([Vx[a, 0] * Vy[b, 0] for b in range(3) for a in range(3)])
            ref += w[p] * w[q] * Js * np.outer(N, phi)
    pieces = qpair.intersections(X, quad, n)
    assert [(e, c) for e, c, _ in pieces] == [(0, 1 * n + 1)]
    q = pieces[0][2]
    errs = [np.abs(qpair.piece_matrix(X, xy, q, 1, 1, n, split=s) - ref).max() / np.abs(ref).max()
            for s in range(3)]
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 16 and errs[2] < errs[1] / 16, errs


def test_inverse_bilinear_map():
    P = np.array([[0.1, 0.2], [0.5, 0.25], [0.55, 0.6], [0.05, 0.5]])
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    N, _, _ = qpair.bilinear(xi, eta)
    a, b = qpair.inverse_bilinear(P, P[:, 0] @ N, P[:, 1] @ N)
    assert np.abs(a - xi).max() < 1e-14 and np.abs(b - eta).max() < 1e-14


def test_invalid_positions_raise():
    xy, quad = inputs.quad_bar(3, 1, 0.3, 0.7, 0.45, 0.55)
    X = xy.copy()
    X[1] = X[2] - [0.0, 0.2]       # a reflex corner
    with pytest.raises(qpair.MeshError):
        qpair.assemble_coupling(X, xy, quad, 8)
    X = xy.copy()
    X[0, 0] = -0.1
    with pytest.raises(qpair.MeshError):
        qpair.assemble_coupling(X, xy, quad, 8)


def test_qsystem_direct_and_gmres():
    """The assembled system is nonsingular and GMRES with the exact blocks (Sec. 5) reaches
    the direct solution."""
    wl = inputs.QWorkload("q8", 8, 5, 2, nu=0.2, dt=0.002, seed=1)
    S = qpair.QSystem.from_workload(wl)
    xy, quad = wl.solid_mesh()
    S.set_position(inputs.rotation(xy, wl.center, 0.2))
    b = S.random_rhs(1)
    x = S.solve_direct(b)
    A = S.matrix()
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    for kind in ("diag", "tri"):
        xg, info = gmres.gmres(lambda v: A @ v, b, lambda r: S.apply_precond(r, kind), rtol=1e-10, restart=30)
        assert info["converged"] and np.linalg.norm(xg - x) <= 1e-8 * np.linalg.norm(x), kind
        assert info["its"] <= 30, (kind, info["its"])
