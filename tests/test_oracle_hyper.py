"""Pins of the oracle's nonlinear solid (the exponential law of Sec. 6.2) and of its Newton step
(Sec. 4, last paragraph; Sec. 6 stopping rule), CPU only.

Checks that do not re-type the formulas: P = dW/dF and dP/dF by central finite differences of W
and P; the assembled residual R(X) is the gradient of the elastic energy E(X) = sum |E| W(F_E)
(finite differences of E) and the tangent K(X) is its Jacobian (finite differences of R), K
symmetric; frame indifference (W(QF) = W(F), R(QX + c) = Q R(X)); eta = 0 gives the linear law
with kappa = gamma (R = gamma K_s X exactly) and small eta tends to it; Newton on the coupled
step: with eta = 0 one iteration gives the linear step's direct solve, with the paper's eta the
residual falls quadratically."""
import numpy as np
import pytest

from oracle import hyper, newton, solid, system
from paper_2301_10041_amd import inputs

RNG = np.random.default_rng(123)


def _rand_F():
    return np.eye(2) + 0.2 * RNG.standard_normal((2, 2))


@pytest.mark.parametrize("eta", [hyper.ETA, 1.0, 0.0])
def test_stress_is_energy_gradient(eta):
    for _ in range(5):
        F = _rand_F()
        Pn = np.zeros((2, 2))
        h = 1e-6
        for a in range(2):
            for b in range(2):
                E = np.zeros((2, 2))
                E[a, b] = h
                Pn[a, b] = (hyper.W(F + E, eta=eta) - hyper.W(F - E, eta=eta)) / (2 * h)
        P = hyper.P(F, eta=eta)
        assert np.abs(Pn - P).max() <= 1e-6 * max(1.0, np.abs(P).max())


@pytest.mark.parametrize("eta", [hyper.ETA, 0.0])
def test_tangent_tensor_is_stress_derivative(eta):
    for _ in range(5):
        F = _rand_F()
        D = hyper.dPdF(F, eta=eta)
        h = 1e-6
        for c in range(2):
            for d in range(2):
                E = np.zeros((2, 2))
                E[c, d] = h
                col = (hyper.P(F + E, eta=eta) - hyper.P(F - E, eta=eta)) / (2 * h)
                assert np.abs(col - D[:, :, c, d]).max() <= 1e-6 * max(1.0, np.abs(D).max())


def _bar_state(nx=6, ny=3, amp=0.03, noise=0.004):
    xy, tri = inputs.bar_mesh(nx, ny)
    X = inputs.bent(xy, amp) + noise * RNG.standard_normal(xy.shape)
    return xy, tri.astype(np.int64), X


def test_residual_is_energy_gradient_and_tangent_its_jacobian():
    xy, tri, X = _bar_state()
    ns = xy.shape[0]
    R = hyper.residual(xy, tri, X)
    K = hyper.tangent(xy, tri, X).toarray()
    h = 1e-6
    for k in RNG.choice(2 * ns, 12, replace=False):
        comp, node = divmod(int(k), ns)
        Xp, Xm = X.copy(), X.copy()
        Xp[node, comp] += h
        Xm[node, comp] -= h
        g = (hyper.energy(xy, tri, Xp) - hyper.energy(xy, tri, Xm)) / (2 * h)
        assert abs(g - R[k]) <= 1e-6 * max(1.0, np.abs(R).max())
        col = (hyper.residual(xy, tri, Xp) - hyper.residual(xy, tri, Xm)) / (2 * h)
        assert np.abs(col - K[:, k]).max() <= 1e-5 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()


def test_frame_indifference():
    xy, tri, X = _bar_state()
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    c = np.array([0.1, -0.05])
    F = _rand_F()
    assert abs(hyper.W(Q @ F) - hyper.W(F)) <= 1e-12 * abs(hyper.W(F))
    R = hyper.residual(xy, tri, X)
    R2 = hyper.residual(xy, tri, X @ Q.T + c)
    ns = xy.shape[0]
    rot = (np.stack([R[:ns], R[ns:]], axis=1)) @ Q.T
    assert np.abs(np.concatenate([rot[:, 0], rot[:, 1]]) - R2).max() <= 1e-12 * np.abs(R).max()
    # the reference position is stress free up to the isotropic gamma I: R(s) = gamma K_s s
    Ks = solid.assemble(xy, tri, 1.0)["Ks"]
    R0 = hyper.residual(xy, tri, xy)
    assert np.abs(R0 - hyper.GAMMA * np.concatenate([Ks @ xy[:, 0], Ks @ xy[:, 1]])).max() <= 1e-12


def test_eta_zero_is_the_linear_law():
    xy, tri, X = _bar_state()
    gamma = 2.5
    Ks = solid.assemble(xy, tri, 1.0)["Ks"]
    R = hyper.residual(xy, tri, X, gamma=gamma, eta=0.0)
    lin = gamma * np.concatenate([Ks @ X[:, 0], Ks @ X[:, 1]])
    assert np.abs(R - lin).max() <= 1e-12 * np.abs(lin).max()
    K = hyper.tangent(xy, tri, X, gamma=gamma, eta=0.0).toarray()
    ns = xy.shape[0]
    Kd = np.zeros((2 * ns, 2 * ns))
    Kd[:ns, :ns] = Kd[ns:, ns:] = gamma * Ks.toarray()
    assert np.abs(K - Kd).max() <= 1e-12 * np.abs(Kd).max()
    # and the law tends to it as eta -> 0
    R1 = hyper.residual(xy, tri, X, gamma=gamma, eta=1e-7)
    assert np.abs(R1 - lin).max() <= 1e-5 * np.abs(lin).max()


def _bar_system(n=16, nx=8, ny=2, kappa=None):
    wl = inputs.Workload("bar", n, [inputs.Bar(m=0, center=(0.2, 0.5), nx=nx, ny=ny)], nu=0.2, rho=1.0,
                         kappa=hyper.GAMMA if kappa is None else kappa, dt=0.002, seed=9)
    return wl, system.FSISystem.from_workload(wl)


def test_newton_eta_zero_is_one_linear_solve():
    wl, S = _bar_system()
    X = inputs.bent(S.xy_ref, 0.03)
    u = inputs.uniform(2 * S.lay.N2, wl.seed)
    x, info = newton.newton_step(S, u, X, np.zeros(S.lay.N), gamma=hyper.GAMMA, eta=0.0, rtol=1e-12)
    assert info["converged"] and info["nit"] == 1
    S.set_position(X)
    xs = S.solve_direct(S.rhs(u, X))   # the linear law with kappa = gamma
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()


def test_newton_converges_quadratically():
    wl, S = _bar_system()
    X = inputs.bent(S.xy_ref, 0.04)
    lay = S.lay
    u = np.zeros(2 * lay.N2)
    f = np.zeros(2 * lay.Ns)
    f[lay.Ns + 12] = -0.05          # a downward load at one node of the right part
    x0 = np.zeros(lay.N)
    sl = lay.slices()
    x0[sl["Xx"]], x0[sl["Xy"]] = X[:, 0], X[:, 1]
    x, info = newton.newton_step(S, u, X, x0, f_X=f, rtol=1e-13, maxit=20)
    r = info["res"]
    assert info["converged"] and 2 <= info["nit"] <= 8
    # quadratic: once in the basin, each residual is below C times the square of the previous
    ratios = [r[k + 1] / r[k] ** 2 for k in range(len(r) - 1) if r[k] < 1e-2 * r[0] and r[k + 1] > 1e-12 * r[0]]
    assert ratios and max(ratios) * r[0] < 50.0
    # the result solves the nonlinear system: R(X) - C_s lam = f on the X rows
    b = newton.rhs(S, u, X, f)
    assert np.linalg.norm(newton.residual(S, x, b)) <= 1e-12 * np.linalg.norm(b)
