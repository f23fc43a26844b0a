"""The nonlinear solid through the C-ABI (the exponential law of the paper's nonlinear test, Newton's
method of Sec. 4) against the oracle: the solid residual R(X) and tangent K(X) entry by entry,
the operator and the block preconditioners with the tangent in place of A_s, and whole Newton
steps on the bar workload (FP64 and mixed precision, both preconditioners) within 1e-8 per block,
with the oracle's Newton iteration counts; the linear law takes one Newton iteration, the linear
step up to rounding."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import hyper, newton, system
from paper_2301_10041_amd import fsi, inputs

from gpu_helpers import assert_block_parity, rel, soa, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    fsi.lib()


def bar_workload(n=32, nx=13, ny=3, seed=9):
    return inputs.Workload(f"bar{n}", n, [inputs.Bar(m=0, center=(0.2, 0.5), nx=nx, ny=ny)], nu=0.2, rho=1.0,
                           kappa=hyper.GAMMA, dt=0.002, seed=seed)


def _X(xy, amp=0.04, noise=0.0, seed=3):
    X = inputs.bent(xy, amp)
    if noise:
        X = X + noise * np.random.default_rng(seed).standard_normal(xy.shape)
    return X


@pytest.mark.parametrize("law", ["exp", "linear"])
def test_solid_residual_and_tangent(law):
    print(f"[solid law {law}]", flush=True)
    torch = torch_dev()
    wl = bar_workload()
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    gamma, eta = (hyper.GAMMA, hyper.ETA) if law == "exp" else (wl.kappa, 0.0)
    if law == "exp":
        ctx.set_law(fsi.LAW_EXP, hyper.GAMMA, hyper.ETA)
    X = _X(xy, noise=0.003)
    Xd = to_dev(soa(X))
    R = torch.zeros(2 * xy.shape[0], dtype=torch.float64, device="cuda")
    ctx.solid_residual(Xd, R)
    R_ref = hyper.residual(xy, tri.astype(np.int64), X, gamma, eta)
    assert np.abs(to_host(R) - R_ref).max() <= 1e-12 * np.abs(R_ref).max()
    ctx.solid_tangent(Xd)
    rp, col, val = ctx.export_csr("KT")
    K = hyper.tangent(xy, tri.astype(np.int64), X, gamma, eta).tocsr()
    ns = xy.shape[0]
    scale = np.abs(K.data).max()
    for l in range(ns):
        for k in range(rp[l], rp[l + 1]):
            j = col[k]
            ref = (K[l, j], K[l, ns + j], K[ns + l, j], K[ns + l, ns + j])
            assert np.abs(val[k] - np.array(ref)).max() <= 1e-12 * scale, (l, j)
    # every entry of K lies on the pattern
    assert sum(rp[l + 1] - rp[l] for l in range(ns)) * 4 >= K.nnz
    ctx.close()


@pytest.fixture(scope="module")
def bar32():
    wl = bar_workload()
    S = system.FSISystem.from_workload(wl)
    X = _X(S.xy_ref)
    S.set_position(X)
    ctx = fsi.Context.from_workload(wl)
    ctx.set_law(fsi.LAW_EXP, hyper.GAMMA, hyper.ETA)
    ctx.assemble_coupling(to_dev(soa(X)))
    yield wl, S, X, ctx
    ctx.close()


def test_operator_and_preconditioner_with_tangent(bar32):
    print("[tangent operator/precond]", flush=True)
    torch = torch_dev()
    wl, S, X, ctx = bar32
    lay = S.lay
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, lay.N)
    sl = lay.slices()
    x[sl["Xx"]], x[sl["Xy"]] = X[:, 0], X[:, 1]
    J = newton.jacobian(S, x)
    ctx.solid_tangent(to_dev(soa(X)))
    y = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    ctx.apply_operator(to_dev(x), y, fsi.FP64)
    yr = J @ x
    assert np.abs(to_host(y) - yr).max() <= 1e-12 * np.abs(yr).max()
    ctx.apply_operator(to_dev(x), y, fsi.FP32)
    assert rel(to_host(y), yr) <= 2e-6
    # exact-block preconditioners of the Jacobian (A22 with the tangent)
    nf = lay.nf
    A11 = J[:nf, :nf].tocsc()
    A22 = J[nf:, nf:].tocsc()
    A21 = J[nf:, :nf]
    lu11, lu22 = spla.splu(A11), spla.splu(A22)
    r = S.random_rhs(0, rng.uniform(-1, 1, lay.N))
    ctx.set_inner(1e-13, 2000)
    for pc, name in ((fsi.PC_DIAG, "diag"), (fsi.PC_TRI, "tri")):
        z = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
        ctx.apply_precond(to_dev(r), z, pc, fsi.FP64)
        z1 = lu11.solve(r[:nf])
        z2 = lu22.solve(r[nf:] - (A21 @ z1 if name == "tri" else 0.0))
        zr = np.concatenate([z1, z2])
        assert rel(to_host(z)[nf:], z2) <= 1e-10, name
        assert rel(to_host(z), zr) <= 1e-9, name
    ctx.set_inner(-1.0, 1000)
    ctx.solid_tangent(None)


def _x0(S, u, X):
    lay = S.lay
    sl = lay.slices()
    x0 = np.zeros(lay.N)
    x0[sl["ux"]], x0[sl["uy"]] = u[:lay.N2], u[lay.N2:]
    x0[sl["Xx"]], x0[sl["Xy"]] = X[:, 0], X[:, 1]
    return x0


@pytest.mark.parametrize("pc", [fsi.PC_TRI, fsi.PC_DIAG])
@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_newton_step_against_oracle(pc, prec):
    print(f"[newton pc={pc} prec={prec}]", flush=True)
    torch = torch_dev()
    wl = bar_workload()
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    X = _X(S.xy_ref)
    u = inputs.uniform(2 * lay.N2, wl.seed) * 0.1
    bnd = np.concatenate([S.F["bnd"], S.F["bnd"]])
    u[bnd] = 0.0
    f = np.zeros(2 * lay.Ns)
    f[lay.Ns + 20] = -0.02           # a downward load at one node
    x0 = _x0(S, u, X)
    x_ref, info_ref = newton.newton_step(S, u, X, x0, f_X=f, rtol=1e-12)
    _, info6 = newton.newton_step(S, u, X, x0, f_X=f, rtol=1e-6)
    ctx = fsi.Context.from_workload(wl)
    ctx.set_law(fsi.LAW_EXP, hyper.GAMMA, hyper.ETA)
    state = to_dev(x0)
    st = ctx.newton_step(to_dev(u), to_dev(soa(X)), state, fsi.Opts(pc=pc, prec=prec, rtol=1e-8), rtol=1e-6,
                         f_X=to_dev(f))
    print(f"  paper tolerances: nit {st['nit']} (oracle {info6['nit']}) its {st['its_total']} "
          f"res {st['res'] / st['res0']:.1e}", flush=True)
    assert st["converged"] and st["nit"] == info6["nit"]
    state = to_dev(x0)
    st = ctx.newton_step(to_dev(u), to_dev(soa(X)), state, fsi.Opts(pc=pc, prec=prec, rtol=1e-11), rtol=1e-10,
                         f_X=to_dev(f))
    assert st["converged"]
    assert_block_parity(S, to_host(state), x_ref, 1e-8, f"newton pc={pc} prec={prec}")
    ctx.close()


def test_newton_with_the_linear_law_is_the_linear_step():
    print("[newton linear law]", flush=True)
    torch = torch_dev()
    wl = bar_workload()
    xy, _ = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    N, N2 = ctx.sizes["N"], ctx.sizes["N2"]
    u = to_dev(inputs.uniform(2 * N2, wl.seed))
    X = to_dev(soa(_X(xy)))
    a = torch.zeros(N, dtype=torch.float64, device="cuda")
    st = ctx.newton_step(u, X, a, fsi.Opts(pc=fsi.PC_TRI), rtol=1e-6)
    assert st["converged"] and st["nit"] == 1
    b = torch.zeros_like(a)
    st2 = ctx.step(u, X, b, fsi.Opts(pc=fsi.PC_TRI))
    # the same solve up to rounding: the tangent of the linear law is kappa K_s summed in another
    # order, and its A22 part runs the per-system form
    assert st["its_total"] == st2["its"]
    assert rel(to_host(a), to_host(b)) <= 1e-10
    ctx.close()


def test_nonlinear_time_loop_against_oracle():
    """Three steps of the released bar: each step's solution (u, X, and the multiplier) feeds the
    next step as its initial guess and its u^n, X^n; every state within 1e-8 of the oracle's."""
    print("[newton time loop]", flush=True)
    wl = bar_workload()
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    sl = lay.slices()
    X = _X(S.xy_ref, amp=0.05)
    u = np.zeros(2 * lay.N2)
    x_ref = _x0(S, u, X)
    ctx = fsi.Context.from_workload(wl)
    ctx.set_law(fsi.LAW_EXP, hyper.GAMMA, hyper.ETA)
    state = to_dev(x_ref)
    for k in range(3):
        x_ref, info = newton.newton_step(S, u, X, x_ref, rtol=1e-11)
        st = ctx.newton_step(to_dev(u), to_dev(soa(X)), state, fsi.Opts(pc=fsi.PC_TRI, rtol=1e-11), rtol=1e-10)
        assert st["converged"]
        assert_block_parity(S, to_host(state), x_ref, 1e-8, f"loop step {k} (nit {st['nit']}/{info['nit']})")
        u = x_ref[:2 * lay.N2].copy()
        X = np.stack([x_ref[sl["Xx"]], x_ref[sl["Xy"]]], axis=1)
        state = to_dev(x_ref)   # both sides continue from the same state
    ctx.close()
