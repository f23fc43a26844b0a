"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bit-exact: sparsity patterns of every block, the intersection list (E, T) and the C_f
pattern.  FP64 values: relative differences at the rounding level of the assembly
(1e-12).  Solutions: relative error 1e-8 against the oracle's direct solve in every block
(u, mean-free p, X, lam), both in the 2-norm and element by element against the block's
largest entry, for FP64, mixed precision and FP32 refinement (the parity solves run to
rtol 1e-10: at rtol 1e-8 the error may exceed the residual by the condition number), with
GMRES iteration counts at rtol 1e-8 within the oracle's exact-block counts plus max(2, 10%).
"""
import math

import numpy as np
import pytest

from oracle import fluid, gmres, system
from paper_2301_10041_amd import fsi, inputs

from gpu_helpers import (assert_block_parity, csr_from_export, make_pair, rel, small_workloads, soa, to_dev,
                         to_host, torch_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    fsi.lib()


def _same_pattern(rp, col, A):
    A = A.tocsr()
    assert np.array_equal(rp, A.indptr.astype(np.int32))
    assert np.array_equal(col, A.indices.astype(np.int32))


@pytest.mark.parametrize("n", [2, 5, 8, 32])
def test_fluid_blocks(n):
    print(f"[fluid blocks n={n}]", flush=True)
    wl = inputs.small_workload(n, 1, (0.5, 0.5), 0.2)
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context(n, xy, tri, nu=1.3, rho=0.9, dt=0.02)
    F = fluid.assemble(n, nu=1.3, rho=0.9, dt=0.02)
    rp, col, val = ctx.export_csr("AF")
    blk = F["Af_blocks"]
    _same_pattern(rp, col, blk[(0, 0)])
    scale = max(abs(blk[(0, 0)].data).max(), 1.0)
    for k, key in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        B = blk[key].tocsr()
        _same_pattern(rp, col, B)
        assert np.abs(val[:, k] - B.data).max() <= 1e-12 * scale
    rp, col, val = ctx.export_csr("MF")
    _same_pattern(rp, col, F["Mf"])
    assert np.abs(val[:, 0] - F["Mf"].data).max() <= 1e-14 * abs(F["Mf"].data).max()
    rp, col, val = ctx.export_csr("B")
    for k, B in enumerate([F["Bx_bc"], F["By_bc"]]):
        _same_pattern(rp, col, B)
        assert np.abs(val[:, k] - B.tocsr().data).max() <= 1e-13 * abs(B.data).max()
    rp, col, val = ctx.export_csr("BT")
    for k, B in enumerate([F["Bx_bc"], F["By_bc"]]):
        Bt = B.T.tocsr()
        Bt.sort_indices()
        _same_pattern(rp, col, Bt)
        assert np.abs(val[:, k] - Bt.data).max() <= 1e-13 * abs(B.data).max()
    rp, col, val = ctx.export_csr("MP")
    _same_pattern(rp, col, F["Mp"])
    assert np.abs(val[:, 0] - F["Mp"].data).max() <= 1e-14 * abs(F["Mp"].data).max()
    ctx.close()


def test_solid_blocks():
    print("[solid blocks]", flush=True)
    wl = inputs.small_workload(16, 7, (0.45, 0.55), semi_axes=(0.25, 0.15), kappa=3.5)
    S = system.FSISystem.from_workload(wl)
    ctx = fsi.Context.from_workload(wl)
    for name, A in (("AS", S.S["As"]), ("CS", S.S["Ms"])):
        rp, col, val = ctx.export_csr(name)
        _same_pattern(rp, col, A)
        assert np.abs(val[:, 0] - A.data).max() <= 1e-13 * abs(A.data).max()
    ctx.close()


def _positions(name, S, angle):
    X = S.xy_ref
    if angle is None:
        return X
    Xr = inputs.rotation(X, (0.5, 0.5), angle)
    Xr[:, 0] = 0.5 + 1.05 * (Xr[:, 0] - 0.5)
    return Xr


@pytest.mark.parametrize("name", list(small_workloads()))
def test_coupling_bitexact(name):
    print(f"[coupling {name}]", flush=True)
    wl, angle = small_workloads()[name]
    S = system.FSISystem.from_workload(wl)
    X = _positions(name, S, angle)
    S.set_position(X)
    ctx = fsi.Context.from_workload(wl)
    info = ctx.assemble_coupling(to_dev(soa(X)))
    E, T = ctx.export_pairs()
    ref = np.array(S.pieces, dtype=np.int64).reshape(-1, 2)
    assert info["n_pairs"] == ref.shape[0]
    assert np.array_equal(E, ref[:, 0]) and np.array_equal(T, ref[:, 1])
    rp, col, val = ctx.export_csr("CF")
    _same_pattern(rp, col, S.Cf)
    assert np.abs(val[:, 0] - S.Cf.data).max() <= 1e-12 * abs(S.Cf.data).max()
    rp, col, val = ctx.export_csr("CFT")
    Ct = S.Cf.T.tocsr()
    Ct.sort_indices()
    _same_pattern(rp, col, Ct)
    assert np.abs(val[:, 0] - Ct.data).max() <= 1e-12 * abs(S.Cf.data).max()
    ctx.close()


def test_coupling_matching_mesh_degenerate_contacts():
    """Solid triangles equal to fluid triangles (every edge on a grid line)."""
    print("[coupling matching mesh]", flush=True)
    n = 8
    p2, p1, _ = fluid.triangle_nodes(n)
    Ts = [2 * (j * n + i) + t for j in (2, 3, 4) for i in (3, 4) for t in (0, 1)]
    verts = sorted(set(int(v) for T in Ts for v in p1[T]))
    ren = {v: k for k, v in enumerate(verts)}
    xy = fluid.p1_coords(n)[verts]
    tri = np.array([[ren[int(v)] for v in p1[T]] for T in Ts], dtype=np.int32)
    S = system.FSISystem(n, xy, tri)
    S.set_position(xy)
    ctx = fsi.Context(n, xy, tri)
    ctx.assemble_coupling(to_dev(soa(xy)))
    E, T = ctx.export_pairs()
    assert list(zip(E.tolist(), T.tolist())) == [(e, t) for e, t in S.pieces]
    assert [t for _, t in S.pieces] == Ts
    rp, col, val = ctx.export_csr("CF")
    _same_pattern(rp, col, S.Cf)
    assert np.abs(val[:, 0] - S.Cf.data).max() <= 1e-12 * abs(S.Cf.data).max()
    ctx.close()


@pytest.fixture(scope="module")
def pair32():
    wl = inputs.WORKLOADS["disk32"]
    S, ctx, X = make_pair(wl)
    yield S, ctx, wl
    ctx.close()


def test_operator_fp64_fp32(pair32):
    print("[operator]", flush=True)
    S, ctx, wl = pair32
    A = S.matrix()
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, S.lay.N)
    y_ref = A @ x
    torch = torch_dev()
    xd = to_dev(x)
    yd = torch.zeros_like(xd)
    ctx.apply_operator(xd, yd, fsi.FP64)
    y = to_host(yd)
    assert rel(y, y_ref) <= 1e-13
    assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max()
    ctx.apply_operator(xd, yd, fsi.FP32)
    assert rel(to_host(yd), y_ref) <= 2e-6


def test_rhs(pair32):
    print("[rhs]", flush=True)
    S, ctx, wl = pair32
    lay = S.lay
    rng = np.random.default_rng(12)
    u = rng.uniform(-1, 1, 2 * lay.N2)
    X = inputs.rotation(S.xy_ref, (0.5, 0.5), 0.1)
    b_ref = S.rhs(u, X)
    torch = torch_dev()
    b = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    ctx.build_rhs(to_dev(u), to_dev(soa(X)), b)
    assert rel(to_host(b), b_ref) <= 1e-13


INNER_MODES = pytest.mark.parametrize("inner", [fsi.INNER_MINRES, fsi.INNER_GMRES], ids=["minres", "gmres"])


@INNER_MODES
def test_precond_blocks(pair32, inner):
    """Both block preconditioners with tight inner solves (inner MINRES, the default, and inner
    GMRES with the block-triangular approximation) against the oracle's exact blocks."""
    print(f"[precond inner {inner}]", flush=True)
    S, ctx, wl = pair32
    ctx.set_inner_mode(inner)
    lay = S.lay
    nf = lay.nf
    rng = np.random.default_rng(13)
    r = S.random_rhs(0, rng.uniform(-1, 1, lay.N))
    torch = torch_dev()
    rd = to_dev(r)
    zd = torch.zeros_like(rd)
    ctx.set_inner(1e-13, 2000)
    ctx.apply_precond(rd, zd, fsi.PC_DIAG, fsi.FP64)
    z = to_host(zd)
    z22 = S.apply_A22_inv(r[nf:])
    assert rel(z[nf:], z22) <= 1e-12
    z11 = S.apply_A11_inv(r[:nf])
    assert rel(z[:nf], z11) <= 1e-9
    ctx.apply_precond(rd, zd, fsi.PC_TRI, fsi.FP64)
    zt = to_host(zd)
    zref = S.apply_precond(r, "tri")
    assert rel(zt, zref) <= 1e-9
    ctx.set_inner(-1.0, 1000)
    ctx.set_inner_mode(fsi.INNER_MINRES)


def _its_bound(its_oracle):
    return its_oracle + max(2, math.ceil(0.1 * its_oracle))


@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_gmres_degenerate_rhs(pair32, prec):
    """b = 0: the solve returns x = 0 at once (converged, no Arnoldi step) whatever x held.
    A non-finite b: FSI_E_NONFINITE with x untouched, and the context still solves after."""
    print(f"[gmres degenerate rhs prec={prec}]", flush=True)
    S, ctx, wl = pair32
    torch = torch_dev()
    N = ctx.sizes["N"]
    b = torch.zeros(N, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 3.0)
    st = ctx.gmres_solve(b, x, fsi.Opts(prec=prec))
    assert st["converged"] == 1 and st["its"] == 0
    assert torch.count_nonzero(x).item() == 0
    bad = to_dev(S.random_rhs(wl.seed))
    bad[5] = float("nan")
    with pytest.raises(fsi.FsiError) as e:
        ctx.gmres_solve(bad, x, fsi.Opts(prec=prec))
    assert e.value.code == fsi.FSI_E_NONFINITE
    assert torch.count_nonzero(x).item() == 0
    good = S.random_rhs(wl.seed)
    st = ctx.gmres_solve(to_dev(good), x, fsi.Opts(prec=prec))
    assert st["converged"] == 1 and st["relres_true"] <= 1e-8
    assert rel(S.matrix() @ to_host(x), good) <= 1e-8 * 1.0001


@pytest.mark.parametrize("pc", ["diag", "tri"])
def test_gmres_small_case(pair32, pc):
    print(f"[gmres {pc}]", flush=True)
    S, ctx, wl = pair32
    b = S.random_rhs(wl.seed)
    A = S.matrix()
    xs = S.solve_direct(b)
    _, info = gmres.gmres(lambda v: A @ v, b, precond=lambda r: S.apply_precond(r, pc), restart=30, rtol=1e-8)
    torch = torch_dev()
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI if pc == "tri" else fsi.PC_DIAG))
    x = to_host(xd)
    print(f"  gpu its {st['its']} oracle its {info['its']} relres {st['relres_true']:.2e}", flush=True)
    assert st["converged"] and st["relres_true"] <= 1e-8
    assert rel(A @ x, b) <= 1e-8 * 1.0001
    assert st["its"] <= _its_bound(info["its"])
    xd.zero_()
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI if pc == "tri" else fsi.PC_DIAG, rtol=1e-10))
    assert st["converged"]
    assert_block_parity(S, to_host(xd), xs, 1e-8, f"fp64 {pc}")


def test_gmres_mixed_precision(pair32):
    print("[gmres mixed]", flush=True)
    S, ctx, wl = pair32
    b = S.random_rhs(wl.seed)
    A = S.matrix()
    xs = S.solve_direct(b)
    torch = torch_dev()
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI, prec=fsi.FP32))
    x = to_host(xd)
    _, info = gmres.gmres(lambda v: A @ v, b, precond=lambda r: S.apply_precond(r, "tri"), restart=30, rtol=1e-8)
    print(f"  mixed its {st['its']} (oracle {info['its']}) relres {st['relres_true']:.2e}", flush=True)
    assert st["converged"] and rel(A @ x, b) <= 1e-8 * 1.0001
    assert st["its"] <= _its_bound(info["its"])
    xd.zero_()
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI, prec=fsi.FP32, rtol=1e-10))
    assert st["converged"]
    assert_block_parity(S, to_host(xd), xs, 1e-8, "mixed tri")


def test_step_against_oracle():
    print("[step]", flush=True)
    wl = inputs.small_workload(16, 4, (0.5, 0.5), 0.2, dt=0.01)
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    rng = np.random.default_rng(21)
    u = rng.uniform(-1, 1, 2 * lay.N2)
    bnd2 = np.concatenate([S.F["bnd"], S.F["bnd"]])
    u[bnd2] = 0.0
    X = inputs.rotation(S.xy_ref, (0.5, 0.5), 0.2)
    from oracle import step as ostep
    x_ref, _ = ostep.step(S, u, X, solver="direct")
    ctx = fsi.Context.from_workload(wl)
    torch = torch_dev()
    out = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    for prec in (fsi.FP64, fsi.FP32):
        st = ctx.step(to_dev(u), to_dev(soa(X)), out, fsi.Opts(pc=fsi.PC_TRI, rtol=1e-10, prec=prec))
        assert st["converged"]
        assert_block_parity(S, to_host(out), x_ref, 1e-8, f"step prec={prec}")
    ctx.close()


def test_step_solid_with_large_windows():
    """A solid much coarser than the fluid grid (C_f rows whose pieces span windows above the
    4,096 lattice nodes of the LDS form, assembled in device memory): a step within 1e-8 of the
    oracle's direct solve in every block.  The solve runs to rtol 1e-12: this coupling (up to
    5,080 entries in a row of C_f) amplifies the residual of an rtol-1e-10 solve to 4e-8 in u and
    3e-7 in p, element by element."""
    print("[step large windows]", flush=True)
    wl, angle = small_workloads()["huge_window128"]
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    X = _positions("huge_window128", S, angle)
    u = inputs.uniform(2 * lay.N2, 77)
    from oracle import step as ostep
    x_ref, _ = ostep.step(S, u, X, solver="direct")
    ctx = fsi.Context.from_workload(wl)
    torch = torch_dev()
    out = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    st = ctx.step(to_dev(u), to_dev(soa(X)), out, fsi.Opts(pc=fsi.PC_TRI, rtol=1e-12))
    assert st["converged"]
    assert_block_parity(S, to_host(out), x_ref, 1e-8, "large windows")
    ctx.close()


class _MeshSolid(inputs.Solid):
    """A solid given by its mesh (for the degenerate cases below)."""

    def __init__(self, xy, tri):
        super().__init__(m=1, center=(0.5, 0.5), radius=0.1)
        self._xy, self._tri = np.asarray(xy, dtype=np.float64), np.asarray(tri, dtype=np.int32)

    def mesh(self):
        return self._xy.copy(), self._tri.copy()


DEGENERATE = {
    # one solid triangle (three nodes: every solid row has three entries)
    "one_triangle16": (16, [[0.41, 0.37], [0.63, 0.45], [0.47, 0.66]], [[0, 1, 2]]),
    # a bar against the wall x = 0 (the paper's position): solid nodes on Dirichlet nodes of the
    # fluid, whose C_f columns are zero
    "bar_at_wall32": (32, None, None),
    # solid nodes exactly on fluid lattice lines and cell diagonals (pieces with edges on the
    # clip lines)
    "on_grid_lines16": (16, [[0.25, 0.25], [0.5, 0.25], [0.5, 0.5], [0.25, 0.5], [0.375, 0.375]],
                        [[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]]),
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_step_degenerate_solids(name):
    """Steps with degenerate solids against the oracle's direct solve, per block within 1e-8:
    a single triangle, a bar whose left end lies on the Dirichlet wall, and a solid whose
    nodes and edges lie on the fluid grid's lines and diagonals."""
    print(f"[step degenerate {name}]", flush=True)
    n, xy, tri = DEGENERATE[name]
    if xy is None:
        solid = inputs.Bar(m=0, center=(0.2, 0.5), nx=13, ny=3, x0=0.0)
    else:
        solid = _MeshSolid(xy, tri)
    wl = inputs.Workload(name, n, [solid], dt=0.01, seed=5)
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    u = inputs.uniform(2 * lay.N2, 31)
    bnd2 = np.concatenate([S.F["bnd"], S.F["bnd"]])
    u[bnd2] = 0.0
    X = S.xy_ref.copy()
    from oracle import step as ostep
    x_ref, _ = ostep.step(S, u, X, solver="direct")
    ctx = fsi.Context.from_workload(wl)
    torch = torch_dev()
    out = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    for prec in (fsi.FP64, fsi.FP32):
        st = ctx.step(to_dev(u), to_dev(soa(X)), out, fsi.Opts(pc=fsi.PC_TRI, rtol=1e-12, prec=prec))
        assert st["converged"]
        assert_block_parity(S, to_host(out), x_ref, 1e-8, f"{name} prec={prec}")
    ctx.close()


def test_error_paths():
    print("[errors]", flush=True)
    wl = inputs.small_workload(8, 2, (0.5, 0.5), 0.2)
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    torch = torch_dev()
    N = ctx.sizes["N"]
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(fsi.FsiError) as e:
        ctx.apply_operator(x, y)
    assert e.value.code == fsi.FSI_E_STATE
    bad = xy.copy()
    bad[:, 0] = 1.0 - bad[:, 0]
    with pytest.raises(fsi.FsiError) as e:
        ctx.assemble_coupling(to_dev(soa(bad)))
    assert e.value.code == fsi.FSI_E_MESH
    out = xy.copy()
    out[:, 0] += 0.45
    with pytest.raises(fsi.FsiError) as e:
        ctx.assemble_coupling(to_dev(soa(out)))
    assert e.value.code == fsi.FSI_E_MESH
    # a valid position afterwards still works
    ctx.assemble_coupling(to_dev(soa(xy)))
    ctx.apply_operator(x, y)
    with pytest.raises(fsi.FsiError) as e:
        fsi.Context(8, xy, tri[:, ::-1])
    assert e.value.code == fsi.FSI_E_MESH
    # an odd grid above the dense-16^2 threshold has one multigrid level, too large for a
    # dense coarsest inverse: refused with FSI_E_ARG
    with pytest.raises(fsi.FsiError) as e:
        fsi.Context(513, xy, tri)
    assert e.value.code == fsi.FSI_E_ARG
    ctx.close()


def test_repeatable_bitwise(pair32):
    print("[determinism]", flush=True)
    S, ctx, wl = pair32
    b = S.random_rhs(wl.seed)
    torch = torch_dev()
    bd = to_dev(b)
    outs = []
    for _ in range(2):
        ctx.assemble_coupling(to_dev(soa(S.xy_ref)))
        xd = torch.zeros_like(bd)
        ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI))
        outs.append(to_host(xd))
    assert np.array_equal(outs[0], outs[1])


def test_time_loop_against_oracle():
    """Row a9: prescribed rotation (0.1 rad/s about the centre), u^{n+1} feeds the next
    step, C_f re-clipped every step; every state within 1e-8 of the oracle's."""
    print("[time loop]", flush=True)
    wl = inputs.small_workload(16, 4, (0.5, 0.5), 0.2, dt=0.05)
    S = system.FSISystem.from_workload(wl)
    lay = S.lay
    from oracle import step as ostep
    Xk = lambda k: inputs.rotation(S.xy_ref, (0.5, 0.5), 0.1 * k * wl.dt * 20)
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, 2 * lay.N2)
    steps = 4
    ref = ostep.time_loop(S, Xk, steps, u0=u0, solver="direct")
    ctx = fsi.Context.from_workload(wl)
    torch = torch_dev()
    u = to_dev(u0)
    out = torch.zeros(lay.N, dtype=torch.float64, device="cuda")
    for k in range(steps):
        st = ctx.step(u, to_dev(soa(Xk(k))), out, fsi.Opts(pc=fsi.PC_TRI, rtol=1e-10))
        assert st["converged"]
        assert_block_parity(S, to_host(out), ref[k], 1e-8, f"time loop step {k}")
        u = out[:2 * lay.N2].clone()
    ctx.close()


def test_gmres_fp32_ir(pair32):
    """The refinement form: FP32 operator inside the Arnoldi process, FP64 residuals."""
    print("[gmres fp32-ir]", flush=True)
    S, ctx, wl = pair32
    b = S.random_rhs(wl.seed)
    A = S.matrix()
    xs = S.solve_direct(b)
    torch = torch_dev()
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI, prec=fsi.FP32_IR))
    x = to_host(xd)
    print(f"  fp32-ir its {st['its']} refinements {st['refinements']} relres {st['relres_true']:.2e}", flush=True)
    assert st["converged"] and st["refinements"] >= 1 and rel(A @ x, b) <= 1e-8 * 1.0001
    xd.zero_()
    st = ctx.gmres_solve(bd, xd, fsi.Opts(pc=fsi.PC_TRI, prec=fsi.FP32_IR, rtol=1e-10))
    assert st["converged"]
    assert_block_parity(S, to_host(xd), xs, 1e-8, "fp32-ir tri")


@INNER_MODES
@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_stencil_smoother_equals_csr(pair32, prec, inner):
    """The matrix-free A_f products of the V-cycle give the same preconditioner as the
    assembled blocks: after one or two inner steps (isolating the V-cycle) and converged.
    At 32^2 the matrix-free cycle runs every fused launch against the CSR products and
    separate transfers: the post-smoothing launch that adds the coarse correction, the
    residual kept in LDS and restricted in one launch, and the one-launch tail (16^2, 8^2
    and the dense 4^2 solve)."""
    print(f"[stencil vs csr prec={prec} inner {inner}]", flush=True)
    S, ctx, wl = pair32
    ctx.set_inner_mode(inner)
    lay = S.lay
    rng = np.random.default_rng(31)
    r = S.random_rhs(0, rng.uniform(-1, 1, lay.N))
    torch = torch_dev()
    rd = to_dev(r)
    out = {}
    for maxit, tol in ((1, 1e-30), (2, 1e-30), (2000, 1e-12)):
        for kind in (fsi.SMOOTH_CSR, fsi.SMOOTH_STENCIL):
            ctx.set_smoother(kind)
            ctx.set_inner(tol, maxit)
            zd = torch.zeros_like(rd)
            ctx.apply_precond(rd, zd, fsi.PC_TRI, prec)
            out[(maxit, kind)] = to_host(zd)
        d = rel(out[(maxit, fsi.SMOOTH_STENCIL)], out[(maxit, fsi.SMOOTH_CSR)])
        print(f"  maxit {maxit}: rel diff {d:.2e}", flush=True)
        assert d <= (1e-12 if prec == fsi.FP64 else 1e-5)
    ctx.set_smoother(fsi.SMOOTH_STENCIL)
    ctx.set_inner(-1.0, 1000)
    ctx.set_inner_mode(fsi.INNER_MINRES)
    if prec == fsi.FP64:
        zref = S.apply_precond(r, "tri")
        assert rel(out[(2000, fsi.SMOOTH_STENCIL)], zref) <= 1e-9


@pytest.mark.parametrize("n", [24, 48, 64, 96])
def test_multigrid_tiles_and_odd_coarsest(n):
    """Grids of 3 x 2^k cells (24, 48, 96): the velocity hierarchy ends on the odd 3^2 level
    (dense solve) and the one-launch tail starts at 12^2; 64 ends on 4^2 with the tail from
    16^2.  At 64 and 96 the finest lattice is 129 and 193 nodes wide, so the tiled launches
    (120-node tiles of the post-smoothing, 124 of the pre-smoothing, 128 of the single-step
    and A11 launches) have two tile columns with a ragged last one, and the seams of the
    smoothing, of the fused residual-restriction and of the coarse-correction fold are
    compared.  The matrix-free cycle equals the CSR one after one and two inner steps, in
    FP64 and FP32, and the converged FP64 inner solve equals the oracle's A11 solve."""
    print(f"[odd coarsest n={n}]", flush=True)
    wl = inputs.small_workload(n, 4, (0.5, 0.5), 0.2)
    S, ctx, _ = make_pair(wl)
    nf = S.lay.nf
    rng = np.random.default_rng(41 + n)
    r = S.random_rhs(0, rng.uniform(-1, 1, S.lay.N))
    torch = torch_dev()
    rd = to_dev(r)
    for prec in (fsi.FP64, fsi.FP32):
        for maxit in (1, 2):
            out = {}
            for kind in (fsi.SMOOTH_CSR, fsi.SMOOTH_STENCIL):
                ctx.set_smoother(kind)
                ctx.set_inner(1e-30, maxit)
                zd = torch.zeros_like(rd)
                ctx.apply_precond(rd, zd, fsi.PC_DIAG, prec)
                out[kind] = to_host(zd)
            d = rel(out[fsi.SMOOTH_STENCIL], out[fsi.SMOOTH_CSR])
            print(f"  prec {prec} maxit {maxit}: rel diff {d:.2e}", flush=True)
            assert d <= (1e-12 if prec == fsi.FP64 else 1e-5)
    ctx.set_smoother(fsi.SMOOTH_STENCIL)
    ctx.set_inner(1e-13, 2000)
    zd = torch.zeros_like(rd)
    ctx.apply_precond(rd, zd, fsi.PC_DIAG, fsi.FP64)
    assert rel(to_host(zd)[:nf], S.apply_A11_inv(r[:nf])) <= 1e-9
    ctx.set_inner(-1.0, 1000)
    ctx.close()


@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_graph_replays_equal_eager(pair32, prec):
    """The captured preconditioner graph (of the inner MINRES, the inner mode that replays
    graphs), replayed many times with different inputs and with eager work and
    synchronisations in between, gives the eager result bitwise."""
    print(f"[graph replays prec={prec}]", flush=True)
    S, ctx, wl = pair32
    lay = S.lay
    torch = torch_dev()
    ctx.set_inner_mode(fsi.INNER_MINRES)
    rng = np.random.default_rng(41)
    rs = [to_dev(S.random_rhs(0, rng.uniform(-1, 1, lay.N))) for _ in range(3)]
    eager = []
    ctx.set_graphs(False)
    for rd in rs:
        zd = torch.zeros_like(rd)
        ctx.apply_precond(rd, zd, fsi.PC_TRI, prec)
        eager.append(to_host(zd))
    ctx.set_graphs(True)
    for rep in range(3):
        for k, rd in enumerate(rs):
            zd = torch.zeros_like(rd)
            ctx.apply_precond(rd, zd, fsi.PC_TRI, prec)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(zd), eager[k]), (rep, k)
            # eager work on the same stream between replays
            y = torch.zeros_like(rd)
            ctx.apply_operator(rd, y)
    b = to_dev(S.random_rhs(wl.seed))
    x1 = torch.zeros_like(b)
    ctx.gmres_solve(b, x1, fsi.Opts(pc=fsi.PC_TRI, prec=prec, inner_mode=fsi.INNER_MINRES))
    ctx.set_graphs(False)
    x0 = torch.zeros_like(b)
    ctx.gmres_solve(b, x0, fsi.Opts(pc=fsi.PC_TRI, prec=prec, inner_mode=fsi.INNER_MINRES))
    assert np.array_equal(to_host(x0), to_host(x1))
    ctx.set_graphs(True)
    ctx.set_inner_mode(fsi.INNER_MINRES)
