"""Lockstep batches of small steps (fsi_step_batch, the batched serving form): every
system's result must equal its step alone bitwise (each system runs the same kernels; the
inner A11 solves of all systems are lanes of one launch), across lane counts that grow
and shrink on one leading context, with and without captured graphs, in FP64, mixed
precision and FP32 refinement; one batch is checked against the FP64 oracle, and batches that mix fluid
grids or repeat a context are refused."""
import numpy as np
import pytest

from oracle import step as ostep
from oracle import system
from paper_2301_10041_amd import fsi, inputs

from gpu_helpers import assert_block_parity, rel, soa, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def workloads(n, count, seed=11):
    rng = np.random.default_rng(seed + n)
    out = []
    for i in range(count):
        cx, cy = rng.uniform(0.35, 0.65, 2)
        r = float(rng.uniform(0.08, 0.2))
        m = int(rng.integers(3, 9))
        axes = (r, r * float(rng.uniform(0.6, 1.0))) if rng.random() < 0.5 else None
        out.append(inputs.Workload(f"b{n}_{i}", n, [inputs.Solid(m, (float(cx), float(cy)), r, axes)], dt=0.01,
                                   seed=3000 + 17 * i + n))
    return out


def inputs_of(wl, ctx):
    torch = torch_dev()
    xy, _ = wl.solid_mesh()
    u = to_dev(inputs.uniform(2 * ctx.sizes["N2"], wl.seed))
    X = to_dev(soa(xy))
    state = torch.zeros(ctx.sizes["N"], dtype=torch.float64, device="cuda")
    return u, X, state


def alone(wl, opts, graphs):
    ctx = fsi.Context.from_workload(wl)
    ctx.set_graphs(graphs)
    u, X, state = inputs_of(wl, ctx)
    st = ctx.step(u, X, state, opts)
    out = to_host(state)
    ctx.close()
    return out, st


def batch(ctxs, wls, opts):
    ins = [inputs_of(wl, c) for wl, c in zip(wls, ctxs)]
    stats, rcs = fsi.step_batch(ctxs, [i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins], opts)
    return [to_host(i[2]) for i in ins], stats, rcs


CASES = [
    ("n16_fp64_graphs", 16, fsi.FP64, True, [4, 2, 5]),
    ("n32_mixed_graphs", 32, fsi.FP32, True, [3, 1]),
    ("n16_fp64_eager", 16, fsi.FP64, False, [3]),
    ("n16_fp32ir_graphs", 16, fsi.FP32_IR, True, [3]),
]


@pytest.mark.parametrize("inner", [fsi.INNER_MINRES, fsi.INNER_GMRES], ids=["minres", "gmres"])
@pytest.mark.parametrize("name,n,prec,graphs,ks", CASES, ids=[c[0] for c in CASES])
def test_batch_equals_alone_bitwise(name, n, prec, graphs, ks, inner):
    """Each system of a lockstep batch equals its step alone bitwise, for lane counts that grow
    and shrink on one context, with the inner MINRES (whose iterations replay captured graphs
    when graphs are on) and the inner GMRES (no graphs)."""
    torch_dev()
    print(f"[batch {name} inner {inner} K={ks}]", flush=True)
    opts = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-8, inner_mode=inner)
    wls = workloads(n, max(ks))
    ref = [alone(wl, opts, graphs) for wl in wls]
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    for c in ctxs:
        c.set_graphs(graphs)
    for K in ks:   # lane counts grow and shrink on the same leading context
        states, stats, rcs = batch(ctxs[:K], wls[:K], opts)
        assert rcs == [fsi.FSI_OK] * K
        for k in range(K):
            a, sa = ref[k]
            assert np.array_equal(states[k], a), (K, k)
            assert stats[k]["its"] == sa["its"] and stats[k]["inner_its"] == sa["inner_its"], (K, k)
            assert stats[k]["converged"] == 1
        print(f"  K={K} its={[s['its'] for s in stats]} inner={[s['inner_its'] for s in stats]}", flush=True)
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_inner_check_modes_bitwise(prec):
    """The inner MINRES convergence check every step, one step late (the step past convergence
    frozen by the device's done flag) and by default: the same states and counts, bitwise, for
    one system and for a lockstep batch of three at 48^2 (where the default is the lagged
    check); an unknown mode is refused."""
    torch_dev()
    print(f"[inner check modes prec={prec}]", flush=True)
    opts = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-8)
    wls = workloads(48, 3, seed=23)
    res = {}
    for mode in (fsi.CHECK_EVERY_STEP, fsi.CHECK_LAGGED, fsi.CHECK_AUTO):
        ctxs = [fsi.Context.from_workload(wl) for wl in wls]
        for c in ctxs:
            c.set_inner_check(mode)
        u, X, state = inputs_of(wls[0], ctxs[0])
        st = ctxs[0].step(u, X, state, opts)
        one = to_host(state)
        states, stats, rcs = batch(ctxs, wls, opts)
        assert rcs == [fsi.FSI_OK] * 3
        res[mode] = (one, st["its"], st["inner_its"], states, [(s["its"], s["inner_its"]) for s in stats])
        for c in ctxs:
            c.close()
    ref = res[fsi.CHECK_EVERY_STEP]
    for mode in (fsi.CHECK_LAGGED, fsi.CHECK_AUTO):
        got = res[mode]
        assert np.array_equal(got[0], ref[0]) and got[1:3] == ref[1:3], mode
        assert all(np.array_equal(a, b) for a, b in zip(got[3], ref[3])) and got[4] == ref[4], mode
    with pytest.raises(fsi.FsiError):
        ctx = fsi.Context.from_workload(wls[0])
        try:
            ctx.set_inner_check(3)
        finally:
            ctx.close()


def test_batch_matches_oracle():
    torch_dev()
    print("[batch oracle]", flush=True)
    wls = workloads(16, 3, seed=5)
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    states, stats, rcs = batch(ctxs, wls, fsi.Opts(prec=fsi.FP64, rtol=1e-10))
    assert rcs == [fsi.FSI_OK] * 3
    for wl, x in zip(wls, states):
        S = system.FSISystem.from_workload(wl)
        u = inputs.uniform(2 * S.lay.N2, wl.seed)
        x_ref, _ = ostep.step(S, u, S.xy_ref, solver="direct")
        assert_block_parity(S, x, x_ref, 1e-8, wl.name)
    for c in ctxs:
        c.close()


def test_batch_refuses_mixed_grids_and_repeats():
    torch_dev()
    print("[batch refusals]", flush=True)
    wa = workloads(16, 1)[0]
    wb = workloads(32, 1)[0]
    ca, cb = fsi.Context.from_workload(wa), fsi.Context.from_workload(wb)
    ia, ib = inputs_of(wa, ca), inputs_of(wb, cb)
    with pytest.raises(fsi.FsiError) as e:
        fsi.step_batch([ca, cb], [ia[0], ib[0]], [ia[1], ib[1]], [ia[2], ib[2]])
    assert e.value.code == fsi.FSI_E_ARG
    with pytest.raises(fsi.FsiError) as e:
        fsi.step_batch([ca, ca], [ia[0], ia[0]], [ia[1], ia[1]], [ia[2], ia[2]])
    assert e.value.code == fsi.FSI_E_ARG
    with pytest.raises(ValueError):
        fsi.step_batch([], [], [], [])
    # the contexts still work after a refused batch
    st = ca.step(ia[0], ia[1], ia[2])
    assert st["converged"] == 1
    ca.close()
    cb.close()


def test_batch_reports_nonconvergence_per_system():
    """A step budget too small for convergence: every system of the batch reports
    FSI_E_NOCONV in its own status, and its last iterate equals that of the same step alone
    (bitwise); the batch call itself does not raise."""
    torch_dev()
    print("[batch noconv]", flush=True)
    opts = fsi.Opts(prec=fsi.FP64, pc=fsi.PC_TRI, rtol=1e-8, maxit=3, restart=2)
    wls = workloads(16, 3, seed=23)
    ref = []
    for wl in wls:
        ctx = fsi.Context.from_workload(wl)
        u, X, state = inputs_of(wl, ctx)
        with pytest.raises(fsi.FsiError) as e:
            ctx.step(u, X, state, opts)
        assert e.value.code == fsi.FSI_E_NOCONV
        ref.append(to_host(state))
        ctx.close()
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    states, stats, rcs = batch(ctxs, wls, opts)
    assert rcs == [fsi.FSI_E_NOCONV] * 3
    for k in range(3):
        assert stats[k]["converged"] == 0 and stats[k]["its"] == 3
        assert np.array_equal(states[k], ref[k]), k
    for c in ctxs:
        c.close()


class FanSolid(inputs.Solid):
    """A fan of k triangles around one centre node: the centre's row of the solid pattern
    has k + 1 entries, more than a ring mesh ever has (at most 7)."""

    def __init__(self, k, center, radius):
        super().__init__(m=1, center=center, radius=radius)
        self.k = k

    def mesh(self):
        a = 2 * np.pi * np.arange(self.k) / self.k
        xy = np.concatenate([[self.center], np.stack([self.center[0] + self.radius * np.cos(a),
                                                      self.center[1] + self.radius * np.sin(a)], axis=1)])
        tri = np.array([[0, 1 + i, 1 + (i + 1) % self.k] for i in range(self.k)], dtype=np.int32)
        return xy, tri


def test_batch_high_valence_solid():
    """Solids whose centre node has 12 or 16 neighbours (rows longer than the unrolled part of
    the batched A22 closed form): a batch equals each step alone bitwise, and the result
    matches the oracle's direct solve."""
    torch_dev()
    print("[batch high valence]", flush=True)
    wls = [inputs.Workload(f"fan{k}", 16, [FanSolid(k, (0.5 + 0.01 * k, 0.47), 0.15)], dt=0.01, seed=700 + k)
           for k in (12, 16)]
    opts = fsi.Opts(prec=fsi.FP64, pc=fsi.PC_TRI, rtol=1e-10)
    ref = [alone(wl, opts, False) for wl in wls]
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    states, stats, rcs = batch(ctxs, wls, opts)
    assert rcs == [fsi.FSI_OK] * 2
    for k, wl in enumerate(wls):
        assert np.array_equal(states[k], ref[k][0]), wl.name
        S = system.FSISystem.from_workload(wl)
        u = inputs.uniform(2 * S.lay.N2, wl.seed)
        x_ref, _ = ostep.step(S, u, S.xy_ref, solver="direct")
        assert_block_parity(S, states[k], x_ref, 1e-8, wl.name)
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_fixed_cost_inner_mode(prec):
    """FSI_INNER_FIXED_DIAG (A11^{-1} by one application of the block-diagonal inner
    preconditioner, no inner Krylov steps):
    the step converges to rtol with no inner steps and more outer steps, matches the oracle's
    direct solve, and a batch equals each step alone bitwise; other modes are refused."""
    torch_dev()
    print(f"[fixed-cost inner mode prec={prec}]", flush=True)
    wls = workloads(16, 3, seed=41)
    opts = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-10, inner_mode=fsi.INNER_FIXED_DIAG)
    ref = [alone(wl, opts, False) for wl in wls]
    base = alone(wls[0], fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-10), False)
    for (x, st) in ref:
        assert st["converged"] == 1 and st["inner_its"] == 0 and st["relres_true"] <= 1e-10
    assert ref[0][1]["its"] > base[1]["its"]
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    states, stats, rcs = batch(ctxs, wls, opts)
    assert rcs == [fsi.FSI_OK] * 3
    for k, wl in enumerate(wls):
        assert np.array_equal(states[k], ref[k][0]), wl.name
        assert stats[k]["its"] == ref[k][1]["its"]
    S = system.FSISystem.from_workload(wls[0])
    u = inputs.uniform(2 * S.lay.N2, wls[0].seed)
    x_ref, _ = ostep.step(S, u, S.xy_ref, solver="direct")
    assert_block_parity(S, states[0], x_ref, 1e-8, "fixed-cost")
    u0, X0, s0 = inputs_of(wls[0], ctxs[0])
    for bad in (fsi.Opts(prec=prec, inner_mode=4), fsi.Opts(prec=prec, inner_mode=fsi.INNER_FIXED_TRI, inner_cycles=101)):
        with pytest.raises(fsi.FsiError) as e:
            ctxs[0].step(u0, X0, s0, bad)
        assert e.value.code == fsi.FSI_E_ARG
    st = ctxs[0].step(u0, X0, s0, fsi.Opts(prec=prec, rtol=1e-10))   # the default mode again
    assert st["inner_its"] > 0 and st["converged"] == 1
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_fixed_cost_block_triangular(prec):
    """FSI_INNER_FIXED_TRI (A11^{-1} by stationary cycles with the block upper-triangular
    approximation, the pressure part before the velocity cycle): the step converges with no
    inner steps and matches the oracle's direct solve per block; one cycle takes fewer outer
    steps than the block-diagonal fixed-cost form, two cycles fewer still; a batch equals each
    step alone bitwise."""
    torch_dev()
    print(f"[fixed-cost block-triangular prec={prec}]", flush=True)
    wls = workloads(16, 3, seed=41)
    # rtol 1e-11: at 1e-10 the largest pressure entry was 1.2e-8 off (2-norm 4e-9)
    o1 = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-11, inner_mode=fsi.INNER_FIXED_TRI, inner_cycles=1)
    o2 = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-11, inner_mode=fsi.INNER_FIXED_TRI, inner_cycles=2)
    ref = [alone(wl, o1, False) for wl in wls]
    diag = alone(wls[0], fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-11, inner_mode=fsi.INNER_FIXED_DIAG), False)
    two = alone(wls[0], o2, False)
    for (x, st) in ref + [two]:
        assert st["converged"] == 1 and st["inner_its"] == 0 and st["relres_true"] <= 1e-11
    print(f"  outer its: block-diagonal {diag[1]['its']}, block-triangular 1 cycle {ref[0][1]['its']}, "
          f"2 cycles {two[1]['its']}", flush=True)
    assert ref[0][1]["its"] < diag[1]["its"]
    assert two[1]["its"] < ref[0][1]["its"]
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    states, stats, rcs = batch(ctxs, wls, o1)
    assert rcs == [fsi.FSI_OK] * 3
    for k, wl in enumerate(wls):
        assert np.array_equal(states[k], ref[k][0]), wl.name
        assert stats[k]["its"] == ref[k][1]["its"]
    for c in ctxs:
        c.close()
    S = system.FSISystem.from_workload(wls[0])
    u = inputs.uniform(2 * S.lay.N2, wls[0].seed)
    x_ref, _ = ostep.step(S, u, S.xy_ref, solver="direct")
    assert_block_parity(S, ref[0][0], x_ref, 1e-8, "block-triangular 1 cycle")
    assert_block_parity(S, two[0], x_ref, 1e-8, "block-triangular 2 cycles")

