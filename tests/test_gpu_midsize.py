"""Parity at the sizes the tiled kernels run at full scale, through the C-ABI.

* A full step (fsi_step) of the two-disk geometry on a 128^2 grid (257-node lattice: three
  tile columns of every tiled launch with a ragged last one; five multigrid levels above the
  one-launch tail) against the oracle's direct solve, block-diagonal and block-triangular,
  FP64 and mixed precision: every block (u, mean-free p, X, lam) within 1e-8 in the 2-norm and
  element by element (parity solves at rtol 1e-10).
* Outer iteration counts at rtol 1e-8 against the oracle's exact-block counts stored in
  tests/golden/its.json (written by tests/golden/make_its.py from oracle/ only):
  its_gpu <= its_oracle + max(2, ceil(0.1 its_oracle)) in FP64 and mixed precision.
* Lockstep batches of K = 4 systems at 64^2 and 128^2 equal each step alone bitwise.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import step as ostep
from oracle import system
from paper_2301_10041_amd import fsi, inputs

from gpu_helpers import assert_block_parity, soa, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "its.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    fsi.lib()


def _step_inputs(wl, N2):
    """u^n ~ U[-1, 1] (the workload's seed; boundary entries are ignored by the step) and X^n the
    reference mesh rotated by 1e-3 rad about (0.5, 0.5)."""
    xy, _ = wl.solid_mesh()
    u = inputs.uniform(2 * N2, wl.seed)
    X = inputs.rotation(xy, (0.5, 0.5), 1e-3)
    return u, X


@pytest.fixture(scope="module")
def twodisk128():
    wl = inputs.WORKLOADS["twodisk128"]
    S = system.FSISystem.from_workload(wl)
    u, X = _step_inputs(wl, S.lay.N2)
    x_ref, _ = ostep.step(S, u, X, solver="direct")
    ctx = fsi.Context.from_workload(wl)
    yield wl, S, u, X, x_ref, ctx
    ctx.close()


STEP128 = [("diag", fsi.FP64, fsi.INNER_MINRES), ("diag", fsi.FP32, fsi.INNER_MINRES),
           ("tri", fsi.FP64, fsi.INNER_MINRES), ("tri", fsi.FP32, fsi.INNER_MINRES),
           ("tri", fsi.FP64, fsi.INNER_GMRES), ("tri", fsi.FP32, fsi.INNER_GMRES)]


@pytest.mark.parametrize("pc,prec,inner", STEP128, ids=[f"{p}-{q}-{m}" for p, q, m in STEP128])
def test_step_twodisk128_against_oracle(twodisk128, pc, prec, inner):
    """A whole step of the two-disk geometry at 128^2 against the oracle's refined direct solve,
    per block within 1e-8: both preconditioners and precisions with the inner MINRES, and the
    block-triangular one with the inner GMRES of the weighted norm."""
    print(f"[step twodisk128 pc={pc} prec={prec} inner={inner}]", flush=True)
    torch = torch_dev()
    wl, S, u, X, x_ref, ctx = twodisk128
    out = torch.zeros(S.lay.N, dtype=torch.float64, device="cuda")
    opts = fsi.Opts(pc=fsi.PC_TRI if pc == "tri" else fsi.PC_DIAG, prec=prec, rtol=1e-10, inner_mode=inner)
    st = ctx.step(to_dev(u), to_dev(soa(X)), out, opts)
    print(f"  its {st['its']} inner {st['inner_its']} relres {st['relres_true']:.2e}", flush=True)
    assert st["converged"] and st["relres_true"] <= 1e-10
    assert_block_parity(S, to_host(out), x_ref, 1e-8, f"twodisk128 {pc} prec={prec} inner={inner}")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _its_bound(its):
    return its + max(2, math.ceil(0.1 * its))


def _dirichlet_zeroed(b, n):
    """Zero the rows of boundary velocity nodes (lattice index on an edge of [0, 2n]^2) and the
    pinned pressure node, as the oracle's seeded right-hand sides do."""
    L = 2 * n + 1
    I, J = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    bnd = ((I == 0) | (J == 0) | (I == 2 * n) | (J == 2 * n)).ravel()
    N2 = L * L
    b = b.copy()
    b[:N2][bnd] = 0.0
    b[N2:2 * N2][bnd] = 0.0
    b[2 * N2] = 0.0
    return b


ITS_CASES = [(case, pc, prec) for case, pcs in (("disk32", ("diag", "tri")), ("twodisk128", ("diag", "tri")),
                                                ("ellipse256", ("diag", "tri")), ("rotdisk256_step0", ("diag", "tri")))
             for pc in pcs for prec in ("fp64", "mixed")]


@pytest.mark.parametrize("case,pc,prec", ITS_CASES, ids=[f"{c}-{p}-{q}" for c, p, q in ITS_CASES])
def test_iterations_within_oracle_bound(case, pc, prec):
    gold = _golden()
    if case not in gold or pc not in gold[case]:
        pytest.fail(f"{case}/{pc} missing from {GOLDEN}: run tests/golden/make_its.py {case}")
    rec = gold[case]
    ref_its = rec[pc]["its"]
    print(f"[its {case} {pc} {prec}: oracle {ref_its}]", flush=True)
    torch = torch_dev()
    wl = inputs.WORKLOADS[rec["workload"]]
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    N, N2 = ctx.sizes["N"], ctx.sizes["N2"]
    assert N == rec["N"]
    X = to_dev(soa(xy))
    p = fsi.PC_TRI if pc == "tri" else fsi.PC_DIAG
    q = fsi.FP64 if prec == "fp64" else fsi.FP32
    opts = fsi.Opts(pc=p, prec=q, rtol=1e-8, restart=30)
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    if rec["rhs"] == "random":
        ctx.assemble_coupling(X)
        b = to_dev(_dirichlet_zeroed(inputs.uniform(N, wl.seed), wl.n))
        st = ctx.gmres_solve(b, x, opts)
    else:   # first step of the time loop: u^0 = 0, X^0 the reference mesh
        u0 = torch.zeros(2 * N2, dtype=torch.float64, device="cuda")
        st = ctx.step(u0, X, x, opts)
    ctx.close()
    print(f"  gpu its {st['its']} (bound {_its_bound(ref_its)}) relres {st['relres_true']:.2e}", flush=True)
    assert st["converged"] and st["relres_true"] <= 1e-8
    assert st["its"] <= _its_bound(ref_its)


def _batch_workloads(n, count, seed):
    """Disks and ellipses with solid triangles about the size of a fluid cell."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        cx, cy = rng.uniform(0.35, 0.65, 2)
        r = float(rng.uniform(0.08, 0.2))
        m = max(3, int(round(r * n / 1.2)))
        axes = (r, r * float(rng.uniform(0.6, 1.0))) if rng.random() < 0.5 else None
        out.append(inputs.Workload(f"m{n}_{i}", n, [inputs.Solid(m, (float(cx), float(cy)), r, axes)], dt=0.01,
                                   seed=5000 + 31 * i + n))
    return out


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("prec", [fsi.FP64, fsi.FP32])
def test_batch4_equals_alone_midsize(n, prec):
    torch = torch_dev()
    print(f"[batch K=4 n={n} prec={prec}]", flush=True)
    wls = _batch_workloads(n, 4, 90 + n)
    opts = fsi.Opts(prec=prec, pc=fsi.PC_TRI, rtol=1e-8)

    def ins(wl, ctx):
        xy, _ = wl.solid_mesh()
        return (to_dev(inputs.uniform(2 * ctx.sizes["N2"], wl.seed)), to_dev(soa(xy)),
                torch.zeros(ctx.sizes["N"], dtype=torch.float64, device="cuda"))

    ref = []
    for wl in wls:
        ctx = fsi.Context.from_workload(wl)
        u, X, s = ins(wl, ctx)
        st = ctx.step(u, X, s, opts)
        ref.append((to_host(s), st))
        ctx.close()
    ctxs = [fsi.Context.from_workload(wl) for wl in wls]
    io = [ins(wl, c) for wl, c in zip(wls, ctxs)]
    stats, rcs = fsi.step_batch(ctxs, [i[0] for i in io], [i[1] for i in io], [i[2] for i in io], opts)
    assert rcs == [fsi.FSI_OK] * 4
    for k in range(4):
        assert np.array_equal(to_host(io[k][2]), ref[k][0]), k
        assert stats[k]["its"] == ref[k][1]["its"] and stats[k]["inner_its"] == ref[k][1]["inner_its"], k
    print(f"  its {[s['its'] for s in stats]} inner {[s['inner_its'] for s in stats]}", flush=True)
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_triangular_cycles_approach_the_exact_block_count(prec):
    """FSI_INNER_FIXED_TRI with many cycles: the stationary block-triangular iteration converges to
    A11^{-1} r, so the outer count reaches the oracle's exact-block count (the iteration bar);
    a wrong sign or block in the iteration would diverge or stall instead."""
    gold = _golden()
    rec = gold["disk32"]
    ref_its = rec["tri"]["its"]
    print(f"[block-triangular cycles disk32 {prec}: oracle {ref_its}]", flush=True)
    torch = torch_dev()
    wl = inputs.WORKLOADS["disk32"]
    xy, _ = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    N = ctx.sizes["N"]
    ctx.assemble_coupling(to_dev(soa(xy)))
    b = to_dev(_dirichlet_zeroed(inputs.uniform(N, wl.seed), wl.n))
    q = fsi.FP64 if prec == "fp64" else fsi.FP32
    its = []
    for cycles in (1, 4, 40):
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st = ctx.gmres_solve(b, x, fsi.Opts(pc=fsi.PC_TRI, prec=q, rtol=1e-8, inner_mode=fsi.INNER_FIXED_TRI,
                                                inner_cycles=cycles))
        assert st["converged"] and st["relres_true"] <= 1e-8
        its.append(st["its"])
    ctx.close()
    print(f"  outer its for 1, 4, 40 cycles: {its}", flush=True)
    assert its[0] > its[1] >= its[2]
    assert its[2] <= _its_bound(ref_its)

