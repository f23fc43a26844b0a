#!/usr/bin/env python3
"""FSI time steps per second on one MI355X: FP64 and mixed precision, every workload.

A step is one call of fsi_step: C_f(X^n) re-clipped and reassembled for the current solid
position, the right-hand side, and the right-preconditioned FGMRES solve of the saddle-point
system (block-triangular preconditioner, rtol 1e-8).  Headline workload: 1024 x 1024 P2/P1
fluid (8.4M velocity unknowns) with two disks of radius 0.1 at (0.3, 0.5) and (0.7, 0.5),
75,264 P1 triangles each; u^n ~ U[-1, 1] (seed 3), X^n the reference mesh rotated about
(0.5, 0.5) at 0.1 rad/s (one new position per step); u^{n+1} of each step is u^n of the next.
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line.  `value` is FP64 steps/s at 1024^2.  Beside it:
  mixed      the same time loop with the inner block solves (multigrid V-cycles, mass and
             Schur solves) in FP32 with FP32 accumulation; FP64 operator, Arnoldi process,
             inner Krylov recurrence, residuals and clipping (FSI_FP32);
  fp32_ir    the operator of the Arnoldi process in FP32 as well, with refinement on the FP64
             residual (FSI_FP32_IR);
  inner_forms  the other inner A11 forms at 1024^2, FP64 and mixed: the fixed-cost
             block-diagonal (one application of the MINRES preconditioner) and
             block-triangular (two stationary cycles) forms, and GMRES with the
             block-triangular approximation in the weighted norm;
  coupling_modes  the coupling assembly per call at 1024^2 and 512^2, detected anew
             (FSI_COUPLING_FULL) against the time-coherent form (FSI_COUPLING_INCREMENTAL), for
             three motions between calls: the rotation step of the time loop, a step of 1e-15
             rad (the same intersections, new values) and none;
  step_roofline   algorithmic bytes of a step (model below, from the measured outer and inner
             step counts) against the step time and 8 TB/s;
  configs    the CPU-fast 32^2 case (both preconditioners), the 256^2 ellipse (both
             preconditioners), the 512^2 rotating-disk time loop (100 steps, dt 1e-3; FP64 and
             mixed, and FP64 with the time-coherent coupling), the nonlinear bar at 256^2
             (Newton, the paper's exponential law), and the paper's own element pair (Q2 /
             P1-disc fluid, Q1 solid) on a 256^2 bar with a bending-and-turning motion;
  serving    the 512-request trace in mixed precision and in FP64;
  accuracy   per-run errors against the FP64 oracle (computed in the oracle leg);
  cpu_baseline / cpu_serving  the oracle on the host's cores (bounded samples).
The oracle runs only in the oracle leg, a separate process started at the end.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak
OMEGA = 0.1                # rad/s, prescribed rotation of the solid
CPU_SHARE = 16             # host cores of one GPU's share on the GPU machine (oracle worker pool)


def _f(v, d=6):
    return float(f"{v:.{d}g}") if isinstance(v, float) else v


def _round(obj):
    if isinstance(obj, dict):
        return {k: _round(v) for k, v in obj.items()}
    if isinstance(obj, list):
        return [_round(v) for v in obj]
    return _f(obj)


# ------------------------------------------------------------------------------------------
# algorithmic bytes of one step (model of the kernels the step launches)
# ------------------------------------------------------------------------------------------
def _levels(n, stop):
    out = []
    while n > stop:
        out.append(n)
        n //= 2
    return out, n


def inner_step_bytes(n, prec):
    """Bytes one inner MINRES step must move (one A11 product with the Lanczos and update
    vectors, one application of diag(V, S^{-1})), per kernel of the matrix-free path, with
    w = 8 (FP64) or 4 (FP32 preconditioner):
      velocity V-cycle, per level above the one-launch tail (cells > 16): pre-smoothing 4w N2_l
        (b read, x written, two components), residual + restriction 4w N2_l + 2w N2_{l+1},
        post-smoothing with the coarse correction 6w N2_l + 2w N2_{l+1};
      tail: 4w N2 of its first level + the dense coarsest inverse (162^2 w);
      pressure V-cycle (P1), per level above the 4^2 dense level: first step 3w, one more
        Chebyshev step 5w, residual 3w, restriction w + w coarse, prolongation 2w + w coarse,
        two post steps 10w per node; dense 25^2 w;
      pressure mass solve 13w Np, pressure residual copy (8 + w) Np, output (2w + 16) Np;
      A11 product with the fused MINRES updates (FP64): 64 N2 + 32 Np;
      remaining MINRES vector work: 4 vectors of nf = 2 N2 + Np doubles (the second
        three-term update, 3; the directions and the iterate are formed once per block of
        stored Lanczos vectors, counted in step_bytes);
      FP32 form: the velocity residual converted (24 N2), the finest post-smoothing writes the
        FP64 output ((4w + 16) N2 instead of 6w N2) and reads the FP64 residual for the sums of
        r . z (16 N2)."""
    w = 8 if prec == "fp64" else 4
    N2 = lambda m: (2 * m + 1) ** 2
    Np = lambda m: (m + 1) ** 2
    full, tail = _levels(n, 16)
    b = 0.0
    for k, m in enumerate(full):
        post = 6 * w * N2(m)
        if k == 0 and prec != "fp64":
            post = (4 * w + 16) * N2(m) + 16 * N2(m)
        b += 4 * w * N2(m) + (4 * w * N2(m) + 2 * w * N2(m // 2)) + post + 2 * w * N2(m // 2)
    b += 4 * w * N2(tail) + 162 * 162 * w
    pfull, _ = _levels(n, 4)
    for m in pfull:
        b += 24 * w * Np(m) + 2 * w * Np(m // 2)
    b += 25 * 25 * w
    b += 13 * w * Np(n) + (8 + w) * Np(n) + (2 * w + 16) * Np(n)
    b += 64 * N2(n) + 32 * Np(n)
    b += 4 * 8 * (2 * N2(n) + Np(n))
    if prec != "fp64":
        b += 24 * N2(n)
    return b


def step_bytes(n, Ns, nnz_s, nnz_cf, n_pairs, its, inner_its, restarts, prec, pc, cs_steps=36):
    """Algorithmic bytes of one step (C_f assembly, right-hand side, the outer FGMRES with its
    inner solves), w = 8 for every outer vector:
      C_f: the piece list and 3 x 6 matrices written and read (2 x 152 B per piece), C_f and
        C_f^T written, ranked and read (4 x 12 B per entry);
      g1 = (rho/dt) M_f u^n: the P2 pattern (46 n^2 entries, 12 B) and two components in and out;
      per outer step j: the operator (matrix-free fluid rows 32 N2 + 16 Np, C_f^T and C_f
        entries 12 B each twice, the solid rows 20 B per entry of the solid pattern and 8
        vectors of Ns), A22 by two C_s Chebyshev solves of cs_steps steps (12 B per entry and
        6 vectors of Ns per step) and one A_s product, the block-triangular C_f product, the
        two Gram-Schmidt passes 16 (j + 1) N + 24 N and the normalisation 16 N;
      inner steps: inner_step_bytes each, plus one more preconditioner application per
        outer step (the start of MINRES), and the iterate formed from the stored Lanczos
        vectors (each read once, the iterate written: (inner steps + 1) nf 8 per solve);
      per restart: the update x += Z y ((k + 1) N 8) and the FP64 true residual (operator + 3N 8)."""
    N2, Np = (2 * n + 1) ** 2, (n + 1) ** 2
    N = 2 * N2 + Np + 4 * Ns
    b = 2 * 152 * n_pairs + 4 * 12 * nnz_cf
    b += (46 * n * n) * 12 + 4 * 8 * N2
    op = 32 * N2 + 16 * Np + 2 * 12 * nnz_cf + 20 * nnz_s + 8 * 8 * Ns
    a22 = 2 * cs_steps * (12 * nnz_s + 6 * 8 * Ns) + 12 * nnz_s + 6 * 8 * Ns
    cf = 12 * nnz_cf + 2 * 8 * Ns if pc == "tri" else 0
    m = 30
    for j in range(its):
        jj = j % m
        b += op + a22 + cf + 16 * (jj + 1) * N + 24 * N + 16 * N
    b += inner_its * inner_step_bytes(n, prec)
    b += its * (inner_step_bytes(n, prec) - 64 * N2 - 32 * Np - 4 * 8 * (2 * N2 + Np))
    b += (inner_its + its) * 8 * (2 * N2 + Np)
    b += restarts * ((min(its, m) + 1) * N * 8 + op + 3 * N * 8)
    return b


# ------------------------------------------------------------------------------------------
# the oracle leg (a separate process; the only part of this file that runs the oracle)
# ------------------------------------------------------------------------------------------
def _cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), cpu_model=model)


def _oracle_step(wl, X, u):
    """One oracle step in the paper's phases (one core): T_setup (assembly and the exact block
    factorisations of A11 and A22, once), T_coup (C_f clipping and integration), T_sol
    (GMRES(30) with the exact block-triangular preconditioner to rtol 1e-8).  Returns the
    system, the right-hand side, the solution and the phase record."""
    from oracle import gmres, system
    t0 = time.perf_counter()
    S = system.FSISystem.from_workload(wl)
    t1 = time.perf_counter()
    S.set_position(X)
    t2 = time.perf_counter()
    S._factor()          # A11 and A22 do not depend on X^n: factorised once (setup)
    t3 = time.perf_counter()
    b = S.rhs(u, X)
    A = S.matrix()
    x, info = gmres.gmres(lambda v: A @ v, b, precond=lambda r: S.apply_precond(r, "tri"), restart=30, rtol=1e-8)
    t4 = time.perf_counter()
    ph = dict(T_setup_s=(t1 - t0) + (t3 - t2), T_coup_s=t2 - t1, T_sol_s=t4 - t3, its=info["its"], N=S.lay.N)
    return S, A, b, x, ph


def _errs(S, x, xs):
    """||x - x*|| / ||x*|| over the whole vector and per block (u, mean-free p, X, lam)."""
    import numpy as np
    sl = S.lay.slices()
    w = S.F["p_weights"] if "p_weights" in S.F else np.asarray(S.F["Mp"].sum(axis=1)).ravel()
    mf = lambda p: p - (w @ p) / w.sum()
    cat = lambda v, a, b: np.concatenate([v[sl[a]], v[sl[b]]])
    parts = {"u": (cat(x, "ux", "uy"), cat(xs, "ux", "uy")), "p": (mf(x[sl["p"]]), mf(xs[sl["p"]])),
             "X": (cat(x, "Xx", "Xy"), cat(xs, "Xx", "Xy")), "lam": (cat(x, "lx", "ly"), cat(xs, "lx", "ly"))}
    res = {"all": float(np.linalg.norm(x - xs) / np.linalg.norm(xs))}
    for k, (a, b) in parts.items():
        res[k] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return res


def oracle_leg(args) -> dict:
    """The oracle on the host (one core per solve): the CPU baseline of the headline metric,
    the CPU serving baseline and the accuracy of the GPU results saved by the main process.

    cpu_baseline: one step of the two-disk geometry at 128^2 (the headline geometry with the
      ring count scaled with the grid) in the paper's phases; steps/s = 1 / (T_coup + T_sol),
      scaled to the full workload by the unknown ratio (extrapolated: the exact block solves
      grow faster than linearly, so the scaled rate bounds the CPU from above).
    cpu_serving: the 512-request trace through a first-come first-served pool of 16 oracle
      workers (the host cores of one GPU's share), with per-size service times: one request
      of 32^2 and of 64^2 solved, the 128^2 step above, 256^2 extrapolated by the 64 -> 128
      growth (modelled, not run).
    accuracy: eps = ||x - x*|| / ||x*||, whole vector and per block, of the GPU results at
      32^2 (x* the direct solve) and of the 128^2 two-disk step (x* the oracle's GMRES continued
      to the residual floor from the rtol 1e-8 solution); at 1024^2 the largest residual
      |b_i - (A x)_i| / ||b|| on the oracle's own rows at sampled unknowns."""
    import numpy as np

    from oracle import gmres, sampled, system
    from paper_2301_10041_amd import inputs
    out = {}
    data = np.load(args.accuracy_in) if args.accuracy_in else None
    full = inputs.WORKLOADS[args.workload]
    wl = inputs.WORKLOADS["twodisk128"]
    X = inputs.rotation(wl.solid_mesh()[0], (0.5, 0.5), OMEGA * wl.dt)
    u = inputs.uniform(2 * (2 * wl.n + 1) ** 2, wl.seed)
    S, A, b, x8, ph = _oracle_step(wl, X, u)
    t = ph["T_coup_s"] + ph["T_sol_s"]
    n_full = full.sizes()["N"]
    scale = n_full / ph["N"]
    cb = {"value": 1.0 / (t * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
          "sample": f"one oracle step (C_f clipping, exact-block GMRES(30) to rtol 1e-8, block-triangular) of the "
                    f"two-disk geometry at 128^2 fluid ({ph['N']} unknowns, {ph['its']} its, {t:.2f} s/step "
                    f"after {ph['T_setup_s']:.1f} s of setup), scaled by the unknown ratio {scale:.1f} to "
                    f"{n_full} unknowns (extrapolated)",
          "sample_steps_per_s": 1.0 / t}
    cb.update(ph)
    cb.update(_cpu_info())
    out["cpu_baseline"] = cb
    acc = {}
    if data is not None:
        xs, info = gmres.gmres(lambda v: A @ v, b, precond=lambda r: S.apply_precond(r, "tri"), x0=x8, restart=30,
                               rtol=5e-12, maxit=200)
        acc["twodisk128"] = {k[len("twodisk128_"):]: _errs(S, data[k], xs) for k in data.files
                             if k.startswith("twodisk128_")}
        acc["twodisk128"]["reference"] = f"oracle GMRES to relres {info['relres']:.1e}"
        w32 = inputs.WORKLOADS["disk32"]
        S32 = system.FSISystem.from_workload(w32)
        S32.set_position(S32.xy_ref)
        xs32 = S32.solve_direct(S32.random_rhs(w32.seed))
        acc["disk32"] = {k[len("disk32_"):]: _errs(S32, data[k], xs32) for k in data.files if k.startswith("disk32_")}
        if any(k.startswith("qbar32_") for k in data.files):   # the paper's pair against its direct solve
            from oracle import qpair
            wq = inputs.QWORKLOADS["qbar32"]
            Sq = qpair.QSystem.from_workload(wq)
            Xq = q_position(inputs, wq, Sq.xy_ref, 0)
            Sq.set_position(Xq)
            xq = Sq.solve_direct(Sq.rhs(inputs.uniform(2 * Sq.lay.N2, wq.seed), Xq))
            acc["qbar32"] = {k[len("qbar32_"):]: _errs(Sq, data[k], xq) for k in data.files if k.startswith("qbar32_")}
        if "big_fp64" in data.files:
            wb = inputs.WORKLOADS["twodisk1024"]
            xy, tri = wb.solid_mesh()
            rng = np.random.default_rng(17)
            vel, prs, sol = sampled.sample_rows(wb.n, inputs.rotation(xy, (0.5, 0.5), 0.0), tri, xy.shape[0], rng)
            X0 = inputs.rotation(xy, (0.5, 0.5), 0.0)   # the first step's position, as the GPU leg makes it
            ss = sampled.SampledSystem(wb.n, xy, tri, X0, vel, prs, sol, wb.nu, wb.rho, wb.dt, wb.kappa)
            ub = data["big_u"]
            big = {"rows": 2 * len(vel) + len(prs) + 4 * len(sol)}
            for tag in ("fp64", "mixed", "fp32_ir"):
                if f"big_{tag}" in data.files:
                    res = ss.residual(data[f"big_{tag}"], ub)
                    big[f"sampled_residual_{tag}"] = max(abs(v) for v in res.values()) / float(data["big_bnorm"])
            acc["twodisk1024"] = big
        out["accuracy"] = acc
    if not args.no_cpu_baseline:
        # the paper's element pair: one oracle step of the 32^2 bar in the same phases (setup with
        # the exact block factorisations, clipping and integration, exact-block GMRES to 1e-8)
        from oracle import qpair
        wq = inputs.QWORKLOADS["qbar32"]
        t0 = time.perf_counter()
        Sq = qpair.QSystem.from_workload(wq)
        t1 = time.perf_counter()
        Xq = q_position(inputs, wq, Sq.xy_ref, 0)
        Sq.set_position(Xq)
        t2 = time.perf_counter()
        Sq._factor()
        t3 = time.perf_counter()
        bq = Sq.rhs(inputs.uniform(2 * Sq.lay.N2, wq.seed), Xq)
        Aq = Sq.matrix()
        _, iq = gmres.gmres(lambda v: Aq @ v, bq, precond=lambda r: Sq.apply_precond(r, "tri"), restart=30, rtol=1e-8)
        t4 = time.perf_counter()
        out["cpu_qbar32"] = {"T_setup_s": (t1 - t0) + (t3 - t2), "T_coup_s": t2 - t1, "T_sol_s": t4 - t3,
                             "its": iq["its"], "N": Sq.lay.N, "cores": 1, "kind": "oracle",
                             "sample": "one step of the paper's element pair on the 32^2 bar (qbar32)"}
        trace = inputs.request_trace(args.serve_requests, 200.0, seed=4)
        svc = {}
        for n in (32, 64):
            w = next(q for _, q in trace if q.n == n)
            xy, _ = w.solid_mesh()
            t0 = time.perf_counter()
            _oracle_step(w, xy, inputs.uniform(2 * (2 * n + 1) ** 2, w.seed))
            svc[n] = time.perf_counter() - t0
        svc[128] = ph["T_setup_s"] + t
        svc[256] = svc[128] * (svc[128] / svc[64])
        free = [0.0] * CPU_SHARE
        lat = []
        for ta, w in trace:
            k = min(range(CPU_SHARE), key=lambda i: free[i])
            free[k] = max(ta, free[k]) + svc[w.n]
            lat.append(free[k] - ta)
        lat = np.array(lat)
        out["cpu_serving"] = {"throughput_req_s": len(trace) / (max(free) - trace[0][0]),
                              "p50_ms": float(np.percentile(lat, 50) * 1e3),
                              "p99_ms": float(np.percentile(lat, 99) * 1e3), "workers": CPU_SHARE,
                              "service_s": {str(k): v for k, v in svc.items()}, "kind": "oracle",
                              "sample": "one oracle request (setup, clipping, exact-block GMRES) per grid size 32 and "
                                        "64 solved, 128 from the baseline step, 256 extrapolated (x the 64->128 "
                                        "growth); the trace replayed through a FIFO pool of 16 workers with those "
                                        "service times (modelled)"}
    return out


def run_oracle_leg(workload, accuracy_path, serve_requests, no_cpu_baseline):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-leg", "--workload", workload,
           "--serve-requests", str(serve_requests)]
    if accuracy_path:
        cmd += ["--accuracy-in", accuracy_path]
    if no_cpu_baseline:
        cmd += ["--no-cpu-baseline"]
    print("[bench] oracle leg (cpu baseline and accuracy) ...", file=sys.stderr, flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-800:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


# ------------------------------------------------------------------------------------------
# GPU legs
# ------------------------------------------------------------------------------------------
def recorded_traffic(workload: str, kernel_key: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    record (profiles/traffic.json), or None when the record is for another workload or
    the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[f"{kernel_key}@{workload}"]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def golden_its():
    try:
        return json.load(open(os.path.join(ROOT, "tests", "golden", "its.json")))
    except (OSError, ValueError):
        return {}


def run_serving(count: int, slots: int, prec, per_grid: int = 1) -> dict:
    """Request loop: `count` independent steps arriving by a Poisson process at 200 req/s
    (grid 32..256, disk or ellipse, 216 to 12,150 triangles; request i draws u^n from seed
    1000 + i) in the given precision; HBM budget = free memory - 8 GB."""
    from paper_2301_10041_amd import fsi, inputs, serve

    trace = inputs.request_trace(count, 200.0, seed=4)
    reqs = serve.requests_from_trace(trace)
    srv = serve.Server(max_slots=slots, prec=prec, pc=fsi.PC_TRI, rtol=1e-8, slots_per_grid=per_grid)
    # resident slots sized for the largest solid of the trace, per_grid per grid size, each
    # with a context for every lane of its batches
    warm = [inputs.Workload(f"warm{n}", n, [inputs.Solid(45, (0.5, 0.5), 0.2)], dt=0.01)
            for n in (32, 64, 128, 256) for _ in range(per_grid)]
    srv.prewarm(warm)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    summ = serve.summarize(res)
    out = dict(summ)
    out.update(slots=slots, slots_per_grid=per_grid, max_inflight=srv.max_inflight, evictions=srv.evictions,
               jobs=srv.batches, requests_per_job=round(srv.batched / max(srv.batches, 1), 2),
               lanes={n: srv.lanes(n) for n in (32, 64, 128, 256)},
               budget_gb=round(srv.budget / 2**30, 1), wall_s=round(wall, 3),
               steps_per_s=len(res) / wall, dtype="f64" if prec == fsi.FP64 else "f32+f64",
               trace=f"{count} requests, Poisson 200 req/s, n in {{32,64,128,256}}, m in 6..45")
    srv.close()
    return out


def coupling_modes(fsi, torch, ctx, position, step_angle, calls=10, warmup=2):
    """Milliseconds per fsi_assemble_coupling call in each mode for three motions of the solid
    between calls (position(angle) -> device X); the incremental form's branch counts."""
    out = {}
    for label, dang in (("rotation_step", step_angle), ("same_pieces_step", 1e-15), ("no_motion", 0.0)):
        Xs = [position(dang * k) for k in range(warmup + calls)]
        rec = {}
        for mode, tag in ((fsi.COUPLING_FULL, "full"), (fsi.COUPLING_INCREMENTAL, "incremental")):
            ctx.set_coupling_mode(mode)
            before = ctx.coupling_counts()
            for k in range(warmup):
                ctx.assemble_coupling(Xs[k])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(warmup, warmup + calls):
                ctx.assemble_coupling(Xs[k], sync=False)
            torch.cuda.synchronize()
            rec[f"{tag}_ms"] = round(1e3 * (time.perf_counter() - t0) / calls, 4)
            if mode == fsi.COUPLING_INCREMENTAL:
                after = ctx.coupling_counts()
                rec["incremental_branches"] = {k: after[k] - before[k] for k in after if k != "calls"}
        rec["speedup"] = round(rec["full_ms"] / rec["incremental_ms"], 3)
        out[label] = rec
        print(f"[bench coupling {label}] full {rec['full_ms']:.3f} ms incremental {rec['incremental_ms']:.3f} ms "
              f"{rec['incremental_branches']}", file=sys.stderr, flush=True)
    ctx.set_coupling_mode(fsi.COUPLING_FULL)
    return out


def time_loop(ctx, u0, Xs, N2, opts, warmup, steps, tag, profile=False, keep_first=False):
    """fsi_step over positions Xs (u^{n+1} of each step is u^n of the next); returns the
    timing record and (optionally) the state after the first step."""
    import torch
    u = u0.clone()
    N = ctx.sizes["N"]
    state = torch.zeros(N, dtype=torch.float64, device=u0.device)
    first = None
    for k in range(warmup):
        st = ctx.step(u, Xs[k], state, opts)
        if k == 0 and keep_first:
            first = state.cpu().numpy()
        u.copy_(state[:2 * N2])
        print(f"[bench {tag}] warmup {k}: its={st['its']} inner={st['inner_its']} "
              f"relres={st['relres_true']:.2e} t={st['t_coup'] + st['t_rhs'] + st['t_solve']:.3f}s",
              file=sys.stderr, flush=True)
    if profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(warmup, warmup + steps):
        st = ctx.step(u, Xs[k], state, opts)
        u.copy_(state[:2 * N2])
        stats.append(st)
        print(f"[bench {tag}] step {k}: its={st['its']} inner={st['inner_its']} refin={st['refinements']} "
              f"relres={st['relres_true']:.2e} coup={st['t_coup']:.4f}s solve={st['t_solve']:.3f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt_total = time.perf_counter() - t0
    rec = dict(value=steps / dt_total, ms_per_step=1e3 * dt_total / steps,
               its=[s["its"] for s in stats], inner_its=[s["inner_its"] for s in stats],
               restarts=[s["restarts"] for s in stats],
               relres_true=max(s["relres_true"] for s in stats),
               t_coup_ms=1e3 * sum(s["t_coup"] for s in stats) / len(stats),
               t_solve_ms=1e3 * sum(s["t_solve"] for s in stats) / len(stats))
    if profile:
        prec = opts.prec if opts.prec != 2 else 1
        launches, kern_ms, bpl = ctx.profile_read(prec)
        ctx.profile(False)
        avg_s = kern_ms / max(launches, 1) / 1e3
        rec["kernel"] = dict(launches=launches, avg_us=1e6 * avg_s, bytes_per_launch=bpl,
                             achieved_gbs=bpl / avg_s / 1e9 if launches else 0.0)
    return rec, first


def step_roofline(ctx, n, rec, prec, pc):
    sz = ctx.refresh_sizes()
    its = rec["its"]
    inner = rec["inner_its"]
    rs = rec["restarts"]
    bs = [step_bytes(n, sz["Ns"], sz["nnz_s"], sz["nnz_Cf"], sz["n_pairs"], i, k, r, prec, pc)
          for i, k, r in zip(its, inner, rs)]
    b = sum(bs) / len(bs)
    gbs = b / (rec["ms_per_step"] * 1e-3) / 1e9
    return dict(bytes_per_step=b, achieved_gbs=gbs, peak=HBM_PEAK_GBS, frac=gbs / HBM_PEAK_GBS,
                roofline_ms=b / (HBM_PEAK_GBS * 1e9) * 1e3, ms_per_step=rec["ms_per_step"],
                its_mean=sum(its) / len(its), inner_its_mean=sum(inner) / len(inner))


def config_legs(args, fsi, inputs, torch, dev, save):
    """The other workloads: 32^2 (both preconditioners), 256^2 ellipse (both), 512^2 rotating
    disk time loop (100 steps)."""
    import numpy as np
    gold = golden_its()
    out = {}

    def vec(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    def dirichlet_zeroed(b, n):
        L = 2 * n + 1
        I, J = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
        bnd = ((I == 0) | (J == 0) | (I == 2 * n) | (J == 2 * n)).ravel()
        N2 = L * L
        b = b.copy()
        b[:N2][bnd] = 0.0
        b[N2:2 * N2][bnd] = 0.0
        b[2 * N2] = 0.0
        return b

    for name, reps in (("disk32", 5), ("ellipse256", 3)):
        wl = inputs.WORKLOADS[name]
        xy, tri = wl.solid_mesh()
        ctx = fsi.Context.from_workload(wl)
        N = ctx.sizes["N"]
        ctx.assemble_coupling(vec(np.concatenate([xy[:, 0], xy[:, 1]])))
        b = vec(dirichlet_zeroed(inputs.uniform(N, wl.seed), wl.n))
        rec = {"n": wl.n, "unknowns": N, "solid_triangles": int(tri.shape[0])}
        for pcn in ("diag", "tri"):
            for tag, prec in (("fp64", fsi.FP64), ("mixed", fsi.FP32)):
                opts = fsi.Opts(pc=fsi.PC_TRI if pcn == "tri" else fsi.PC_DIAG, prec=prec, rtol=1e-8)
                x = torch.zeros(N, dtype=torch.float64, device=dev)
                ctx.gmres_solve(b, x, opts)
                ts = []
                for _ in range(reps):
                    x.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = ctx.gmres_solve(b, x, opts)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                ms = 1e3 * sorted(ts)[len(ts) // 2]
                sz = ctx.refresh_sizes()
                bb = step_bytes(wl.n, sz["Ns"], sz["nnz_s"], sz["nnz_Cf"], 0, st["its"], st["inner_its"],
                                st["restarts"], tag, pcn)
                r = dict(its=st["its"], its_oracle=gold.get(name, {}).get(pcn, {}).get("its"),
                         inner_its=st["inner_its"], solve_ms=ms, relres_true=st["relres_true"],
                         alg_gbs=bb / (ms * 1e-3) / 1e9, hbm_frac=bb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
                rec[f"{pcn}_{tag}"] = r
                if name == "disk32":
                    save[f"disk32_{pcn}_{tag}"] = x.cpu().numpy()
                print(f"[bench {name} {pcn} {tag}] its={st['its']} (oracle {r['its_oracle']}) solve={ms:.1f} ms",
                      file=sys.stderr, flush=True)
        ctx.close()
        out[name] = rec
    # the 512^2 time loop: 100 steps of dt 1e-3, prescribed rotation, u^0 = 0
    wl = inputs.WORKLOADS["rotdisk512"]
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    N2 = ctx.sizes["N2"]
    steps = args.loop_steps
    Xs = [vec(np.concatenate(list(inputs.rotation(xy, (0.5, 0.5), OMEGA * k * wl.dt).T))) for k in range(steps + 1)]
    rec = {"n": wl.n, "unknowns": ctx.sizes["N"], "solid_triangles": int(tri.shape[0]), "steps": steps,
           "dt": wl.dt}
    u0 = torch.zeros(2 * N2, dtype=torch.float64, device=dev)
    for tag, prec, cmode in (("fp64", fsi.FP64, fsi.COUPLING_FULL), ("mixed", fsi.FP32, fsi.COUPLING_FULL),
                             ("fp64_incremental", fsi.FP64, fsi.COUPLING_INCREMENTAL)):
        ctx.set_coupling_mode(cmode)
        before = ctx.coupling_counts()
        opts = fsi.Opts(pc=fsi.PC_TRI, prec=prec, rtol=1e-8)
        r, _ = time_loop(ctx, u0, Xs, N2, opts, 1, steps, f"rotdisk512 {tag}")
        rec[tag] = dict(steps_per_s=r["value"], ms_per_step=r["ms_per_step"], t_coup_ms=r["t_coup_ms"],
                        t_sol_ms=r["t_solve_ms"], its_mean=sum(r["its"]) / steps,
                        its_max=max(r["its"]), inner_its_mean=sum(r["inner_its"]) / steps,
                        relres_true_max=r["relres_true"])
        if cmode == fsi.COUPLING_INCREMENTAL:
            after = ctx.coupling_counts()
            rec[tag]["incremental_branches"] = {k: after[k] - before[k] for k in after if k != "calls"}
    ctx.set_coupling_mode(fsi.COUPLING_FULL)
    rec["coupling_modes"] = coupling_modes(
        fsi, torch, ctx, lambda a: vec(np.concatenate(list(inputs.rotation(xy, (0.5, 0.5), a).T))),
        OMEGA * wl.dt)
    ctx.close()
    out["rotdisk512"] = rec
    # the first step of the same loop at 256^2, where the oracle's counts exist
    if "rotdisk256_step0" in gold:
        wl = inputs.WORKLOADS["rotdisk256"]
        xy, _ = wl.solid_mesh()
        ctx = fsi.Context.from_workload(wl)
        X = vec(np.concatenate([xy[:, 0], xy[:, 1]]))
        u0 = torch.zeros(2 * ctx.sizes["N2"], dtype=torch.float64, device=dev)
        s = torch.zeros(ctx.sizes["N"], dtype=torch.float64, device=dev)
        r = {}
        for pcn in ("diag", "tri"):
            for tag, prec in (("fp64", fsi.FP64), ("mixed", fsi.FP32)):
                st = ctx.step(u0, X, s, fsi.Opts(pc=fsi.PC_TRI if pcn == "tri" else fsi.PC_DIAG, prec=prec))
                r[f"{pcn}_{tag}"] = dict(its=st["its"], its_oracle=gold["rotdisk256_step0"][pcn]["its"],
                                         solve_ms=1e3 * st["t_solve"])
        ctx.close()
        out["rotdisk256_step0"] = r
    out["bar256_nonlinear"] = nonlinear_leg(args, fsi, inputs, torch, dev)
    out["qbar256"] = qpair_leg(args, fsi, inputs, torch, dev, save)
    return out


def q_position(inputs, wl, xy, k):
    """The prescribed motion of the paper's-pair bar: bent by 0.02 (non-affine on every
    quadrilateral) and turned about its centre at 0.5 rad/s."""
    return inputs.rotation(inputs.bent(xy, 0.02, 0.4, wl.x0), wl.center, 0.5 * k * wl.dt)


def qpair_leg(args, fsi, inputs, torch, dev, save):
    """The paper's own element pair (Q2 / P1-disc fluid, Q1 solid; fsi_create_q2): a time loop
    of the 256^2 bar (102 x 26 quadrilaterals) with a prescribed bending-and-turning motion,
    block-triangular, FP64 and mixed: T_coup and T_sol per step, outer and inner counts; and
    the 32^2 bar's step saved for the oracle's accuracy check."""
    import numpy as np

    def vec(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    w32 = inputs.QWORKLOADS["qbar32"]
    xy, _ = w32.solid_mesh()
    ctx = fsi.Context.from_workload(w32)
    N = ctx.sizes["N"]
    u = vec(inputs.uniform(2 * ctx.sizes["N2"], w32.seed))
    X = vec(np.concatenate(list(q_position(inputs, w32, xy, 0).T)))
    small = {}
    for tag, prec in (("fp64", fsi.FP64), ("mixed", fsi.FP32)):
        x = torch.zeros(N, dtype=torch.float64, device=dev)
        ctx.step(u, X, x, fsi.Opts(pc=fsi.PC_TRI, prec=prec, rtol=1e-8))
        save[f"qbar32_tri_{tag}"] = x.cpu().numpy()
        ts = []
        for _ in range(3):   # the same step again, timed (beside the oracle's in the oracle leg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.step(u, X, x, fsi.Opts(pc=fsi.PC_TRI, prec=prec, rtol=1e-8))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        small[tag] = dict(step_ms=1e3 * sorted(ts)[1], its=st["its"], t_coup_ms=1e3 * st["t_coup"])
    ctx.close()
    wl = inputs.QWORKLOADS["qbar256"]
    xy, quad = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    N2 = ctx.sizes["N2"]
    steps = args.q_steps
    Xs = [vec(np.concatenate(list(q_position(inputs, wl, xy, k).T))) for k in range(steps + 1)]
    rec = {"n": wl.n, "unknowns": ctx.sizes["N"], "pressure_unknowns": ctx.sizes["Np"],
           "solid_quadrilaterals": int(quad.shape[0]), "steps": steps, "dt": wl.dt}
    u0 = vec(inputs.uniform(2 * N2, wl.seed))
    for tag, prec in (("fp64", fsi.FP64), ("mixed", fsi.FP32)):
        r, _ = time_loop(ctx, u0, Xs, N2, fsi.Opts(pc=fsi.PC_TRI, prec=prec, rtol=1e-8), 1, steps, f"qbar256 {tag}",
                         profile=True)
        rec[tag] = dict(steps_per_s=r["value"], ms_per_step=r["ms_per_step"], t_coup_ms=r["t_coup_ms"],
                        t_sol_ms=r["t_solve_ms"], its_mean=sum(r["its"]) / steps, its_max=max(r["its"]),
                        inner_its_mean=sum(r["inner_its"]) / steps, relres_true_max=r["relres_true"])
        k = r.get("kernel")
        if k and k["launches"]:   # the finest velocity level's class-stencil Chebyshev step (HIP events)
            rec[tag]["roofline"] = dict(
                bound="hbm", kernel="k_q2_stencil (finest velocity level, one Chebyshev step: x, b, d read, d, y "
                                    "written)", launches=k["launches"], avg_us=k["avg_us"],
                bytes_per_launch=k["bytes_per_launch"], achieved=k["achieved_gbs"], peak=HBM_PEAK_GBS,
                unit="GB/s", frac=k["achieved_gbs"] / HBM_PEAK_GBS,
                traffic=recorded_traffic("qbar256", "k_q2_stencil<double>") if prec == fsi.FP64 else None)
    sz = ctx.refresh_sizes()
    rec["pieces"] = sz["n_pairs"]
    rec["nnz_Cf"] = sz["nnz_Cf"]
    rec["qbar32"] = small
    ctx.close()
    return rec


def nonlinear_leg(args, fsi, inputs, torch, dev):
    """The nonlinear solid (the exponential law of the paper's nonlinear test, Newton's method):
    the bar on a 256^2 grid released from a bent position (u^0 = 0), Newton to a 1e-6 residual
    reduction with the Jacobian systems to rtol 1e-8 (Sec. 6), each step's solution the next
    step's initial guess, u^n and X^n; the columns of the paper's nonlinear tables per step: T_coup,
    T_sol (Jacobian solves), Newton iterations and GMRES steps per Newton iteration."""
    import numpy as np
    wl = inputs.WORKLOADS["bar256"]
    xy, tri = wl.solid_mesh()
    ctx = fsi.Context.from_workload(wl)
    ctx.set_law(fsi.LAW_EXP, fsi.GAMMA, fsi.ETA)
    N, N2, Ns = ctx.sizes["N"], ctx.sizes["N2"], ctx.sizes["Ns"]
    off = N - 4 * Ns
    X0 = inputs.bent(xy, 0.04, x0=wl.solids[0].x0)
    rec = {"n": wl.n, "unknowns": N, "solid_triangles": int(tri.shape[0]), "dt": wl.dt, "law": "exp",
           "gamma": fsi.GAMMA, "eta": fsi.ETA, "steps": args.nl_steps}
    for tag, prec in (("fp64", fsi.FP64), ("mixed", fsi.FP32)):
        state = torch.zeros(N, dtype=torch.float64, device=dev)
        state[off:off + Ns] = torch.from_numpy(X0[:, 0]).to(dev)
        state[off + Ns:off + 2 * Ns] = torch.from_numpy(X0[:, 1]).to(dev)
        opts = fsi.Opts(pc=fsi.PC_TRI, prec=prec, rtol=1e-8)
        stats = []
        t0 = None
        for k in range(args.nl_steps + 1):
            if k == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            u = state[:2 * N2].clone()
            X = state[off:off + 2 * Ns].clone()
            st = ctx.newton_step(u, X, state, opts, rtol=1e-6)
            if k >= 1:
                stats.append(st)
            print(f"[bench bar256 {tag}] step {k}: nit={st['nit']} its={st['its_total']} "
                  f"res={st['res'] / max(st['res0'], 1e-300):.1e} coup={st['t_coup']:.4f}s solve={st['t_solve']:.3f}s",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt_total = time.perf_counter() - t0
        nit = sum(s["nit"] for s in stats)
        rec[tag] = dict(steps_per_s=len(stats) / dt_total, ms_per_step=1e3 * dt_total / len(stats),
                        nit_mean=nit / len(stats), its_per_newton=sum(s["its_total"] for s in stats) / max(nit, 1),
                        t_coup_ms=1e3 * sum(s["t_coup"] for s in stats) / len(stats),
                        t_sol_ms=1e3 * sum(s["t_solve"] for s in stats) / max(nit, 1),
                        res_reduction_max=max(s["res"] / max(s["res0"], 1e-300) for s in stats))
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="twodisk1024")
    ap.add_argument("--pc", choices=["tri", "diag"], default="tri")
    ap.add_argument("--loop-steps", type=int, default=100, help="steps of the 512^2 time loop")
    ap.add_argument("--nl-steps", type=int, default=10, help="steps of the nonlinear bar loop")
    ap.add_argument("--q-steps", type=int, default=10, help="steps of the paper's-pair bar loop")
    ap.add_argument("--leg", choices=["qbar256"], default="",
                    help="run only this leg and print its record (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="skip the whole oracle leg")
    ap.add_argument("--oracle-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--accuracy-in", default="", help=argparse.SUPPRESS)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-fixed-cost", action="store_true",
                    help="skip the other inner A11 forms (fixed-cost and inner GMRES)")
    ap.add_argument("--no-ir", action="store_true", help="skip the FP32-refinement leg")
    ap.add_argument("--forms", default="fp64,mixed,fp32_ir",
                    help="headline forms to time (comma list of fp64, mixed, fp32_ir; profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run 3 plain device copies of 2 GiB (counter calibration)")
    args = ap.parse_args()

    if args.oracle_leg:
        print(json.dumps(oracle_leg(args)))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1"}))
        print("bench.py: one GPU only (the multi-GPU partition is a design, not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2301_10041_amd import fsi, inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.leg == "qbar256":
        print(json.dumps(_round(qpair_leg(args, fsi, inputs, torch, dev, {}))), flush=True)
        return
    wl = inputs.WORKLOADS[args.workload]
    xy, tri = wl.solid_mesh()
    t0 = time.perf_counter()
    ctx = fsi.Context(wl.n, xy, tri, nu=wl.nu, rho=wl.rho, dt=wl.dt, kappa=wl.kappa)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    sz = ctx.sizes
    N, N2 = sz["N"], sz["N2"]
    u0 = torch.from_numpy(inputs.uniform(2 * N2, wl.seed)).to(dev)
    total = args.warmup + args.steps
    Xs = []
    for k in range(total):
        X = inputs.rotation(xy, (0.5, 0.5), OMEGA * k * wl.dt)
        Xs.append(torch.from_numpy(np.concatenate([X[:, 0], X[:, 1]])).to(dev))
    pc = fsi.PC_TRI if args.pc == "tri" else fsi.PC_DIAG
    save = {}
    res = {}
    want = set(args.forms.split(","))
    forms = [(t, p) for t, p in (("fp64", fsi.FP64), ("mixed", fsi.FP32), ("fp32_ir", fsi.FP32_IR))
             if t in want and not (t == "fp32_ir" and args.no_ir)]
    assert forms and forms[0][0] == "fp64", "the headline needs the fp64 form"
    for tag, prec in forms:
        opts = fsi.Opts(restart=30, rtol=1e-8, pc=pc, prec=prec)
        rec, first = time_loop(ctx, u0, Xs, N2, opts, args.warmup, args.steps, tag, profile=tag != "fp32_ir",
                               keep_first=True)
        res[tag] = rec
        if first is not None and args.workload == "twodisk1024":
            save[f"big_{tag}"] = first
    if args.workload == "twodisk1024" and "big_fp64" in save:
        # the first step of every form has the same inputs: u^0 and X^0
        b = torch.zeros(N, dtype=torch.float64, device=dev)
        ctx.assemble_coupling(Xs[0])
        ctx.build_rhs(u0, Xs[0], b)
        save["big_u"] = u0.cpu().numpy()
        save["big_bnorm"] = np.array(float(torch.linalg.norm(b)))
        ref = save["big_fp64"]
        for tag in ("mixed", "fp32_ir"):
            if f"big_{tag}" in save:
                res[tag]["vs_fp64_first_step"] = float(np.linalg.norm(save[f"big_{tag}"] - ref) / np.linalg.norm(ref))
        del b
    sroof = {tag: step_roofline(ctx, wl.n, res[tag], "fp64" if tag == "fp64" else "fp32", args.pc)
             for tag in res}
    # the other inner A11 forms, timed the same way; reported beside the method's configuration
    fixed = {}
    if not args.no_fixed_cost:
        for form, mode, cycles in (("fixed_diag", fsi.INNER_FIXED_DIAG, 0), ("fixed_tri_2", fsi.INNER_FIXED_TRI, 2),
                                   ("gmres_tri", fsi.INNER_GMRES, 0)):
            fixed[form] = {}
            for tag, prec in [f for f in forms if f[0] != "fp32_ir"]:
                opts = fsi.Opts(restart=30, rtol=1e-8, pc=pc, prec=prec, inner_mode=mode, inner_cycles=cycles)
                r, first = time_loop(ctx, u0, Xs, N2, opts, args.warmup, args.steps, f"{form} {tag}",
                                     keep_first=True)
                rec = dict(value=r["value"], ms_per_step=r["ms_per_step"], its=r["its"],
                           inner_its=r["inner_its"], relres_true=r["relres_true"])
                if "big_fp64" in save and first is not None:
                    rec["vs_fp64_first_step"] = float(np.linalg.norm(first - save["big_fp64"]) /
                                                      np.linalg.norm(save["big_fp64"]))
                fixed[form][tag] = rec
    cmodes = coupling_modes(
        fsi, torch, ctx,
        lambda a: torch.from_numpy(np.concatenate(list(inputs.rotation(xy, (0.5, 0.5), a).T))).to(dev),
        OMEGA * wl.dt)
    ctx.close()
    del Xs, u0
    torch.cuda.empty_cache()
    # the two-disk geometry at 128^2: steps checked against the oracle's direct solve
    wl128 = inputs.WORKLOADS["twodisk128"]
    ctx128 = fsi.Context.from_workload(wl128)
    xy128, _ = wl128.solid_mesh()
    X128 = inputs.rotation(xy128, (0.5, 0.5), OMEGA * wl128.dt)
    X128d = torch.from_numpy(np.concatenate([X128[:, 0], X128[:, 1]])).to(dev)
    u128 = torch.from_numpy(inputs.uniform(2 * ctx128.sizes["N2"], wl128.seed)).to(dev)
    for tag, prec in forms:
        s128 = torch.zeros(ctx128.sizes["N"], dtype=torch.float64, device=dev)
        ctx128.step(u128, X128d, s128, fsi.Opts(pc=pc, prec=prec, rtol=1e-8))
        save[f"twodisk128_{tag}"] = s128.cpu().numpy()
    ctx128.close()

    configs = {} if args.no_configs else config_legs(args, fsi, inputs, torch, dev, save)
    m = res["fp64"]
    k = m["kernel"]
    roofline = {"bound": "hbm", "achieved": round(k["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(k["achieved_gbs"] / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(args.workload, "k_cheb3<double>"),
                "kernel": "k_cheb3<double> (finest-level matrix-free A_f smoothing: the coarse correction added "
                          "while staging x, then the three post-smoothing Chebyshev steps, in one launch)",
                "bytes_per_launch": k["bytes_per_launch"], "avg_us": round(k["avg_us"], 2),
                "launches": k["launches"]}
    out = {
        "metric": "FSI time-steps/s at 1024^2 fluid (FP64 vs mixed) + batched p50/p99 latency",
        "value": _f(m["value"]), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms_per_step"], 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.n}^2 P2/P1 fluid, "
                               f"{len(wl.solids)} disk(s), {sz['Nt']} P1 solid triangles, "
                               f"{N} unknowns, block-{args.pc} FGMRES(30) rtol 1e-8",
                   "n": wl.n, "unknowns": N, "solid_triangles": sz["Nt"], "pc": args.pc,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "step_roofline": dict(sroof, model="bench.step_bytes: per-kernel algorithmic bytes x launches of a step, "
                                           "from the measured outer and inner step counts"),
        "setup_s": round(t_setup, 3),
    }
    for tag, r in res.items():
        out[tag] = _round(r)
    if "mixed" in res:
        out["mixed_speedup"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
    if "fp32_ir" in res:
        out["fp32_ir_speedup"] = round(res["fp32_ir"]["value"] / res["fp64"]["value"], 3)
    if fixed:
        out["inner_forms"] = _round(dict(
            fixed, note="A11^{-1} other than by the inner MINRES: the fixed-cost forms take more outer steps than "
                        "the block inverses (outside the iteration bar), the inner GMRES more inner steps at this "
                        "size; vs_fp64_first_step: distance of the first step's solution from the headline's"))
    out["coupling_modes"] = _round(dict(
        cmodes, note=f"{args.workload}: ms per fsi_assemble_coupling call, detected anew (full) against the "
                     "time-coherent form (incremental: moved triangles re-clipped into kept slots, pattern kept "
                     "when the pieces are), bitwise the same C_f"))
    if configs:
        out["configs"] = _round(configs)
    if not args.no_serve:
        out["serving"] = {"mixed": _round(run_serving(args.serve_requests, args.serve_slots, fsi.FP32)),
                          "fp64": _round(run_serving(args.serve_requests, args.serve_slots, fsi.FP64))}
    if not args.no_oracle:
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "gpu_results.npz")
            np.savez(path, **save)
            leg = run_oracle_leg(args.workload, path, args.serve_requests, args.no_cpu_baseline)
        for key in ("cpu_baseline", "cpu_serving", "accuracy"):
            if key in leg:
                out[key] = _round(leg[key])
        if "cpu_qbar32" in leg and "qbar256" in out.get("configs", {}):   # beside the GPU's 32^2 step
            out["configs"]["qbar256"]["qbar32"]["cpu_oracle"] = _round(leg["cpu_qbar32"])
        if "error" in leg:
            out["oracle_leg_error"] = leg["error"]
    out["step_roofline"] = _round(out["step_roofline"])
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
