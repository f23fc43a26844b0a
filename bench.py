#!/usr/bin/env python3
"""FSI time steps per second on one MI355X: FP64 and mixed precision.

A step is one call of fsi_step: C_f(X^n) re-clipped and reassembled for the current
solid position, the right-hand side, and the right-preconditioned FGMRES solve of the
saddle-point system (block-triangular preconditioner, rtol 1e-8).  Default workload:
1024 x 1024 P2/P1 fluid (8.4M velocity unknowns) with two disks of radius 0.1 at
(0.3, 0.5) and (0.7, 0.5), 75,264 P1 triangles each; u^n ~ U[-1, 1] (seed 3), X^n the
reference mesh rotated about (0.5, 0.5) at 0.1 rad/s (one new position per step);
u^{n+1} of each step is u^n of the next (a time loop).
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line.  `value` is FP64 steps/s; the `mixed` object holds the same
measurement with FP32 SpMV and inner solves (FP64 Arnoldi, residuals and clipping).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak
OMEGA = 0.1                # rad/s, prescribed rotation of the solid


def cpu_baseline_leg(workload: str) -> dict:
    """Oracle (FP64, SciPy direct solve) on a bounded sample of the workload's shape,
    single-threaded; scaled by the unknown count to the full workload (the sparse direct
    solve grows faster than linearly, so the scaled rate is an upper bound for the CPU)."""
    import numpy as np

    from oracle import step as ostep
    from oracle import system
    from paper_2301_10041_amd import inputs

    full = inputs.WORKLOADS[workload]
    # same geometry, fluid 128^2 and ring count scaled by the same factor as the grid
    f = full.n // 128
    sample = inputs.Workload(f"{workload}_sample128", 128,
                             [inputs.Solid(max(2, s.m // f), s.center, s.radius, s.semi_axes)
                              for s in full.solids], nu=full.nu, rho=full.rho, kappa=full.kappa,
                             dt=full.dt, seed=full.seed)
    S = system.FSISystem.from_workload(sample)
    lay = S.lay
    u = inputs.uniform(2 * lay.N2, sample.seed)
    steps = 1
    t0 = time.perf_counter()
    for k in range(steps):
        X = inputs.rotation(S.xy_ref, (0.5, 0.5), OMEGA * k * sample.dt)
        ostep.step(S, u, X, solver="direct")
    t = (time.perf_counter() - t0) / steps
    n_full = full.sizes()["N"]
    scale = n_full / lay.N
    return {"value": 1.0 / (t * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} oracle steps (C_f clipping + sparse direct solve) of the same two-disk "
                      f"geometry at 128^2 fluid ({lay.N} unknowns, {t:.2f} s/step), scaled by the "
                      f"unknown ratio {scale:.1f} to {n_full} unknowns",
            "sample_s_per_step": t}


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


def run_cpu_baseline(workload: str):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--workload", workload]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def run_serving(count: int, slots: int, per_grid: int = 1) -> dict:
    """Request loop: `count` independent mixed-precision steps arriving by a Poisson
    process at 200 req/s (grid 32..256, disk or ellipse, 216 to 12,150 triangles; request
    i draws u^n from seed 1000 + i); HBM budget = free memory - 8 GB."""
    from paper_2301_10041_amd import fsi, inputs, serve

    trace = inputs.request_trace(count, 200.0, seed=4)
    reqs = serve.requests_from_trace(trace)
    srv = serve.Server(max_slots=slots, prec=fsi.FP32, pc=fsi.PC_TRI, rtol=1e-8, slots_per_grid=per_grid)
    # resident slots sized for the largest solid of the trace, per_grid per grid size, each
    # with a context for every lane of its batches
    warm = [inputs.Workload(f"warm{n}", n, [inputs.Solid(45, (0.5, 0.5), 0.2)], dt=0.01)
            for n in (32, 64, 128, 256) for _ in range(per_grid)]
    srv.prewarm(warm)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    summ = serve.summarize(res)
    out = {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in summ.items()}
    out.update(slots=slots, slots_per_grid=per_grid, max_inflight=srv.max_inflight, evictions=srv.evictions,
               jobs=srv.batches, requests_per_job=round(srv.batched / max(srv.batches, 1), 2),
               lanes={n: srv.lanes(n) for n in (32, 64, 128, 256)},
               budget_gb=round(srv.budget / 2**30, 1), wall_s=round(wall, 3),
               steps_per_s=float(f"{len(res) / wall:.6g}"), dtype="f32+f64",
               trace="512 requests, Poisson 200 req/s, n in {32,64,128,256}, m in 6..45")
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="twodisk1024")
    ap.add_argument("--prec", choices=["both", "fp64", "fp32"], default="both")
    ap.add_argument("--pc", choices=["tri", "diag"], default="tri")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fixed-cost", action="store_true",
                    help="skip the fixed-cost inexact A11 leg (inner_mode 1)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run 3 plain device copies of 2 GiB (counter calibration)")
    args = ap.parse_args()

    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_leg(args.workload)))
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
    state = torch.zeros(N, dtype=torch.float64, device=dev)
    pc = fsi.PC_TRI if args.pc == "tri" else fsi.PC_DIAG
    precs = {"both": [fsi.FP64, fsi.FP32], "fp64": [fsi.FP64], "fp32": [fsi.FP32]}[args.prec]
    res = {}
    for prec in precs:
        tag = "fp64" if prec == fsi.FP64 else "mixed"
        opts = fsi.Opts(restart=30, rtol=1e-8, pc=pc, prec=prec)
        # time loop: u^{n+1} of each step is u^n of the next (reset per precision)
        u = u0.clone()
        for k in range(args.warmup):
            st = ctx.step(u, Xs[k], state, opts)
            u.copy_(state[:2 * N2])
            print(f"[bench {tag}] warmup {k}: its={st['its']} inner={st['inner_its']} "
                  f"relres={st['relres_true']:.2e} t={st['t_coup'] + st['t_rhs'] + st['t_solve']:.3f}s",
                  file=sys.stderr, flush=True)
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for k in range(args.warmup, total):
            st = ctx.step(u, Xs[k], state, opts)
            u.copy_(state[:2 * N2])
            stats.append(st)
            print(f"[bench {tag}] step {k}: its={st['its']} inner={st['inner_its']} "
                  f"relres={st['relres_true']:.2e} coup={st['t_coup']:.4f}s solve={st['t_solve']:.3f}s",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt_total = time.perf_counter() - t0
        launches, kern_ms, bpl = ctx.profile_read(prec)
        ctx.profile(False)
        avg_s = kern_ms / max(launches, 1) / 1e3
        achieved = bpl / avg_s / 1e9 if launches else 0.0
        res[tag] = dict(
            value=args.steps / dt_total, ms_per_step=1e3 * dt_total / args.steps,
            its=[s["its"] for s in stats], inner_its=[s["inner_its"] for s in stats],
            relres_true=max(s["relres_true"] for s in stats),
            t_coup_ms=1e3 * sum(s["t_coup"] for s in stats) / len(stats),
            t_solve_ms=1e3 * sum(s["t_solve"] for s in stats) / len(stats),
            kernel=dict(launches=launches, avg_us=1e6 * avg_s, bytes_per_launch=bpl,
                        achieved_gbs=achieved))
    # the fixed-cost inexact A11 (inner_mode 1: one application of the inner preconditioner,
    # no inner MINRES), timed the same way; reported beside the method's configuration
    fixed = {}
    if not args.no_fixed_cost:
        for prec in precs:
            tag = "fp64" if prec == fsi.FP64 else "mixed"
            opts = fsi.Opts(restart=30, rtol=1e-8, pc=pc, prec=prec, inner_mode=1)
            u = u0.clone()
            for k in range(args.warmup):
                ctx.step(u, Xs[k], state, opts)
                u.copy_(state[:2 * N2])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stats = []
            for k in range(args.warmup, total):
                st = ctx.step(u, Xs[k], state, opts)
                u.copy_(state[:2 * N2])
                stats.append(st)
                print(f"[bench fixed-cost {tag}] step {k}: its={st['its']} relres={st['relres_true']:.2e} "
                      f"solve={st['t_solve']:.3f}s", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            dt_total = time.perf_counter() - t0
            fixed[tag] = dict(value=float(f"{args.steps / dt_total:.6g}"),
                              ms_per_step=round(1e3 * dt_total / args.steps, 2),
                              its=[s["its"] for s in stats],
                              relres_true=float(f"{max(s['relres_true'] for s in stats):.6g}"))
    main_tag = "fp64" if "fp64" in res else "mixed"
    m = res[main_tag]
    k = m["kernel"]
    roofline = {"bound": "hbm", "achieved": round(k["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(k["achieved_gbs"] / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(args.workload, "k_cheb3<double>")
                if main_tag == "fp64" else None,
                "kernel": ("k_cheb3<%s> (finest-level matrix-free A_f smoothing: the coarse "
                           "correction added while staging x, then the three post-smoothing "
                           "Chebyshev steps, in one launch)"
                           % ("double" if main_tag == "fp64" else "float")),
                "bytes_per_launch": k["bytes_per_launch"], "avg_us": round(k["avg_us"], 2),
                "launches": k["launches"]}
    out = {
        "metric": "FSI time-steps/s at 1024^2 fluid (FP64 vs mixed) + batched p50/p99 latency",
        "value": float(f"{m['value']:.6g}"), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms_per_step"], 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if main_tag == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.n}^2 P2/P1 fluid, "
                               f"{len(wl.solids)} disk(s), {sz['Nt']} P1 solid triangles, "
                               f"{N} unknowns, block-{args.pc} FGMRES(30) rtol 1e-8",
                   "n": wl.n, "unknowns": N, "solid_triangles": sz["Nt"], "pc": args.pc,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "setup_s": round(t_setup, 3),
    }
    for tag, r in res.items():
        out[tag] = {kk: (float(f"{v:.6g}") if isinstance(v, float) else v) for kk, v in r.items()}
    if "fp64" in res and "mixed" in res:
        out["mixed_speedup"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
    if fixed:
        out["fixed_cost_a11"] = dict(fixed, note="A11^{-1} by one application of its preconditioner "
                                                 "(inner_mode 1), no inner MINRES: more outer steps than "
                                                 "with the block inverses, so not the method's configuration")
    ctx.close()
    del state, Xs, u0
    torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = run_serving(args.serve_requests, args.serve_slots)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(args.workload)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
