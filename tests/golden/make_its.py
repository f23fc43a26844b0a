"""Write tests/golden/its.json: the oracle's outer iteration counts for the evaluation workloads.

Each count is that of the oracle's right-preconditioned GMRES(30) from x0 = 0 to
||b - A x|| <= 1e-8 ||b|| (Sec. 6), with the block-diagonal or block-triangular preconditioner
of Sec. 5 and both diagonal blocks inverted exactly (SuperLU of A11 and A22, the way the paper
inverts them with a direct solver).  "its" counts Arnoldi steps summed over restarts.  These
are the reference counts of the iteration bar its_gpu <= its + max(2, ceil(0.1 its)).

Right-hand sides:
  random   the seeded U[-1, 1] vector of the workload's seed, Dirichlet and pinned rows zeroed
           (the CPU-fast and 256^2 workloads);
  step0    the first step of the prescribed-rotation time loop: u^0 = 0, X^0 the reference
           mesh, b = (0, 0, 0, -(1/dt) C_s X^0) with C_f(X^0) (the rotating disk at 256^2).

Only oracle/ and the shared input generators are called.  Usage (from the repository root):
    python tests/golden/make_its.py [case ...]      (default: every case; merges into the file)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "its.json")

# case -> (workload, right-hand side, preconditioners)
CASES = {
    "disk32": ("disk32", "random", ("diag", "tri")),
    "twodisk128": ("twodisk128", "random", ("diag", "tri")),
    "ellipse256": ("ellipse256", "random", ("diag", "tri")),
    "rotdisk256_step0": ("rotdisk256", "step0", ("diag", "tri")),
}
# The 512^2 rotating disk itself is not a case: SuperLU's factorisation of its A11 (2.4M
# unknowns) ran for more than an hour and past 43 GB of host memory without finishing; the
# same geometry and time step at 256^2 stands in for it.


def run_case(name):
    import numpy as np

    from oracle import gmres, system
    from paper_2301_10041_amd import inputs

    wname, rhs, pcs = CASES[name]
    wl = inputs.WORKLOADS[wname]
    t0 = time.perf_counter()
    S = system.FSISystem.from_workload(wl)
    S.set_position(S.xy_ref)
    if rhs == "random":
        b = S.random_rhs(wl.seed)
    else:
        b = S.rhs(np.zeros(2 * S.lay.N2), S.xy_ref)
    A = S.matrix()
    S._factor()
    t_setup = time.perf_counter() - t0
    rec = dict(workload=wname, rhs=rhs, N=int(S.lay.N), restart=30, rtol=1e-8, setup_s=round(t_setup, 1))
    for pc in pcs:
        t1 = time.perf_counter()
        _, info = gmres.gmres(lambda v: A @ v, b, precond=lambda r: S.apply_precond(r, pc), restart=30, rtol=1e-8)
        rec[pc] = dict(its=int(info["its"]), restarts=int(info["restarts"]), relres=float(info["relres"]),
                       converged=bool(info["converged"]), solve_s=round(time.perf_counter() - t1, 1))
        print(f"{name} {pc}: its={info['its']} relres={info['relres']:.2e} "
              f"({time.perf_counter() - t1:.1f} s)", flush=True)
    return rec


def main(argv):
    names = argv or list(CASES)
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for name in names:
        data[name] = run_case(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
