"""Shared pieces of the GPU parity tests: device tensors, the oracle system for a workload,
and comparison helpers.  The oracle is test infrastructure; the HIP path is reached only
through the C-ABI binding."""
import numpy as np
import scipy.sparse as sp

from oracle import system
from paper_2301_10041_amd import fsi, inputs


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def to_host(t):
    return t.detach().to("cpu").numpy()


def soa(X):
    X = np.asarray(X, dtype=np.float64)
    return np.concatenate([X[:, 0], X[:, 1]])


def make_pair(wl, Xn=None):
    """(oracle system with C_f at X^n, GPU context with C_f at X^n, X^n)."""
    S = system.FSISystem.from_workload(wl)
    X = S.xy_ref if Xn is None else Xn
    S.set_position(X)
    ctx = fsi.Context.from_workload(wl)
    ctx.assemble_coupling(to_dev(soa(X)))
    return S, ctx, X


def csr_from_export(rp, col, val, shape):
    return sp.csr_matrix((val, col, rp), shape=shape)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def small_workloads():
    """Seeded small cases spanning several tiles, ragged sizes and degenerate contacts."""
    return {
        "disk32": (inputs.WORKLOADS["disk32"], None),
        "ellipse16_rot": (inputs.small_workload(16, 5, (0.45, 0.55), semi_axes=(0.25, 0.15)), 0.4),
        "disk8_edge": (inputs.small_workload(8, 3, (0.5, 0.5), 0.25), None),
        # solid triangles of about 8 x 8 cells: the pieces around a solid node span more than
        # 1,024 lattice nodes (the wide-window form of the C_f rows)
        "coarse_disk128": (inputs.small_workload(128, 3, (0.47, 0.52), 0.2), 0.3),
    }
