"""ctypes binding of libfsi (include/fsi.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch tensors to device
pointers, host arrays to C arrays, and status codes to exceptions.  It raises
``FsiLibraryMissing`` when libfsi.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsi.so")

FSI_OK, FSI_E_ARG, FSI_E_MESH, FSI_E_NOMEM, FSI_E_NOCONV, FSI_E_NONFINITE, FSI_E_HIP, \
    FSI_E_CAPACITY, FSI_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32, FP32_IR = 0, 1, 2
PC_DIAG, PC_TRI = 0, 1
# inner A11 modes (fsi_inner): MINRES with the block-diagonal approximation (default), the
# fixed-cost block-diagonal and block-triangular forms, GMRES with the block-triangular one
INNER_MINRES, INNER_FIXED_DIAG, INNER_FIXED_TRI, INNER_GMRES = 0, 1, 2, 3
COUPLING_FULL, COUPLING_INCREMENTAL = 0, 1
CHECK_AUTO, CHECK_EVERY_STEP, CHECK_LAGGED = 0, 1, 2
SMOOTH_CSR, SMOOTH_STENCIL = 0, 1
MAX_LANES = 32                 # FSI_MAX_LANES: systems per fsi_step_batch
COUPLING_SCRATCH_BYTES = 32 << 20   # FSI_COUPLING_SCRATCH_BYTES
BLOCKS = dict(AF=0, MF=1, B=2, BT=3, AS=4, CS=5, CF=6, CFT=7, MP=8, KT=9)
LAW_LINEAR, LAW_EXP = 0, 1
GAMMA, ETA = 1.333, 9.242      # the exponential law of the nonlinear test


class FsiLibraryMissing(RuntimeError):
    pass


class FsiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfsi error {code}: {msg}")
        self.code = code


class FluidDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("nu", C.c_double), ("rho", C.c_double), ("dt", C.c_double)]


class SolidDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tris", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("tri", C.POINTER(C.c_int32)), ("kappa", C.c_double)]


class Sizes(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("N2", "Np", "Ns", "Nt", "N", "off_ux", "off_uy", "off_p",
                                          "off_Xx", "off_Xy", "off_lx", "off_ly", "nnz_Af", "nnz_B",
                                          "nnz_s", "nnz_Cf", "n_pairs", "device_bytes")] + \
              [("mg_levels_u", C.c_int32), ("mg_levels_p", C.c_int32)]


class CouplingInfo(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("nnz", C.c_int64)]


class CouplingCounts(C.Structure):
    _fields_ = [("calls", C.c_int64), ("rebuilds", C.c_int64), ("pattern_builds", C.c_int64),
                ("value_refills", C.c_int64), ("unchanged", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("rtol", C.c_double), ("pc", C.c_int32),
                ("prec", C.c_int32), ("inner_rtol", C.c_double), ("inner_maxit", C.c_int32),
                ("cycle_rtol", C.c_double), ("inner_mode", C.c_int32),
                ("inner_cycles", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("its", C.c_int32), ("restarts", C.c_int32), ("inner_its", C.c_int64),
                ("converged", C.c_int32), ("refinements", C.c_int32), ("relres_true", C.c_double),
                ("relres_est", C.c_double), ("t_coup", C.c_double), ("t_rhs", C.c_double),
                ("t_solve", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32)]


class NewtonStats(C.Structure):
    _fields_ = [("nit", C.c_int32), ("converged", C.c_int32), ("its_total", C.c_int32), ("inner_its", C.c_int64),
                ("res0", C.c_double), ("res", C.c_double), ("t_coup", C.c_double), ("t_res", C.c_double),
                ("t_solve", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "fsi_create": (C.c_int, [C.POINTER(FluidDesc), C.POINTER(SolidDesc), C.c_void_p, C.c_size_t,
                             C.POINTER(C.c_void_p)]),
    "fsi_create_q2": (C.c_int, [C.POINTER(FluidDesc), C.POINTER(SolidDesc), C.c_void_p, C.c_size_t,
                                C.POINTER(C.c_void_p)]),
    "fsi_destroy": (None, [C.c_void_p]),
    "fsi_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fsi_set_solid": (C.c_int, [C.c_void_p, C.POINTER(SolidDesc)]),
    "fsi_set_smoother": (C.c_int, [C.c_void_p, C.c_int]),
    "fsi_set_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "fsi_set_inner_check": (C.c_int, [C.c_void_p, C.c_int]),
    "fsi_footprint": (C.c_int, [C.POINTER(FluidDesc), C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "fsi_sizes": (C.c_int, [C.c_void_p, C.POINTER(Sizes)]),
    "fsi_assemble_coupling": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(CouplingInfo)]),
    "fsi_assemble_coupling_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(CouplingInfo)]),
    "fsi_build_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsi_apply_operator": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "fsi_apply_precond": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "fsi_set_inner": (C.c_int, [C.c_void_p, C.c_double, C.c_int32]),
    "fsi_set_inner_mode": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fsi_set_coupling_mode": (C.c_int, [C.c_void_p, C.c_int]),
    "fsi_get_coupling_counts": (C.c_int, [C.c_void_p, C.POINTER(CouplingCounts)]),
    "fsi_gmres_solve": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                                  C.POINTER(SolveStats)]),
    "fsi_step": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                           C.POINTER(SolveStats)]),
    "fsi_step_batch": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(SolveOpts), C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(SolveStats),
                                 C.POINTER(C.c_int32)]),
    "fsi_set_law": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double]),
    "fsi_solid_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsi_solid_tangent": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fsi_newton_step": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.POINTER(NewtonOpts), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.POINTER(NewtonStats)]),
    "fsi_export_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "fsi_export_csr": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsi_export_lattice": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "fsi_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "fsi_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "fsi_strerror": (C.c_char_p, [C.c_int]),
    "fsi_last_error": (C.c_char_p, [C.c_void_p]),
}


def lib():
    """Load libfsi.so (once).  Raises FsiLibraryMissing if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FsiLibraryMissing(f"{LIB_PATH} not built: run python -m paper_2301_10041_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t, dtype_name="float64"):
    """Device pointer of a contiguous CUDA tensor of the given dtype."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU")
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"expected a contiguous {dtype_name} CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


LAT_AF, LAT_LP, LAT_MP, LAT_BT, LAT_B, LAT_R, LAT_Q2AF = 0, 1, 2, 3, 4, 5, 6
LAT_MAX_ENTRIES = 81


def export_lattice(n, table, nu=1.0, rdt=0.0):
    """Host-only export of a matrix-free coefficient table (see fsi_export_lattice):
    returns (counts[9], offs[9, 81, 2], vals[9, 81, 4]) as numpy arrays."""
    import numpy as np
    counts = np.zeros(9, dtype=np.int32)
    offs = np.zeros((9, LAT_MAX_ENTRIES, 2), dtype=np.int32)
    vals = np.zeros((9, LAT_MAX_ENTRIES, 4), dtype=np.float64)
    rc = lib().fsi_export_lattice(int(n), float(nu), float(rdt), int(table), counts.ctypes.data_as(C.c_void_p),
                                  offs.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise FsiError(rc, lib().fsi_strerror(rc).decode())
    return counts, offs, vals


def footprint(n, n_nodes, n_tris, nu=1.0, rho=1.0, dt=0.01):
    """Device bytes a context of this size would hold (admission estimate)."""
    b = C.c_size_t()
    rc = lib().fsi_footprint(C.byref(FluidDesc(int(n), nu, rho, dt)), int(n_nodes), int(n_tris), C.byref(b))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_footprint")
    return b.value


@dataclass
class Opts:
    restart: int = 30
    maxit: int = 10000
    rtol: float = 1e-8
    pc: int = PC_TRI
    prec: int = FP64
    inner_rtol: float = 0.0
    inner_maxit: int = 0
    cycle_rtol: float = 0.0
    inner_mode: int = 0
    inner_cycles: int = 0

    def c(self):
        return SolveOpts(self.restart, self.maxit, self.rtol, self.pc, self.prec, self.inner_rtol,
                         self.inner_maxit, self.cycle_rtol, self.inner_mode, self.inner_cycles)


def step_batch(ctxs, u_n, X_n, states, opts: Opts | None = None):
    """K independent steps in lockstep (fsi_step_batch): system k is
    ``ctxs[k].step(u_n[k], X_n[k], states[k], opts)``, bitwise, run on ctxs[0]'s stream with
    the inner solves of all systems batched into the same launches.  Returns (stats, rcs):
    per-system statistics dicts and statuses (FSI_OK, FSI_E_NOCONV or FSI_E_NONFINITE).
    Raises FsiError when the batch as a whole fails."""
    K = len(ctxs)
    if K < 1 or K > MAX_LANES or not (len(u_n) == len(X_n) == len(states) == K):
        raise ValueError(f"need 1..{MAX_LANES} contexts and as many vectors of each kind")
    P = C.c_void_p * K
    hs = P(*[c._h.value for c in ctxs])
    us = P(*[_ptr(t).value for t in u_n])
    xs = P(*[_ptr(t).value for t in X_n])
    ss = P(*[_ptr(t).value for t in states])
    st = (SolveStats * K)()
    rcs = (C.c_int32 * K)()
    o = (opts or Opts()).c()
    rc = lib().fsi_step_batch(K, hs, C.byref(o), us, xs, ss, st, rcs)
    if rc != FSI_OK and not any(r != FSI_OK for r in rcs):
        raise FsiError(rc, lib().fsi_last_error(ctxs[0]._h).decode())
    return [st[k].as_dict() for k in range(K)], [int(r) for r in rcs]


# element pairs (fsi_pair)
PAIR_P2P1, PAIR_Q2P1DISC = 0, 1


class Context:
    """One fluid grid, one solid mesh and all device state of libfsi."""

    def __init__(self, n, xy, tri, nu=1.0, rho=1.0, dt=0.01, kappa=10.0, stream=None, budget=0, pair=PAIR_P2P1):
        """``pair`` PAIR_P2P1: P2/P1 fluid, ``tri`` [Nt, 3] triangles; PAIR_Q2P1DISC: the paper's
        Q2 / P1-disc fluid, ``tri`` [Nq, 4] quadrilaterals of the Q1 solid (fsi_create_q2)."""
        L = lib()
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
        if xy.ndim != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be [Ns, 2]")
        nv = 4 if pair == PAIR_Q2P1DISC else 3
        self._xy_soa = np.ascontiguousarray(np.concatenate([xy[:, 0], xy[:, 1]]))
        self._tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1))
        if self._tri.size % nv:
            raise ValueError(f"the solid elements need {nv} nodes each")
        fd = FluidDesc(int(n), float(nu), float(rho), float(dt))
        sd = SolidDesc(xy.shape[0], self._tri.size // nv,
                       self._xy_soa.ctypes.data_as(C.POINTER(C.c_double)),
                       self._tri.ctypes.data_as(C.POINTER(C.c_int32)), float(kappa))
        h = C.c_void_p()
        create = L.fsi_create_q2 if pair == PAIR_Q2P1DISC else L.fsi_create
        rc = create(C.byref(fd), C.byref(sd), _stream_handle(stream), int(budget), C.byref(h))
        if rc != FSI_OK:
            raise FsiError(rc, L.fsi_last_error(None).decode())
        self._h = h
        self.pair = pair
        self.n, self.nu, self.rho, self.dt, self.kappa = int(n), nu, rho, dt, kappa
        self.sizes = self._sizes()

    @classmethod
    def from_workload(cls, wl, **kw):
        """A context of an ``inputs.Workload`` (triangle pair) or ``inputs.QWorkload`` (the paper's
        Q2 / P1-disc pair with a Q1 solid)."""
        xy, tri = wl.solid_mesh()
        if np.asarray(tri).shape[-1] == 4:
            kw.setdefault("pair", PAIR_Q2P1DISC)
        return cls(wl.n, xy, tri, nu=wl.nu, rho=wl.rho, dt=wl.dt, kappa=wl.kappa, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().fsi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != FSI_OK:
            raise FsiError(rc, lib().fsi_last_error(self._h).decode())

    def _sizes(self):
        s = Sizes()
        self._check(lib().fsi_sizes(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Sizes._fields_}

    def refresh_sizes(self):
        self.sizes = self._sizes()
        return self.sizes

    def set_solid(self, xy, tri, kappa=None):
        """Replace the solid mesh (keeps fluid blocks; buffers only grow)."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
        self._xy_soa = np.ascontiguousarray(np.concatenate([xy[:, 0], xy[:, 1]]))
        self._tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1))
        k = self.kappa if kappa is None else float(kappa)
        sd = SolidDesc(xy.shape[0], self._tri.size // 3,
                       self._xy_soa.ctypes.data_as(C.POINTER(C.c_double)),
                       self._tri.ctypes.data_as(C.POINTER(C.c_int32)), k)
        self._check(lib().fsi_set_solid(self._h, C.byref(sd)))
        self.kappa = k
        self.sizes = self._sizes()

    def set_stream(self, stream=None):
        self._check(lib().fsi_set_stream(self._h, _stream_handle(stream)))

    def assemble_coupling(self, Xn, sync=True):
        info = CouplingInfo()
        self._check(lib().fsi_assemble_coupling(self._h, _ptr(Xn), C.byref(info) if sync else None))
        return dict(n_pairs=info.n_pairs, nnz=info.nnz)

    def assemble_coupling_noalloc(self, Xn, sync=True):
        """fsi_assemble_coupling_noalloc: the same C_f with no device allocation (work space in the
        library's per-GPU static array; overlapping calls on one GPU race)."""
        info = CouplingInfo()
        self._check(lib().fsi_assemble_coupling_noalloc(self._h, _ptr(Xn), C.byref(info) if sync else None))
        return dict(n_pairs=info.n_pairs, nnz=info.nnz)

    def set_coupling_mode(self, mode):
        """COUPLING_FULL (detect anew every call) or COUPLING_INCREMENTAL (re-clip the moved
        triangles into kept slots; bitwise the same C_f)."""
        self._check(lib().fsi_set_coupling_mode(self._h, int(mode)))

    def coupling_counts(self):
        cc = CouplingCounts()
        self._check(lib().fsi_get_coupling_counts(self._h, C.byref(cc)))
        return {k: getattr(cc, k) for k, _ in CouplingCounts._fields_}

    def build_rhs(self, u_n, X_n, b):
        self._check(lib().fsi_build_rhs(self._h, _ptr(u_n), _ptr(X_n), _ptr(b)))

    def apply_operator(self, x, y, prec=FP64):
        self._check(lib().fsi_apply_operator(self._h, int(prec), _ptr(x), _ptr(y)))

    def apply_precond(self, r, z, pc=PC_TRI, prec=FP64):
        self._check(lib().fsi_apply_precond(self._h, int(pc), int(prec), _ptr(r), _ptr(z)))

    def set_smoother(self, kind):
        self._check(lib().fsi_set_smoother(self._h, int(kind)))

    def set_graphs(self, enable=True):
        self._check(lib().fsi_set_graphs(self._h, 1 if enable else 0))

    def set_inner_check(self, mode):
        """CHECK_AUTO, CHECK_EVERY_STEP or CHECK_LAGGED: when the inner MINRES solve learns
        that it has converged (the same results in every mode)."""
        self._check(lib().fsi_set_inner_check(self._h, int(mode)))

    def set_inner(self, rtol, maxit=0):
        self._check(lib().fsi_set_inner(self._h, float(rtol), int(maxit)))

    def set_inner_mode(self, mode, cycles=0):
        """The context's inner A11 mode (INNER_*) for apply_precond; solves take theirs from Opts."""
        self._check(lib().fsi_set_inner_mode(self._h, int(mode), int(cycles)))

    def gmres_solve(self, b, x, opts: Opts | None = None, raise_noconv=True):
        st = SolveStats()
        o = (opts or Opts()).c()
        rc = lib().fsi_gmres_solve(self._h, C.byref(o), _ptr(b), _ptr(x), C.byref(st))
        if rc != FSI_OK and (raise_noconv or rc != FSI_E_NOCONV):
            self._check(rc)
        return st.as_dict()

    def step(self, u_n, X_n, state, opts: Opts | None = None):
        st = SolveStats()
        o = (opts or Opts()).c()
        self._check(lib().fsi_step(self._h, C.byref(o), _ptr(u_n), _ptr(X_n), _ptr(state), C.byref(st)))
        return st.as_dict()

    def set_law(self, law, gamma=GAMMA, eta=ETA):
        """Solid law: LAW_LINEAR (P = kappa F) or LAW_EXP (the exponential law of the nonlinear test)."""
        self._check(lib().fsi_set_law(self._h, int(law), float(gamma), float(eta)))

    def solid_residual(self, X, R):
        """R(X) of the context's law (X, R: device 2 Ns)."""
        self._check(lib().fsi_solid_residual(self._h, _ptr(X), _ptr(R)))

    def solid_tangent(self, X=None):
        """Use the tangent K(X) in place of A_s (None: back to A_s)."""
        self._check(lib().fsi_solid_tangent(self._h, None if X is None else _ptr(X)))

    def newton_step(self, u_n, X_n, state, opts: Opts | None = None, rtol=1e-6, maxit=50, f_X=None,
                    raise_noconv=True):
        """One Newton step (fsi_newton_step); state holds the initial guess on entry."""
        st = NewtonStats()
        o = (opts or Opts()).c()
        no = NewtonOpts(float(rtol), int(maxit))
        rc = lib().fsi_newton_step(self._h, C.byref(o), C.byref(no), _ptr(u_n), _ptr(X_n),
                                   None if f_X is None else _ptr(f_X), _ptr(state), C.byref(st))
        if rc != FSI_OK and (raise_noconv or rc != FSI_E_NOCONV):
            self._check(rc)
        return st.as_dict()

    def profile(self, enable=True):
        self._check(lib().fsi_profile(self._h, 1 if enable else 0))

    def profile_read(self, prec=FP64):
        """(launches, total_ms, algorithmic bytes per launch) of the dominant kernel."""
        n, t, b = C.c_int64(), C.c_double(), C.c_double()
        self._check(lib().fsi_profile_read(self._h, int(prec), C.byref(n), C.byref(t), C.byref(b)))
        return n.value, t.value, b.value

    def export_pairs(self):
        cnt = C.c_int64()
        self._check(lib().fsi_export_pairs(self._h, None, None, 0, C.byref(cnt)))
        E = np.zeros(cnt.value, dtype=np.int32)
        T = np.zeros(cnt.value, dtype=np.int32)
        self._check(lib().fsi_export_pairs(self._h, E.ctypes.data_as(C.c_void_p),
                                           T.ctypes.data_as(C.c_void_p), cnt.value, C.byref(cnt)))
        return E, T

    def export_csr(self, block):
        """(rowptr, col, val[nnz, width]) host copies of one block."""
        bid = BLOCKS[block] if isinstance(block, str) else int(block)
        nr, nz, w = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(lib().fsi_export_csr(self._h, bid, C.byref(nr), C.byref(nz), C.byref(w), None, None, None))
        rp = np.zeros(nr.value + 1, dtype=np.int32)
        col = np.zeros(max(nz.value, 1), dtype=np.int32)
        val = np.zeros(max(nz.value, 1) * w.value, dtype=np.float64)
        self._check(lib().fsi_export_csr(self._h, bid, C.byref(nr), C.byref(nz), C.byref(w),
                                         rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                                         val.ctypes.data_as(C.c_void_p)))
        return rp, col[:nz.value], val[:nz.value * w.value].reshape(nz.value, w.value)
