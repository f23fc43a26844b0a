"""The C-ABI library: it loads and exports every entry point that include/fsi.h declares
(no compute call: CPU only); the binding fails loudly when the library is missing."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(fsi_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("fsi_create", "fsi_destroy", "fsi_assemble_coupling", "fsi_apply_operator",
                     "fsi_apply_precond", "fsi_gmres_solve", "fsi_step", "fsi_export_pairs",
                     "fsi_export_csr", "fsi_build_rhs", "fsi_sizes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2301_10041_amd import fsi
    if not os.path.exists(fsi.LIB_PATH):
        pytest.fail("libfsi.so is not built (run python -m paper_2301_10041_amd.build)")
    L = ctypes.CDLL(fsi.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    # the binding's signature table covers the header
    assert set(fsi._SIGS) == set(declared_symbols())


def test_strerror_without_gpu():
    from paper_2301_10041_amd import fsi
    L = fsi.lib()
    assert L.fsi_strerror(fsi.FSI_E_MESH) == b"invalid mesh or solid position"
    assert L.fsi_strerror(12345) == b"unknown status"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2301_10041_amd import fsi
    monkeypatch.setattr(fsi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fsi, "_lib", None)
    with pytest.raises(fsi.FsiLibraryMissing):
        fsi.lib()


def test_null_context_and_bad_arguments_without_gpu():
    """Every entry point that takes a context refuses a null one with FSI_E_ARG before any
    device call; the footprint query refuses impossible sizes."""
    import ctypes as C
    from paper_2301_10041_amd import fsi
    L = fsi.lib()
    assert L.fsi_set_coupling_mode(None, fsi.COUPLING_INCREMENTAL) == fsi.FSI_E_ARG
    assert L.fsi_set_inner_check(None, fsi.CHECK_LAGGED) == fsi.FSI_E_ARG
    assert L.fsi_set_graphs(None, 1) == fsi.FSI_E_ARG
    assert L.fsi_set_inner_mode(None, fsi.INNER_MINRES, 0) == fsi.FSI_E_ARG
    assert L.fsi_get_coupling_counts(None, None) == fsi.FSI_E_ARG
    assert L.fsi_assemble_coupling(None, None, None) == fsi.FSI_E_ARG
    assert L.fsi_assemble_coupling_noalloc(None, None, None) == fsi.FSI_E_ARG
    size = C.c_size_t(0)
    bad = fsi.FluidDesc(1, 1.0, 1.0, 0.01)   # n < 2
    assert L.fsi_footprint(C.byref(bad), 3, 1, C.byref(size)) == fsi.FSI_E_ARG
    # grids of one multigrid level (odd n, also above the size where the velocity levels end
    # on a dense 16^2 level) and of several are estimated; a large odd grid's only level
    # would be its dense coarsest level, far beyond any device (creation refuses it)
    est = {}
    for n in (3, 511, 512, 513, 1024):
        assert L.fsi_footprint(C.byref(fsi.FluidDesc(n, 1.0, 1.0, 0.01)), 100, 150, C.byref(size)) == fsi.FSI_OK
        est[n] = size.value
    assert est[3] < est[512] < est[1024] < (64 << 30)
    assert min(est[511], est[513]) > (1 << 40)
    # both creation entry points refuse missing or impossible descriptors before any device call
    h = C.c_void_p()
    for create in (L.fsi_create, L.fsi_create_q2):
        assert create(None, None, None, 0, C.byref(h)) == fsi.FSI_E_ARG
        assert create(C.byref(bad), None, None, 0, C.byref(h)) == fsi.FSI_E_ARG
        assert create(None, None, None, 0, None) == fsi.FSI_E_ARG
        assert not h.value
