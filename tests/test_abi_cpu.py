"""CPU-side checks of the C ABI: the library loads, exports every function
that include/hsd.h declares, and its host-only entry points (defaults,
workspace sizing, argument and cone validation) behave as documented.
No GPU computation is started here."""

import ctypes
import os
import re
from ctypes import byref, c_int64, c_size_t

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(hsd_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1312_3039_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhsd.so is not built (run python -m paper_1312_3039_amd.build)")
    return _lib


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for required in ["hsd_setup", "hsd_solve", "hsd_project_cone", "hsd_batch_setup",
                     "hsd_batch_solve", "hsd_workspace_bytes", "hsd_iterate"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    L = lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in lib.SIGNATURES, f"{name} has no ctypes signature"


def test_default_settings(lib):
    L = lib.load()
    st = lib.HsdSettings()
    L.hsd_default_settings(byref(st))
    assert st.alpha == 1.5 and st.cg_zeta_pow == 1.5
    assert st.eps_pri == st.eps_dual == st.eps_gap == 1e-4
    assert st.max_iters == 10000 and st.check_every == 1 and st.scale == 1
    assert st.precision == 0 and st.lds_matrix == 0 and st.slab_cols == 0


def _csr(m, n, nnz):
    return lib_csr(m, n, nnz)


def lib_csr(m, n, nnz):
    from paper_1312_3039_amd import _lib
    return _lib.HsdCsr(m=m, n=n, nnz=nnz, row_ptr=None, col_idx=None, val=None)


def test_workspace_bytes_and_cone_validation(lib):
    L = lib.load()
    st = lib.HsdSettings()
    L.hsd_default_settings(byref(st))
    K, keep = lib.make_cone({"f": 1, "l": 4, "q": [3, 5], "s": [2], "ep": 1, "ed": 0})
    m = 1 + 4 + 8 + 3 + 3
    nb = c_size_t(0)
    assert L.hsd_workspace_bytes(byref(lib_csr(m, 7, 30)), byref(K), byref(st), byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    # FP32 mode needs more (FP32 copies of the values)
    st.precision = 1
    nb32 = c_size_t(0)
    assert L.hsd_workspace_bytes(byref(lib_csr(m, 7, 30)), byref(K), byref(st), byref(nb32)) == 0
    assert nb32.value >= nb.value
    st.precision = 0
    # cone dimension must equal m
    rc = L.hsd_workspace_bytes(byref(lib_csr(m + 1, 7, 30)), byref(K), byref(st), byref(nb))
    assert rc == lib.ERR_CONE
    assert b"cone dimension" in L.hsd_last_error()
    # bad cone sizes
    K2, keep2 = lib.make_cone({"f": 0, "l": 2, "q": [0], "s": [], "ep": 0, "ed": 0})
    assert L.hsd_workspace_bytes(byref(lib_csr(2, 3, 1)), byref(K2), byref(st), byref(nb)) == lib.ERR_CONE
    K3, keep3 = lib.make_cone({"f": 0, "l": -1, "q": [], "s": [], "ep": 0, "ed": 0})
    assert L.hsd_workspace_bytes(byref(lib_csr(2, 3, 1)), byref(K3), byref(st), byref(nb)) == lib.ERR_CONE


def test_settings_validation(lib):
    L = lib.load()
    K, keep = lib.make_cone({"f": 0, "l": 5, "q": [], "s": [], "ep": 0, "ed": 0})
    nb = c_size_t(0)
    for field, bad in [("alpha", 2.0), ("alpha", 0.0), ("precision", 3), ("block_threads", 96),
                       ("lanes_a", 3), ("check_every", 0), ("team_blocks", -1),
                       ("lds_matrix", 2), ("lds_matrix", -1), ("slab_cols", -2)]:
        st = lib.HsdSettings()
        L.hsd_default_settings(byref(st))
        setattr(st, field, bad)
        assert L.hsd_workspace_bytes(byref(lib_csr(5, 2, 4)), byref(K), byref(st), byref(nb)) == lib.ERR_ARG, field


def test_batch_workspace_validation(lib):
    L = lib.load()
    st = lib.HsdSettings()
    L.hsd_default_settings(byref(st))
    cones = [lib.make_cone({"f": 0, "l": 6, "q": [], "s": [], "ep": 0, "ed": 0}),
             lib.make_cone({"f": 0, "l": 3, "q": [3], "s": [], "ep": 0, "ed": 0})]
    Ks = (lib.HsdCone * 2)(*[c[0] for c in cones])
    ro = (c_int64 * 3)(0, 6, 12)
    co = (c_int64 * 3)(0, 2, 5)
    nb = c_size_t(0)
    assert L.hsd_batch_workspace_bytes(2, byref(lib_csr(12, 5, 20)), ro, co, Ks, byref(st), byref(nb)) == 0
    assert nb.value > 0
    bad_ro = (c_int64 * 3)(0, 5, 12)    # program 0 would have 5 rows, its cone has 6
    assert L.hsd_batch_workspace_bytes(2, byref(lib_csr(12, 5, 20)), bad_ro, co, Ks, byref(st),
                                       byref(nb)) == lib.ERR_CONE
    bad_end = (c_int64 * 3)(0, 6, 11)
    assert L.hsd_batch_workspace_bytes(2, byref(lib_csr(12, 5, 20)), bad_end, co, Ks, byref(st),
                                       byref(nb)) == lib.ERR_ARG


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1312_3039_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.load()


def test_power_cone_validation(lib):
    """Power-cone parameters (Sect. 6.1): one triple each, |p| <= 1; a
    parameter outside [-1, 1] or a null array is rejected on the host."""
    L = lib.load()
    st = lib.HsdSettings()
    L.hsd_default_settings(byref(st))
    nb = c_size_t(0)
    K, keep = lib.make_cone({"f": 0, "l": 2, "q": [], "s": [], "ep": 0, "ed": 0, "p": [0.3, -0.7, 1.0]})
    assert L.hsd_workspace_bytes(byref(lib_csr(11, 3, 5)), byref(K), byref(st), byref(nb)) == 0
    assert L.hsd_workspace_bytes(byref(lib_csr(10, 3, 5)), byref(K), byref(st), byref(nb)) == lib.ERR_CONE
    for bad in ([1.5], [-1.01], [float("nan")]):
        Kb, kb = lib.make_cone({"f": 0, "l": 2, "q": [], "s": [], "ep": 0, "ed": 0, "p": bad})
        assert L.hsd_workspace_bytes(byref(lib_csr(5, 3, 5)), byref(Kb), byref(st), byref(nb)) == lib.ERR_CONE
        assert b"power-cone parameter" in L.hsd_last_error()
    Kn, kn = lib.make_cone({"f": 0, "l": 2, "q": [], "s": [], "ep": 0, "ed": 0, "p": [0.5]})
    Kn.p = None
    assert L.hsd_workspace_bytes(byref(lib_csr(5, 3, 5)), byref(Kn), byref(st), byref(nb)) == lib.ERR_ARG


def test_state_calls_reject_null_handle(lib):
    L = lib.load()
    k = ctypes.c_int32(0)
    assert L.hsd_get_state(None, None, None, None, None, byref(k)) == lib.ERR_STATE
    assert L.hsd_set_state(None, None, None, None, None, 0) == lib.ERR_STATE
    assert L.hsd_update_bc(None, None, None) == lib.ERR_STATE
