"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, and rejects bad input on the host before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    txt = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"\b(djtled_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["djtled_precompute", "djtled_forces", "djtled_step", "djtled_destroy", "djtled_info",
              "djtled_loadset_create", "djtled_loadset_destroy", "djtled_export_constants", "djtled_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2106_14189_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def _mesh(X, conn):
    from paper_2106_14189_amd import _lib as L
    X = np.ascontiguousarray(X, np.float64)
    conn = np.ascontiguousarray(conn, np.int32)
    m = L.djtled_mesh(X.shape[0], conn.shape[0], conn.shape[1],
                      X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return m, (X, conn)


def _call_precompute(m, model=0, variant=0, precision=0, rho=1000.0, formulation=0):
    from paper_2106_14189_amd import _lib as L
    mat = L.djtled_material()
    mat.model = model
    mat.E_uniform, mat.nu_uniform, mat.rho = 3000.0, 0.45, rho
    prm = L.djtled_params(precision, 0.0, 0.9, 0.0, 0, 0, variant, 0, formulation)
    h = ctypes.c_void_p()
    return L.lib.djtled_precompute(ctypes.byref(m), ctypes.byref(mat), ctypes.byref(prm), ctypes.byref(h))


def test_host_validation_errors():
    from paper_2106_14189_amd import _lib as L
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    m, keep = _mesh(X, [[0, 1, 2, 7]])
    assert _call_precompute(m) == L.DJ_ERR_BAD_MESH
    assert "out of range" in L.lib.djtled_last_error().decode()
    m, keep = _mesh(X, [[0, 1, 2, 3]])
    assert _call_precompute(m, model=5) == L.DJ_ERR_UNSUPPORTED
    assert _call_precompute(m, variant=99) == L.DJ_ERR_ARG
    assert _call_precompute(m, precision=7) == L.DJ_ERR_UNSUPPORTED
    assert _call_precompute(m, rho=-1.0) == L.DJ_ERR_ARG
    assert _call_precompute(m, variant=-2) == L.DJ_ERR_ARG
    assert _call_precompute(m, formulation=3) == L.DJ_ERR_ARG
    # the average-nodal-pressure form: neo-Hookean / transversely isotropic, variants 0..3
    assert _call_precompute(m, formulation=L.DJ_FORM_NODAL_PRESSURE, variant=4) == L.DJ_ERR_UNSUPPORTED
    assert "average-nodal-pressure form" in L.lib.djtled_last_error().decode()
    assert _call_precompute(m, formulation=L.DJ_FORM_NODAL_PRESSURE, model=L.DJ_MR) == L.DJ_ERR_UNSUPPORTED
    assert _call_precompute(m, formulation=L.DJ_FORM_CLASSICAL, precision=L.DJ_FP64) == L.DJ_ERR_UNSUPPORTED
    assert "classical TLED form" in L.lib.djtled_last_error().decode()
    assert _call_precompute(m, model=L.DJ_OT) == L.DJ_ERR_ARG  # OT needs both fibre families
    # batches take the Jacobian form only (checked before any device call)
    mat = L.djtled_material()
    mat.E_uniform, mat.nu_uniform, mat.rho = 3000.0, 0.45, 1000.0
    ld = L.djtled_loads()
    prm = L.djtled_params(L.DJ_FP32, 0.0, 0.9, 0.0, 0, 0, 0, 0, L.DJ_FORM_CLASSICAL)
    h = ctypes.c_void_p()
    assert L.lib.djtled_batch_create(1, ctypes.byref(m), ctypes.byref(mat), ctypes.byref(ld), None, ctypes.byref(prm),
                                     None, ctypes.byref(h)) == L.DJ_ERR_UNSUPPORTED
    Xn = X.copy()
    Xn[1, 0] = np.nan
    m, keep = _mesh(Xn, [[0, 1, 2, 3]])
    assert _call_precompute(m) == L.DJ_ERR_BAD_MESH
    assert L.lib.djtled_step(None, None, None, 1, None, None, None) == L.DJ_ERR_ARG
    assert L.lib.djtled_forces(None, None, None, None) == L.DJ_ERR_ARG
