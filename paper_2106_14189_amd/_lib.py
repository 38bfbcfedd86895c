"""ctypes binding of libdjtled.so (argument marshalling only).

Every call goes straight to the C ABI declared in ``include/djtled.h``; the
names are the same.  PyTorch supplies device memory and streams.  There is no
fallback: if the library is missing or fails to load, importing this module
raises.
"""
from __future__ import annotations

import ctypes
import os

# PyTorch bundles its own HIP runtime under the same soname as the system one
# (libamdhip64.so.7); importing torch first makes libdjtled.so bind to that
# single runtime, which then serves both torch tensors and the library.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdjtled.so")

DJ_OK, DJ_CONVERGED = 0, 1
DJ_ERR_ARG, DJ_ERR_BAD_MESH, DJ_ERR_INVERTED, DJ_ERR_NONFINITE = -1, -2, -3, -4
DJ_ERR_UNSUPPORTED, DJ_ERR_UNSTABLE_DT, DJ_ERR_HIP, DJ_ERR_BARRIER = -5, -6, -7, -8
DJ_T4, DJ_H8 = 4, 8
DJ_NH, DJ_TI, DJ_OT, DJ_MR = 0, 1, 2, 3
DJ_FP32, DJ_FP64 = 0, 1
DJ_FORM_JACOBIAN, DJ_FORM_CLASSICAL, DJ_FORM_NODAL_PRESSURE = 0, 1, 2
DJ_RAMP_NONE, DJ_RAMP_LINEAR, DJ_RAMP_SMOOTH = 0, 1, 2
DJ_MODE_FIXED, DJ_MODE_RELAX = 0, 1

ERROR_NAMES = {0: "DJ_OK", 1: "DJ_CONVERGED", -1: "DJ_ERR_ARG", -2: "DJ_ERR_BAD_MESH", -3: "DJ_ERR_INVERTED",
               -4: "DJ_ERR_NONFINITE", -5: "DJ_ERR_UNSUPPORTED", -6: "DJ_ERR_UNSTABLE_DT", -7: "DJ_ERR_HIP",
               -8: "DJ_ERR_BARRIER"}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class djtled_mesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_elems", ctypes.c_int32), ("elem_type", ctypes.c_int32),
                ("X", _dp), ("conn", _ip)]


class djtled_material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("E", _dp), ("nu", _dp), ("E_uniform", ctypes.c_double),
                ("nu_uniform", ctypes.c_double), ("rho", ctypes.c_double), ("eta_ratio", _dp),
                ("eta_ratio_uniform", ctypes.c_double), ("fibre", _dp), ("hg_kappa", ctypes.c_double),
                ("fibre_b", _dp), ("eta_b_ratio", _dp), ("eta_b_ratio_uniform", ctypes.c_double), ("c01", _dp),
                ("c01_uniform", ctypes.c_double)]


class djtled_params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("dt", ctypes.c_double), ("dt_factor", ctypes.c_double),
                ("alpha", ctypes.c_double), ("allow_unstable_dt", ctypes.c_int32), ("chunk_elems", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("device", ctypes.c_int32), ("formulation", ctypes.c_int32)]


class djtled_info_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_elems", ctypes.c_int32), ("elem_type", ctypes.c_int32),
                ("model", ctypes.c_int32), ("precision", ctypes.c_int32), ("dt", ctypes.c_double),
                ("dt_crit", ctypes.c_double), ("alpha", ctypes.c_double), ("n_chunks", ctypes.c_int32),
                ("chunk_elems", ctypes.c_int32), ("n_copies", ctypes.c_int32), ("n_shared_copies", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("bytes_per_step", ctypes.c_double), ("elem_bytes", ctypes.c_double),
                ("mass_total", ctypes.c_double), ("formulation", ctypes.c_int32)]


class djtled_loads(ctypes.Structure):
    _fields_ = [("n_bc", ctypes.c_int32), ("bc_node", _ip), ("bc_mask", _ip), ("bc_target", _dp),
                ("ramp", ctypes.c_int32), ("t_ramp", ctypes.c_double), ("R", _dp)]


class djtled_state(ctypes.Structure):
    _fields_ = [("u_cur", _vp), ("u_prev", _vp), ("step", ctypes.c_int64)]


class djtled_step_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tol", ctypes.c_double), ("check_every", ctypes.c_int32)]


class djtled_status(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("steps_done", ctypes.c_int32), ("error_step", ctypes.c_int64),
                ("error_elem", ctypes.c_int32), ("residual", ctypes.c_double), ("kernel_ms", ctypes.c_double)]


class djtled_tune(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("variant", ctypes.c_int32), ("chunk_elems", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tune_steps", ctypes.c_int32)]


class djtled_batch_info_t(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_kinds", ctypes.c_int32), ("n_items", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("chunk_elems", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("tune_candidates", ctypes.c_int32), ("n_elems", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("bytes_per_step", ctypes.c_double), ("tune_ms", ctypes.c_double), ("error_inst", ctypes.c_int32)]


_fp = ctypes.POINTER(ctypes.c_float)
_u16p = ctypes.POINTER(ctypes.c_uint16)


class djtled_mlp(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("ld_out", ctypes.c_int32), ("W1", _vp), ("b1", _vp), ("W2", _vp), ("b2", _vp), ("W3", _vp),
                ("b3", _vp), ("W1_bf16", _vp), ("W2_bf16", _vp), ("W3_bf16", _vp)]


class djtled_mlp_grads(ctypes.Structure):
    _fields_ = [("W1", _vp), ("b1", _vp), ("W2", _vp), ("b2", _vp), ("W3", _vp), ("b3", _vp)]


EXPORTS = {
    "djtled_precompute": (ctypes.c_int, [ctypes.POINTER(djtled_mesh), ctypes.POINTER(djtled_material),
                                         ctypes.POINTER(djtled_params), ctypes.POINTER(_vp)]),
    "djtled_destroy": (ctypes.c_int, [_vp]),
    "djtled_info": (ctypes.c_int, [_vp, ctypes.POINTER(djtled_info_t)]),
    "djtled_forces": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "djtled_forces_anp": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "djtled_forces_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "djtled_loadset_create": (ctypes.c_int, [_vp, ctypes.POINTER(djtled_loads), ctypes.POINTER(_vp)]),
    "djtled_loadset_destroy": (ctypes.c_int, [_vp]),
    "djtled_step": (ctypes.c_int, [_vp, ctypes.POINTER(djtled_state), _vp, ctypes.c_int32,
                                   ctypes.POINTER(djtled_step_opts), ctypes.POINTER(djtled_status), _vp]),
    "djtled_step_multi": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(djtled_state), ctypes.POINTER(_vp),
                                         ctypes.c_int32, ctypes.POINTER(djtled_step_opts),
                                         ctypes.POINTER(djtled_status), _dp, ctypes.POINTER(ctypes.c_int32), _vp]),
    "djtled_export_constants": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "djtled_last_error": (ctypes.c_char_p, []),
    "djtled_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(djtled_mesh), ctypes.POINTER(djtled_material),
                                           ctypes.POINTER(djtled_loads), _dp, ctypes.POINTER(djtled_params),
                                           ctypes.POINTER(djtled_tune), ctypes.POINTER(_vp)]),
    "djtled_batch_destroy": (ctypes.c_int, [_vp]),
    "djtled_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(djtled_batch_info_t)]),
    "djtled_batch_instance": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(djtled_info_t)]),
    "djtled_batch_run": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(djtled_status), _vp]),
    "djtled_batch_stats": (ctypes.c_int, [_vp, _dp]),
    "djtled_batch_read": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
    "djtled_batch_write": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
    "djtled_batch_reset": (ctypes.c_int, [_vp, _vp]),
    "djtled_mlp_workspace_size": (ctypes.c_int, [ctypes.POINTER(djtled_mlp), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "djtled_mlp_forward": (ctypes.c_int, [ctypes.POINTER(djtled_mlp), ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t,
                                          _vp]),
    "djtled_mlp_loss_grad": (ctypes.c_int, [ctypes.POINTER(djtled_mlp), ctypes.c_int32, _vp, _vp,
                                            ctypes.POINTER(djtled_mlp_grads), ctypes.POINTER(ctypes.c_double), _vp,
                                            ctypes.c_size_t, _vp]),
    "djtled_mlp_adam": (ctypes.c_int, [ctypes.POINTER(djtled_mlp), ctypes.POINTER(djtled_mlp_grads),
                                       ctypes.POINTER(djtled_mlp_grads), ctypes.POINTER(djtled_mlp_grads),
                                       ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       _vp]),
    "djtled_mlp_sync_bf16": (ctypes.c_int, [ctypes.POINTER(djtled_mlp), _vp]),
    "djtled_mlp_gemm_test": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                            ctypes.c_int32, _vp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64,
                                            ctypes.c_int32, _vp]),
    "djtled_mlp_last_error": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libdjtled.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class DJError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        err = lib.djtled_mlp_last_error if where.startswith("djtled_mlp") else lib.djtled_last_error
        msg = err().decode(errors="replace")
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")


def check(code: int, where: str) -> int:
    if code < 0:
        raise DJError(code, where)
    return code
