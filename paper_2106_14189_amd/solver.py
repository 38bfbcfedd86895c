"""Thin PyTorch-facing wrapper over the DJ-TLED C ABI.

Only marshals arguments: tensors supply device memory (``data_ptr``) and the
current torch stream supplies the HIP stream.  All computation happens in
libdjtled.so.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Status:
    code: int
    steps_done: int
    error_step: int
    error_elem: int
    residual: float
    kernel_ms: float

    @property
    def name(self) -> str:
        return L.ERROR_NAMES.get(self.code, str(self.code))


class LoadSet:
    def __init__(self, solver: "Solver", handle):
        self.solver = solver
        self.handle = handle

    def close(self):
        if self.handle:
            L.check(L.lib.djtled_loadset_destroy(self.handle), "djtled_loadset_destroy")
            self.handle = None


class Solver:
    """One mesh + material + time step on one GPU (``djtled_precompute``)."""

    def __init__(self, X, conn, E, nu, model=L.DJ_NH, rho=1000.0, eta_ratio=None, fibre=None, hg_kappa=0.1,
                 precision="fp32", dt=0.0, dt_factor=0.9, alpha=0.0, chunk_elems=0, variant=0, device=0,
                 allow_unstable_dt=False):
        torch.cuda.init()
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.n_nodes, self.n_elems = self.X.shape[0], self.conn.shape[0]
        ne = self.conn.shape[1]
        mesh = L.djtled_mesh(self.n_nodes, self.n_elems, ne, _dptr(self.X), _iptr(self.conn))
        Ea = np.ascontiguousarray(np.broadcast_to(np.asarray(E, np.float64), (self.n_elems,)))
        nua = np.ascontiguousarray(np.broadcast_to(np.asarray(nu, np.float64), (self.n_elems,)))
        keep = [Ea, nua]
        mat = L.djtled_material()
        mat.model = model
        mat.E, mat.nu = _dptr(Ea), _dptr(nua)
        mat.rho = float(rho)
        mat.hg_kappa = float(hg_kappa)
        if model == L.DJ_TI:
            er = np.ascontiguousarray(np.broadcast_to(np.asarray(eta_ratio, np.float64), (self.n_elems,)))
            fb = np.ascontiguousarray(np.broadcast_to(np.asarray(fibre, np.float64), (self.n_elems, 3)))
            keep += [er, fb]
            mat.eta_ratio, mat.fibre = _dptr(er), _dptr(fb)
        self.precision = L.DJ_FP64 if precision in ("fp64", L.DJ_FP64) else L.DJ_FP32
        self.dtype = torch.float64 if self.precision == L.DJ_FP64 else torch.float32
        prm = L.djtled_params(self.precision, float(dt), float(dt_factor), float(alpha), int(allow_unstable_dt),
                              int(chunk_elems), int(variant), int(device))
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        L.check(L.lib.djtled_precompute(ctypes.byref(mesh), ctypes.byref(mat), ctypes.byref(prm), ctypes.byref(h)),
                "djtled_precompute")
        self.handle = h
        del keep

    def close(self):
        if getattr(self, "handle", None):
            L.lib.djtled_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = L.djtled_info_t()
        L.check(L.lib.djtled_info(self.handle, ctypes.byref(inf)), "djtled_info")
        return {k: getattr(inf, k) for k, _ in L.djtled_info_t._fields_}

    def zeros(self):
        return torch.zeros((self.n_nodes, 3), dtype=self.dtype, device=self.device)

    def _check_vec(self, t: torch.Tensor, name: str):
        if (t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != (self.n_nodes, 3)
                or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape ({self.n_nodes}, 3) "
                             f"on {self.device}")

    def forces(self, u: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._check_vec(u, "u")
        if out is None:
            out = torch.empty_like(u)
        self._check_vec(out, "out")
        L.check(L.lib.djtled_forces(self.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)), "djtled_forces")
        return out

    def loadset(self, bc_node=None, bc_mask=None, bc_target=None, ramp=L.DJ_RAMP_NONE, t_ramp=0.0, R=None):
        bn = np.ascontiguousarray(bc_node if bc_node is not None else np.zeros(0), dtype=np.int32)
        bm = np.ascontiguousarray(bc_mask if bc_mask is not None else np.zeros(0), dtype=np.int32)
        bt = np.ascontiguousarray(bc_target if bc_target is not None else np.zeros((0, 3)), dtype=np.float64)
        bt = bt.reshape(-1, 3)
        if not (len(bn) == len(bm) == len(bt)):
            raise ValueError("bc_node, bc_mask and bc_target must have the same length")
        ld = L.djtled_loads(len(bn), _iptr(bn), _iptr(bm), _dptr(bt), int(ramp), float(t_ramp), None)
        Rn = None
        if R is not None:
            Rn = np.ascontiguousarray(R, dtype=np.float64).reshape(self.n_nodes, 3)
            ld.R = _dptr(Rn)
        h = ctypes.c_void_p()
        L.check(L.lib.djtled_loadset_create(self.handle, ctypes.byref(ld), ctypes.byref(h)), "djtled_loadset_create")
        return LoadSet(self, h)

    def step(self, u_cur: torch.Tensor, u_prev: torch.Tensor, n_steps: int, loads: LoadSet | None = None,
             step0: int = 0, relax: bool = False, tol: float = 0.0, check_every: int = 1, stream=None,
             raise_on_error: bool = True) -> tuple[Status, int]:
        """Advance (u_cur, u_prev) in place by up to n_steps steps; returns (status, new step index)."""
        self._check_vec(u_cur, "u_cur")
        self._check_vec(u_prev, "u_prev")
        st = L.djtled_state(ctypes.c_void_p(u_cur.data_ptr()), ctypes.c_void_p(u_prev.data_ptr()), int(step0))
        opts = L.djtled_step_opts(L.DJ_MODE_RELAX if relax else L.DJ_MODE_FIXED, float(tol), int(check_every))
        out = L.djtled_status()
        code = L.lib.djtled_step(self.handle, ctypes.byref(st), loads.handle if loads else None, int(n_steps),
                                 ctypes.byref(opts), ctypes.byref(out), _stream(stream))
        status = Status(out.code, out.steps_done, out.error_step, out.error_elem, out.residual, out.kernel_ms)
        if code < 0 and raise_on_error:
            raise L.DJError(code, "djtled_step")
        return status, st.step

    def export_constants(self):
        V = np.zeros(self.n_elems)
        ne = self.conn.shape[1]
        B = np.zeros((self.n_elems, 3, ne))
        m = np.zeros(self.n_nodes)
        L.check(L.lib.djtled_export_constants(self.handle, _dptr(V), _dptr(B), _dptr(m)), "djtled_export_constants")
        return V, B, m


def from_workload(wl, **kw) -> Solver:
    """Build a Solver for a workloads.Workload (precision from the workload)."""
    mat = wl.material
    args = dict(model=mat.model, rho=mat.rho, hg_kappa=mat.hg_kappa, precision="fp64" if wl.fp64 else "fp32",
                dt_factor=wl.dt_factor, alpha=wl.alpha)
    if mat.model == L.DJ_TI:
        args.update(eta_ratio=mat.eta_ratio, fibre=mat.fibre)
    args.update(kw)
    return Solver(wl.mesh.X, wl.mesh.conn, mat.E, mat.nu, **args)
