"""Thin PyTorch-facing wrapper over the DJ-TLED C ABI.

Only marshals arguments: tensors supply device memory (``data_ptr``) and the
current torch stream supplies the HIP stream.  All computation happens in
libdjtled.so.
"""
from __future__ import annotations

import ctypes
import sys
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
                 precision="fp32", dt=0.0, dt_factor=0.9, alpha=0.0, chunk_elems=0, variant=-1, device=0,
                 allow_unstable_dt=False, eta_b_ratio=None, fibre_b=None, c01=None, formulation="jacobian"):
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
        E1 = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (self.n_elems,)))
        E3 = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (self.n_elems, 3)))
        if model in (L.DJ_TI, L.DJ_OT):
            er, fb = E1(eta_ratio), E3(fibre)
            keep += [er, fb]
            mat.eta_ratio, mat.fibre = _dptr(er), _dptr(fb)
        if model == L.DJ_OT:
            er, fb = E1(eta_b_ratio), E3(fibre_b)
            keep += [er, fb]
            mat.eta_b_ratio, mat.fibre_b = _dptr(er), _dptr(fb)
        if model == L.DJ_MR:
            cc = E1(c01)
            keep.append(cc)
            mat.c01 = _dptr(cc)
        self.precision = L.DJ_FP64 if precision in ("fp64", L.DJ_FP64) else L.DJ_FP32
        self.dtype = torch.float64 if self.precision == L.DJ_FP64 else torch.float32
        form = {"jacobian": L.DJ_FORM_JACOBIAN, "classical": L.DJ_FORM_CLASSICAL,
                "nodal_pressure": L.DJ_FORM_NODAL_PRESSURE}.get(formulation, formulation)
        prm = L.djtled_params(self.precision, float(dt), float(dt_factor), float(alpha), int(allow_unstable_dt),
                              int(chunk_elems), int(variant), int(device), int(form))
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

    def __del__(self, _finalizing=sys.is_finalizing):
        # nothing is released while the interpreter shuts down: the HIP
        # runtime may already be torn down by then (close() explicitly)
        if _finalizing():
            return
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

    def forces_anp(self, u: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Internal forces with the average nodal pressure (djtled_forces_anp)."""
        self._check_vec(u, "u")
        if out is None:
            out = torch.empty_like(u)
        self._check_vec(out, "out")
        L.check(L.lib.djtled_forces_anp(self.handle, ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream(stream)), "djtled_forces_anp")
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

    def zeros_multi(self, k: int):
        return torch.zeros((k, self.n_nodes, 3), dtype=self.dtype, device=self.device)

    def step_multi(self, u_cur: torch.Tensor, u_prev: torch.Tensor, n_steps: int, loads=None, step0: int = 0,
                   relax: bool = False, tol: float = 0.0, check_every: int = 1, stream=None,
                   raise_on_error: bool = True):
        """Advance k load cases in one launch: u_cur, u_prev are (k, n_nodes, 3)
        tensors, loads a list of k LoadSets (common ramp) or None.  Returns
        (status, new step index, per-case residuals, case of an error or -1)."""
        if u_cur.dim() != 3 or u_cur.shape != u_prev.shape:
            raise ValueError("u_cur and u_prev must be (k, n_nodes, 3) tensors of one shape")
        k = u_cur.shape[0]
        for t in (u_cur, u_prev):
            if (t.device != self.device or t.dtype != self.dtype or tuple(t.shape[1:]) != (self.n_nodes, 3)
                    or not t.is_contiguous()):
                raise ValueError(f"state must be a contiguous {self.dtype} (k, {self.n_nodes}, 3) tensor")
        st = L.djtled_state(ctypes.c_void_p(u_cur.data_ptr()), ctypes.c_void_p(u_prev.data_ptr()), int(step0))
        lsp = None
        if loads is not None:
            if len(loads) != k:
                raise ValueError("one LoadSet per load case")
            lsp = (ctypes.c_void_p * k)(*[ls.handle for ls in loads])
        opts = L.djtled_step_opts(L.DJ_MODE_RELAX if relax else L.DJ_MODE_FIXED, float(tol), int(check_every))
        out = L.djtled_status()
        res = np.full(k, np.nan)
        ecase = ctypes.c_int32(-1)
        code = L.lib.djtled_step_multi(self.handle, k, ctypes.byref(st), lsp, int(n_steps), ctypes.byref(opts),
                                       ctypes.byref(out), _dptr(res), ctypes.byref(ecase), _stream(stream))
        status = Status(out.code, out.steps_done, out.error_step, out.error_elem, out.residual, out.kernel_ms)
        if code < 0 and raise_on_error:
            raise L.DJError(code, "djtled_step_multi")
        return status, st.step, res, ecase.value

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
    if mat.model in (L.DJ_TI, L.DJ_OT):
        args.update(eta_ratio=mat.eta_ratio, fibre=mat.fibre)
    if mat.model == L.DJ_OT:
        args.update(eta_b_ratio=mat.eta_b_ratio, fibre_b=mat.fibre_b)
    if mat.model == L.DJ_MR:
        args.update(c01=mat.c01)
    args.update(kw)
    return Solver(wl.mesh.X, wl.mesh.conn, mat.E, mat.nu, **args)


@dataclass
class Instance:
    """One mesh + material + load case of a batch (host arrays)."""
    X: np.ndarray
    conn: np.ndarray
    E: object
    nu: object
    model: int = L.DJ_NH
    rho: float = 1000.0
    eta_ratio: object = None
    fibre: object = None
    hg_kappa: float = 0.1
    bc_node: object = None
    bc_mask: object = None
    bc_target: object = None
    ramp: int = L.DJ_RAMP_NONE
    t_ramp: float = 0.0          # seconds; < 0: |t_ramp| steps of the instance's own dt
    alpha: float | None = None


class Batch:
    """Many independent instances advanced by one persistent kernel per run
    (``djtled_batch_*``).  The batch owns every instance's state."""

    def __init__(self, instances, precision="fp32", dt_factor=0.9, alpha=0.0, autotune=False, variant=-1,
                 chunk_elems=0, steps_per_launch=0, use_graph=True, tune_steps=0, device=0,
                 allow_unstable_dt=False):
        torch.cuda.init()
        n = len(instances)
        meshes = (L.djtled_mesh * n)()
        mats = (L.djtled_material * n)()
        loads = (L.djtled_loads * n)()
        keep = []
        self.sizes = []
        al = np.zeros(n)
        for i, ins in enumerate(instances):
            X = np.ascontiguousarray(ins.X, dtype=np.float64)
            conn = np.ascontiguousarray(ins.conn, dtype=np.int32)
            ne_ = conn.shape[1]
            E = np.ascontiguousarray(np.broadcast_to(np.asarray(ins.E, np.float64), (conn.shape[0],)))
            nu = np.ascontiguousarray(np.broadcast_to(np.asarray(ins.nu, np.float64), (conn.shape[0],)))
            keep += [X, conn, E, nu]
            meshes[i] = L.djtled_mesh(X.shape[0], conn.shape[0], ne_, _dptr(X), _iptr(conn))
            m = L.djtled_material()
            m.model, m.E, m.nu, m.rho, m.hg_kappa = ins.model, _dptr(E), _dptr(nu), float(ins.rho), float(ins.hg_kappa)
            if ins.model == L.DJ_TI:
                er = np.ascontiguousarray(np.broadcast_to(np.asarray(ins.eta_ratio, np.float64), (conn.shape[0],)))
                fb = np.ascontiguousarray(np.broadcast_to(np.asarray(ins.fibre, np.float64), (conn.shape[0], 3)))
                keep += [er, fb]
                m.eta_ratio, m.fibre = _dptr(er), _dptr(fb)
            mats[i] = m
            bn = np.ascontiguousarray(ins.bc_node if ins.bc_node is not None else np.zeros(0), dtype=np.int32)
            bm = np.ascontiguousarray(ins.bc_mask if ins.bc_mask is not None else np.zeros(0), dtype=np.int32)
            bt = np.ascontiguousarray(ins.bc_target if ins.bc_target is not None else np.zeros((0, 3)),
                                      dtype=np.float64).reshape(-1, 3)
            keep += [bn, bm, bt]
            loads[i] = L.djtled_loads(len(bn), _iptr(bn), _iptr(bm), _dptr(bt), int(ins.ramp), float(ins.t_ramp), None)
            al[i] = alpha if ins.alpha is None else ins.alpha
            self.sizes.append((X.shape[0], conn.shape[0]))
        self.precision = L.DJ_FP64 if precision in ("fp64", L.DJ_FP64) else L.DJ_FP32
        self.dtype = torch.float64 if self.precision == L.DJ_FP64 else torch.float32
        self.device = torch.device("cuda", device)
        prm = L.djtled_params(self.precision, 0.0, float(dt_factor), float(alpha), int(allow_unstable_dt), 0, 0,
                              int(device))
        tn = L.djtled_tune(int(autotune), int(variant), int(chunk_elems), int(steps_per_launch), int(use_graph),
                           int(tune_steps))
        h = ctypes.c_void_p()
        L.check(L.lib.djtled_batch_create(n, meshes, mats, loads, _dptr(al), ctypes.byref(prm), ctypes.byref(tn),
                                          ctypes.byref(h)), "djtled_batch_create")
        self.handle = h
        self.n = n
        self.step_index = 0
        del keep

    def close(self):
        if getattr(self, "handle", None):
            L.lib.djtled_batch_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # nothing is released while the interpreter shuts down: the HIP
        # runtime may already be torn down by then (close() explicitly)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = L.djtled_batch_info_t()
        L.check(L.lib.djtled_batch_info(self.handle, ctypes.byref(inf)), "djtled_batch_info")
        return {k: getattr(inf, k) for k, _ in L.djtled_batch_info_t._fields_}

    def instance(self, i: int) -> dict:
        inf = L.djtled_info_t()
        L.check(L.lib.djtled_batch_instance(self.handle, int(i), ctypes.byref(inf)), "djtled_batch_instance")
        return {k: getattr(inf, k) for k, _ in L.djtled_info_t._fields_}

    def run(self, n_steps: int, stream=None, raise_on_error: bool = True) -> Status:
        out = L.djtled_status()
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p(None)
        code = L.lib.djtled_batch_run(self.handle, int(n_steps), ctypes.byref(out), s)
        st = Status(out.code, out.steps_done, out.error_step, out.error_elem, out.residual, out.kernel_ms)
        self.step_index += st.steps_done
        if code < 0 and raise_on_error:
            raise L.DJError(code, "djtled_batch_run")
        return st

    def stats(self) -> np.ndarray:
        ms = np.zeros(self.n)
        L.check(L.lib.djtled_batch_stats(self.handle, _dptr(ms)), "djtled_batch_stats")
        return ms

    def read(self, i: int, with_prev: bool = False):
        nn = self.sizes[i][0]
        u = torch.empty((nn, 3), dtype=self.dtype, device=self.device)
        up = torch.empty_like(u) if with_prev else None
        L.check(L.lib.djtled_batch_read(self.handle, int(i), ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(up.data_ptr()) if up is not None else None,
                                        _stream(None)), "djtled_batch_read")
        torch.cuda.current_stream().synchronize()
        return (u, up) if with_prev else u

    def write(self, i: int, u: torch.Tensor, u_prev: torch.Tensor | None = None):
        nn = self.sizes[i][0]
        for t in (u, u_prev):
            if t is not None and (t.dtype != self.dtype or tuple(t.shape) != (nn, 3) or not t.is_contiguous()
                                  or t.device != self.device):
                raise ValueError(f"state must be a contiguous {self.dtype} tensor of shape ({nn}, 3) on {self.device}")
        L.check(L.lib.djtled_batch_write(self.handle, int(i), ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(u_prev.data_ptr()) if u_prev is not None else None,
                                         _stream(None)), "djtled_batch_write")
        torch.cuda.current_stream().synchronize()

    def reset(self):
        L.check(L.lib.djtled_batch_reset(self.handle, _stream(None)), "djtled_batch_reset")
        self.step_index = 0
