"""DJ-TLED oracle: TEST INFRASTRUCTURE ONLY.

A plain double-precision CPU implementation of the DJ-TLED method
(Zhang, arXiv 2106.14189), written in C (``djtled_oracle.c``) and loaded here
through ctypes.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the GPU library
never does, and shares no code with it.

The element force is Table 3 evaluated literally from the constants of
Algorithm 1 (Appendix B G matrices, Appendix C vectors, Eqs. 37 and 45);
``route=1`` selects the independent classical TLED force (Eq. 4 with Eq. 54).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "djtled_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP (all host cores; timing only, never parity)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

NH, TI, OT, MR = 0, 1, 2, 3
RAMP_NONE, RAMP_LINEAR, RAMP_SMOOTH = 0, 1, 2
OK, CONVERGED, ERR_INVERTED, ERR_NONFINITE = 0, 1, -3, -4


def _build_one(path: str, extra: list, force: bool) -> None:
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", *extra, "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain -O2, single thread (liboracle.so, the
    one the tests use), and the same source with -fopenmp (liboracle_omp.so,
    all host cores, for the CPU timing baseline only)."""
    _build_one(_LIB, [], force)
    _build_one(_LIB_OMP, ["-fopenmp"], force)
    return _LIB


_libs = {}


def _load(omp: bool = False):
    path = _LIB_OMP if omp else _LIB
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.ora_create.restype = P
        lib.ora_create.argtypes = [I, I, I, dp, ip, I, dp, dp, dp, dp, dp, dp, dp, D, D, ip]
        lib.ora_destroy.argtypes = [P]
        lib.ora_dt_crit.restype = D
        lib.ora_dt_crit.argtypes = [P]
        lib.ora_mass.argtypes = [P, dp]
        lib.ora_element_constants.argtypes = [P, I, dp]
        lib.ora_forces.restype = I
        lib.ora_forces.argtypes = [P, dp, dp, I, ip]
        lib.ora_forces_anp.restype = I
        lib.ora_forces_anp.argtypes = [P, dp, dp, ip]
        lib.ora_element_force.argtypes = [P, I, dp, dp, I]
        lib.ora_energy.restype = D
        lib.ora_energy.argtypes = [P, dp]
        lib.ora_jacobian_invariants.argtypes = [dp, dp, dp, dp]
        lib.ora_lame.argtypes = [D, D, dp, dp]
        lib.ora_run.restype = I
        lib.ora_run.argtypes = [P, dp, dp, dp, I, ip, ip, dp, I, D, D, D, ctypes.c_long, I, I, D, I, dp, ip, I]
        lib.ora_threads.restype = I
        lib.ora_threads.argtypes = []
        lib.ora_residual.restype = D
        lib.ora_residual.argtypes = [P, dp, dp, I, ip, ip]
        _libs[path] = lib
    return _libs[path]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def threads(omp: bool = False) -> int:
    """Threads the oracle's element loop uses in the given build."""
    return _load(omp).ora_threads()


def lame(E: float, nu: float):
    """mu, kappa from E, nu (the oracle's own conversion)."""
    lib = _load()
    mu = ctypes.c_double()
    ka = ctypes.c_double()
    lib.ora_lame(E, nu, ctypes.byref(mu), ctypes.byref(ka))
    return mu.value, ka.value


def jacobian_invariants(J0, tJ, a):
    """[I1, I2, I3, I4] by the Jacobian formulations of Table 1."""
    lib = _load()
    out = np.zeros(4)
    lib.ora_jacobian_invariants(_dp(_f64(J0, 9)), _dp(_f64(tJ, 9)), _dp(_f64(a, 3)), _dp(out))
    return out


class Oracle:
    """One mesh + material with Algorithm 1's pre-computation done in FP64."""

    def __init__(self, X, conn, E, nu, model=NH, eta_ratio=None, fibre=None, rho=1000.0, hg_kappa=0.1,
                 eta_b_ratio=None, fibre_b=None, c01=None, omp: bool = False):
        """omp=True loads the all-cores build (same results; CPU timing baseline only)."""
        lib = _load(omp)
        self.X = _f64(X)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.ne = self.conn.shape[1]
        self.n_nodes = self.X.shape[0]
        self.n_elems = self.conn.shape[0]
        E = np.broadcast_to(np.asarray(E, dtype=np.float64), (self.n_elems,))
        nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (self.n_elems,))
        self._E = _f64(E)
        self._nu = _f64(nu)
        self.model = model
        per = lambda v, shape: _f64(np.broadcast_to(np.asarray(v, dtype=np.float64), shape))  # noqa: E731
        etap = fibp = etabp = fibbp = c01p = None
        if model in (TI, OT):
            self._eta, self._fib = per(eta_ratio, (self.n_elems,)), per(fibre, (self.n_elems, 3))
            etap, fibp = _dp(self._eta), _dp(self._fib)
        if model == OT:
            self._etab, self._fibb = per(eta_b_ratio, (self.n_elems,)), per(fibre_b, (self.n_elems, 3))
            etabp, fibbp = _dp(self._etab), _dp(self._fibb)
        if model == MR:
            self._c01 = per(c01, (self.n_elems,))
            c01p = _dp(self._c01)
        err = ctypes.c_int(0)
        self._ctx = lib.ora_create(self.ne, self.n_nodes, self.n_elems, _dp(self.X), _ip(self.conn), model,
                                   _dp(self._E), _dp(self._nu), etap, fibp, etabp, fibbp, c01p, float(rho),
                                   float(hg_kappa), ctypes.byref(err))
        if not self._ctx:
            raise ValueError(f"oracle rejected the mesh/material (code {err.value})")
        self.rho = rho
        self._lib = lib

    def __del__(self):
        if getattr(self, "_ctx", None):
            self._lib.ora_destroy(self._ctx)
            self._ctx = None

    @property
    def dt_crit(self) -> float:
        return self._lib.ora_dt_crit(self._ctx)

    def mass(self):
        m = np.zeros(self.n_nodes)
        self._lib.ora_mass(self._ctx, _dp(m))
        return m

    def element_constants(self, e: int) -> dict:
        ne = self.ne
        out = np.zeros(9 + 2 + 9 + 6 + 9 + 6 + 3 * ne + 4 + 32)
        self._lib.ora_element_constants(self._ctx, int(e), _dp(out))
        o = 0

        def take(n, shape=None):
            nonlocal o
            v = out[o:o + n].copy()
            o += n
            return v.reshape(shape) if shape else v

        d = {}
        d["J0"] = take(9, (3, 3))
        d["detJ0"] = take(1)[0]
        d["V"] = take(1)[0]
        d["I1m"] = take(9, (3, 3))
        d["m1"] = take(6)
        d["I4m"] = take(9, (3, 3))
        d["m4"] = take(6)
        d["dhdX"] = take(3 * ne, (3, ne))
        d["mu"], d["kappa"], d["eta"] = take(3)
        d["khg"] = take(1)[0]
        d["gamma"] = take(32, (4, 8))
        return d

    def forces(self, u, route: int = 0):
        u = _f64(u, (self.n_nodes, 3))
        f = np.zeros((self.n_nodes, 3))
        bad = ctypes.c_int(-1)
        rc = self._lib.ora_forces(self._ctx, _dp(u), _dp(f), int(route), ctypes.byref(bad))
        if rc != 0:
            raise FloatingPointError(f"element {bad.value} inverted (J <= 0)")
        return f

    def forces_anp(self, u):
        """Internal forces with the average nodal pressure (see ora_forces_anp)."""
        u = _f64(u, (self.n_nodes, 3))
        f = np.zeros((self.n_nodes, 3))
        bad = ctypes.c_int(-1)
        rc = self._lib.ora_forces_anp(self._ctx, _dp(u), _dp(f), ctypes.byref(bad))
        if rc != 0:
            raise FloatingPointError(f"element {bad.value} inverted (J <= 0)")
        return f

    def element_force(self, e: int, Ue, route: int = 0):
        Ue = _f64(Ue, (self.ne, 3))
        Fe = np.zeros((self.ne, 3))
        self._lib.ora_element_force(self._ctx, int(e), _dp(Ue), _dp(Fe), int(route))
        return Fe

    def energy(self, u) -> float:
        return self._lib.ora_energy(self._ctx, _dp(_f64(u, (self.n_nodes, 3))))

    def run(self, u_cur, u_prev, n_steps, dt, alpha, bc_node=None, bc_mask=None, bc_target=None, R=None,
            ramp=RAMP_SMOOTH, t_ramp=0.0, step0=0, relax=False, tol=0.0, check_every=1, anp=False):
        """Advance (u_cur, u_prev) in place; returns (rc, steps_done, last_residual).
        anp=True steps with the average-nodal-pressure force (forces_anp)."""
        assert u_cur.dtype == np.float64 and u_cur.flags.c_contiguous
        assert u_prev.dtype == np.float64 and u_prev.flags.c_contiguous
        if bc_node is None:
            bc_node = np.zeros(0, np.int32)
            bc_mask = np.zeros(0, np.int32)
            bc_target = np.zeros((0, 3))
        bn = np.ascontiguousarray(bc_node, dtype=np.int32)
        bm = np.ascontiguousarray(bc_mask, dtype=np.int32)
        bt = _f64(bc_target, (len(bn), 3))
        Rp = _dp(_f64(R, (self.n_nodes, 3))) if R is not None else None
        res = ctypes.c_double(0.0)
        done = ctypes.c_int(0)
        rc = self._lib.ora_run(self._ctx, _dp(u_cur), _dp(u_prev), Rp, len(bn), _ip(bn), _ip(bm), _dp(bt),
                               int(ramp), float(t_ramp), float(dt), float(alpha), int(step0), int(n_steps),
                               int(bool(relax)), float(tol), int(check_every), ctypes.byref(res),
                               ctypes.byref(done), int(bool(anp)))
        return rc, done.value, res.value

    def residual(self, u, bc_node, bc_mask, R=None) -> float:
        bn = np.ascontiguousarray(bc_node, dtype=np.int32)
        bm = np.ascontiguousarray(bc_mask, dtype=np.int32)
        Rp = _dp(_f64(R, (self.n_nodes, 3))) if R is not None else None
        return self._lib.ora_residual(self._ctx, _dp(_f64(u, (self.n_nodes, 3))), Rp, len(bn), _ip(bn), _ip(bm))
