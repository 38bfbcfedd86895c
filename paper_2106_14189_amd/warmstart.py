"""Learned warm start for dynamic relaxation.

A load family on a fixed mesh -- the bottom cap fixed and four seeded
surface patches, each prescribed with amplitude x unit direction x a smooth
window -- is parameterised by p in R^16.  Steady states of the plain DJ-TLED
dynamic relaxation (computed here in batches of instances that share the
mesh) train the surrogate MLP p -> u on the GPU; for new loads its
prediction seeds u^0 = u^{-1} and the relaxation runs on to convergence, so
the network only changes where the iteration starts.  The comparison counts
steps, device time and wall time to a relative displacement error of 1e-3
against the converged plain solution, from the prediction and from rest with
the best of several ramp lengths (including the load applied at once).

Everything numerical runs in libdjtled.so (DJ-TLED kernels, BF16 MFMA
network kernels); this module chooses loads, moves tensors and keeps time.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from . import solver as S
from .mlp import SurrogateMLP

AMP_MAX = 0.003  # largest patch displacement [m] (surface stretch of the window near 25 %)


@dataclass
class PatchFamily:
    """Bottom cap fixed; `n_patches` disjoint patches of upper-surface nodes."""
    mesh: object
    n_patches: int = 4
    frac: float = 0.03
    seed: int = 0
    fixed: np.ndarray = field(init=False)
    patches: list = field(init=False)
    windows: list = field(init=False)

    def __post_init__(self):
        m = self.mesh
        rng = np.random.default_rng(self.seed)
        surf = m.surface
        upper = surf[m.X[surf, 2] > -0.2 * np.abs(m.X[:, 2]).max()]
        k = max(4, int(round(self.frac * len(surf))))
        # spread the centres: farthest-point choice among random upper-surface nodes
        cand = rng.choice(upper, size=min(len(upper), 64), replace=False)
        centres = [cand[0]]
        for _ in range(1, self.n_patches):
            d = np.min([np.linalg.norm(m.X[cand] - m.X[c], axis=1) for c in centres], axis=0)
            centres.append(cand[int(np.argmax(d))])
        taken = np.zeros(m.n_nodes, bool)
        self.patches, self.windows = [], []
        for c in centres:
            d = np.linalg.norm(m.X[surf] - m.X[c], axis=1)
            order = surf[np.argsort(d)]
            nodes = [n for n in order[: 2 * k] if not taken[n]][:k]
            nodes = np.array(nodes, np.int32)
            taken[nodes] = True
            r = np.linalg.norm(m.X[nodes] - m.X[c], axis=1)
            R = r.max() * 1.05 + 1e-12
            self.patches.append(nodes)
            self.windows.append((1.0 - (r / R) ** 2) ** 2)
        self.fixed = np.array([n for n in m.bottom if not taken[n]], np.int32)
        self.bc_node = np.concatenate([self.fixed] + self.patches).astype(np.int32)
        self.bc_mask = np.full(len(self.bc_node), 7, np.int32)

    @property
    def dim(self) -> int:
        return 4 * self.n_patches

    def sample(self, rng, n: int) -> np.ndarray:
        """n load vectors (amplitude in [0, 1] x AMP_MAX, unit direction) per patch."""
        p = np.zeros((n, self.dim))
        for j in range(self.n_patches):
            d = rng.normal(size=(n, 3))
            p[:, 4 * j] = rng.uniform(0.0, 1.0, n)
            p[:, 4 * j + 1:4 * j + 4] = d / np.linalg.norm(d, axis=1, keepdims=True)
        return p

    def encode(self, P: np.ndarray) -> np.ndarray:
        """Network input of load vectors: per patch (a d_x, a d_y, a d_z, a)."""
        E = np.zeros_like(P)
        for j in range(self.n_patches):
            a = P[:, 4 * j:4 * j + 1]
            E[:, 4 * j:4 * j + 3] = a * P[:, 4 * j + 1:4 * j + 4]
            E[:, 4 * j + 3] = P[:, 4 * j]
        return E

    def targets(self, p: np.ndarray) -> np.ndarray:
        """BC targets (n_bc x 3) of one load vector."""
        out = [np.zeros((len(self.fixed), 3))]
        for j in range(self.n_patches):
            a, d = p[4 * j] * AMP_MAX, p[4 * j + 1:4 * j + 4]
            out.append(a * self.windows[j][:, None] * d[None, :])
        return np.concatenate(out)


def _instances(mesh, mat, fam: PatchFamily, P: np.ndarray, t_ramp: float, alpha: float):
    ins = []
    for p in P:
        ins.append(S.Instance(mesh.X, mesh.conn, mat.E, mat.nu, model=mat.model, rho=mat.rho,
                              eta_ratio=mat.eta_ratio, fibre=mat.fibre, hg_kappa=mat.hg_kappa,
                              bc_node=fam.bc_node, bc_mask=fam.bc_mask, bc_target=fam.targets(p),
                              ramp=L.DJ_RAMP_SMOOTH, t_ramp=t_ramp, alpha=alpha))
    return ins


def steady_states(mesh, mat, fam: PatchFamily, P: np.ndarray, n_steps: int, t_ramp: float, alpha: float,
                  per_batch: int = 64, log=None) -> tuple[torch.Tensor, float]:
    """u after n_steps of damped explicit dynamics for every load in P, computed
    per_batch instances at a time in one batched persistent launch; returns
    (U [n x 3N] float32 on the GPU, device seconds)."""
    n, N = len(P), mesh.n_nodes
    U = torch.empty((n, 3 * N), dtype=torch.float32, device="cuda")
    dev_ms = 0.0
    for s in range(0, n, per_batch):
        chunk = P[s:s + per_batch]
        b = S.Batch(_instances(mesh, mat, fam, chunk, t_ramp, alpha), use_graph=True)
        st = b.run(n_steps)
        if st.code != 0:
            raise RuntimeError(f"steady-state batch failed: {st}")
        dev_ms += st.kernel_ms
        for i in range(len(chunk)):
            U[s + i] = b.read(i).reshape(-1)
        b.close()
        if log:
            log(f"  steady states {s + len(chunk)}/{n}: {st.kernel_ms:.0f} ms")
    return U, dev_ms / 1e3


def steady_states_single(sv: S.Solver, fam: PatchFamily, P: np.ndarray, tol: float, t_ramp: float,
                         check_every: int = 100, max_steps: int = 400000, sv64: S.Solver | None = None,
                         tol64: float = 1e-6, log=None) -> tuple[torch.Tensor, float]:
    """Relaxed states for every load in P on one context (meshes too large to
    batch): relaxation to r <= tol, optionally continued on an FP64 context to
    r <= tol64.  Returns (U [n x 3N] float32 on the GPU, device seconds)."""
    n, N = len(P), sv.n_nodes
    U = torch.empty((n, 3 * N), dtype=torch.float32, device="cuda")
    dev_ms = 0.0
    for i, p in enumerate(P):
        ls = sv.loadset(fam.bc_node, fam.bc_mask, fam.targets(p), L.DJ_RAMP_SMOOTH, t_ramp)
        u, up = sv.zeros(), sv.zeros()
        st, step = sv.step(u, up, max_steps, ls, relax=True, tol=tol, check_every=check_every)
        ls.close()
        if st.code != 1:
            raise RuntimeError(f"relaxation of load {i} did not converge: {st}")
        dev_ms += st.kernel_ms
        if sv64 is not None:
            ls = sv64.loadset(fam.bc_node, fam.bc_mask, fam.targets(p), L.DJ_RAMP_SMOOTH, t_ramp)
            u64, up64 = u.double(), up.double()
            st, _ = sv64.step(u64, up64, max_steps, ls, step0=step, relax=True, tol=tol64, check_every=check_every)
            ls.close()
            if st.code != 1:
                raise RuntimeError(f"FP64 relaxation of load {i} did not converge: {st}")
            dev_ms += st.kernel_ms
            u = u64.float()
        U[i] = u.reshape(-1)
        if log and (i % max(1, n // 8) == 0 or i == n - 1):
            log(f"  relaxed {i + 1}/{n}: {st.steps_done} steps, r = {st.residual:.2e}")
    return U, dev_ms / 1e3


def residual_of(sv: S.Solver, fam: PatchFamily, p: np.ndarray, u: torch.Tensor, check_every: int = 1) -> float:
    """The relaxation residual of state u under load p (one RELAX check, no step)."""
    ls = sv.loadset(fam.bc_node, fam.bc_mask, fam.targets(p), L.DJ_RAMP_NONE, 0.0)
    uc, up = u.clone(), u.clone()
    st, _ = sv.step(uc, up, 1, ls, step0=0, relax=True, tol=float("inf"), check_every=check_every)
    ls.close()
    return st.residual


@dataclass
class SolveTrace:
    steps: int          # steps to the error target (-1: not reached)
    device_ms: float    # device time of the steps taken up to then
    wall_ms: float      # host wall time up to then (chunked runs + error checks)
    errors: list


def solve_to_error(sv: S.Solver, fam: PatchFamily, p: np.ndarray, u_ref: torch.Tensor, u0: torch.Tensor | None,
                   t_ramp: float, target: float = 1e-3, chunk: int = 50, max_steps: int = 200000,
                   extra_ms: float = 0.0, extra_wall_ms: float = 0.0) -> SolveTrace:
    """Runs the relaxation from u0 (or from rest with a smooth ramp) in chunks
    of `chunk` steps until |u - u_ref| / |u_ref| <= target."""
    ramp = L.DJ_RAMP_SMOOTH if u0 is None else L.DJ_RAMP_NONE
    ls = sv.loadset(fam.bc_node, fam.bc_mask, fam.targets(p), ramp, t_ramp if u0 is None else 0.0)
    u = sv.zeros() if u0 is None else u0.clone()
    up = u.clone()
    ref = u_ref.reshape(-1, 3)
    nref = torch.linalg.vector_norm(ref).item()
    step, dev, errs = 0, extra_ms, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = SolveTrace(-1, 0.0, 0.0, errs)
    while step < max_steps:
        st, step = sv.step(u, up, chunk, ls, step0=step)
        if st.code != 0:
            raise RuntimeError(f"relaxation failed: {st}")
        dev += st.kernel_ms
        e = torch.linalg.vector_norm(u - ref).item() / nref
        errs.append(e)
        if e <= target:
            out.steps = step
            break
    out.device_ms = dev
    out.wall_ms = (time.perf_counter() - t0) * 1e3 + extra_wall_ms
    ls.close()
    return out


COLD_RAMPS = (0.0, 0.025, 0.05, 0.1, 0.2, 0.4)  # cold-start ramp lengths swept [s]; 0: step load


def _trace_stats(tr: list) -> dict:
    ok = [t for t in tr if t is not None and t.steps > 0]
    d = {"reached": len(ok), "of": len(tr)}
    if ok:
        d.update(steps_median=float(np.median([t.steps for t in ok])),
                 device_ms_median=float(np.median([t.device_ms for t in ok])),
                 wall_ms_median=float(np.median([t.wall_ms for t in ok])))
    return d


def experiment(mesh, mat, alpha: float, n_train: int, n_test: int, seed: int, relax_steps: int, t_ramp: float,
               hidden: int = 512, epochs: int = 200, batch: int = 64, lr: float = 1e-3, per_batch: int = 64,
               chunk: int = 50, single: bool = False, tol_train: float = 1e-3, cold_ramps=COLD_RAMPS,
               log=print) -> dict:
    """Train on n_train steady states, compare warm and cold starts on n_test loads.
    single=False: steady states from batches of instances (relax_steps fixed
    steps); single=True (large meshes): one context, FP32 relaxation to
    tol_train for training data, and an FP64 finish to 1e-6 for the held-out
    references.  t_ramp is the ramp of the data-generating relaxations.  The
    cold start is tuned: every ramp length in cold_ramps (0 = the full load
    applied at once) is run on every held-out load, and the warm start is
    compared with the ramp whose median wall time to the target is lowest
    among those that reach it on every load (a run that inverts an element
    does not reach it)."""
    rng = np.random.default_rng(seed)
    fam = PatchFamily(mesh, seed=seed)
    P_tr, P_te = fam.sample(rng, n_train), fam.sample(rng, n_test)
    log(f"mesh {mesh.n_elems} elements / {mesh.n_nodes} nodes; {len(fam.bc_node)} prescribed nodes; "
        f"{n_train} training and {n_test} held-out loads")
    sv = S.Solver(mesh.X, mesh.conn, mat.E, mat.nu, model=mat.model, rho=mat.rho, eta_ratio=mat.eta_ratio,
                  fibre=mat.fibre, hg_kappa=mat.hg_kappa, alpha=alpha)
    t0 = time.perf_counter()
    if single:
        sv64 = S.Solver(mesh.X, mesh.conn, mat.E, mat.nu, model=mat.model, rho=mat.rho, eta_ratio=mat.eta_ratio,
                        fibre=mat.fibre, hg_kappa=mat.hg_kappa, alpha=alpha, precision="fp64")
        U_tr, gen_s = steady_states_single(sv, fam, P_tr, tol_train, t_ramp, log=log)
        U_te, gen_te_s = steady_states_single(sv, fam, P_te, tol_train, t_ramp, sv64=sv64, log=log)
        sv64.close()
    else:
        U_tr, gen_s = steady_states(mesh, mat, fam, P_tr, relax_steps, t_ramp, alpha, per_batch, log)
        U_te, gen_te_s = steady_states(mesh, mat, fam, P_te, relax_steps, t_ramp, alpha, per_batch, log)
    gen_wall = time.perf_counter() - t0
    # the reference states must be converged: residual of a few of them
    res = [residual_of(sv, fam, P_te[i], U_te[i].reshape(-1, 3)) for i in range(min(4, n_test))]
    log(f"  data: {gen_s + gen_te_s:.1f} s device, {gen_wall:.1f} s wall; held-out residuals {max(res):.2e}")
    # network: inputs are the encoded load vectors, outputs u / AMP_MAX
    net = SurrogateMLP(fam.dim, hidden, 3 * mesh.n_nodes, seed=seed)
    Pd = torch.from_numpy(fam.encode(P_tr)).float().cuda()
    Ud = torch.zeros((n_train, net.ld_out), dtype=torch.float32, device="cuda")
    Ud[:, : 3 * mesh.n_nodes] = U_tr / AMP_MAX
    t0 = time.perf_counter()
    losses = net.fit(Pd, Ud, epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # held-out evaluation
    cold = {tr: [] for tr in cold_ramps}
    warm, pred_err, infer_ms = [], [], []
    Pt = torch.from_numpy(fam.encode(P_te)).float().cuda()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(n_test):
        torch.cuda.synchronize()
        tw = time.perf_counter()
        ev0.record()
        Y = net.forward(Pt[i:i + 1])
        ev1.record()
        torch.cuda.synchronize()
        inf_wall_ms = (time.perf_counter() - tw) * 1e3
        inf_ms = ev0.elapsed_time(ev1)
        infer_ms.append(inf_ms)
        u0 = (Y[0, : 3 * mesh.n_nodes] * AMP_MAX).reshape(-1, 3).contiguous()
        ref = U_te[i]
        pred_err.append(torch.linalg.vector_norm(u0.reshape(-1) - ref).item() / torch.linalg.vector_norm(ref).item())
        warm.append(solve_to_error(sv, fam, P_te[i], ref, u0, t_ramp, chunk=chunk, extra_ms=inf_ms,
                                   extra_wall_ms=inf_wall_ms))
        for tr in cold_ramps:
            try:
                cold[tr].append(solve_to_error(sv, fam, P_te[i], ref, None, tr, chunk=chunk))
            except RuntimeError:  # the load applied too fast inverts an element
                cold[tr].append(None)
    sv.close()
    sweep = {f"{tr:g}": _trace_stats(cold[tr]) for tr in cold_ramps}
    full = [tr for tr in cold_ramps if sweep[f"{tr:g}"]["reached"] == n_test]
    best = min(full, key=lambda tr: sweep[f"{tr:g}"]["wall_ms_median"]) if full else None
    ws = _trace_stats(warm)
    out = {
        "n_train": n_train, "n_test": n_test, "elements": mesh.n_elems, "nodes": mesh.n_nodes,
        "relax_steps_for_data": relax_steps, "data_device_s": gen_s + gen_te_s, "train_s": train_s,
        "train_loss_first_last": [losses[0], losses[-1]], "held_out_residual_max": max(res),
        "prediction_error_median": float(np.median(pred_err)),
        "inference_ms_median": float(np.median(infer_ms)),
        "cold_sweep": sweep, "cold_ramp_s": best,
        "warm_steps_median": ws.get("steps_median", -1.0),
        "warm_device_ms_median": ws.get("device_ms_median", -1.0),
        "warm_wall_ms_median": ws.get("wall_ms_median", -1.0),
        "all_reached": bool(best is not None and ws["reached"] == n_test),
    }
    if best is not None:
        b = sweep[f"{best:g}"]
        out.update(cold_steps_median=b["steps_median"], cold_device_ms_median=b["device_ms_median"],
                   cold_wall_ms_median=b["wall_ms_median"])
        out["speedup_steps"] = out["cold_steps_median"] / max(out["warm_steps_median"], 1)
        out["speedup_device_time"] = out["cold_device_ms_median"] / max(out["warm_device_ms_median"], 1e-9)
        out["speedup_wall_time"] = out["cold_wall_ms_median"] / max(out["warm_wall_ms_median"], 1e-9)
    return out
