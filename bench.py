#!/usr/bin/env python3
"""DJ-TLED time-step benchmark on one MI355X.

Headline workload (synthetic, seeded): a batch of 256 independent box
instances with element counts log-uniform in [5k, 200k] (14.19M elements in
total), each a fair coin between linear tetrahedra and one-point hexahedra
with hourglass control and between neo-Hookean and transversely isotropic
material, E ~ U[2, 6] kPa, nu = 0.45, rho = 1000, jittered +-5 %, permuted;
bottom face fixed, top face moved by U[5 %, 20 %] of the height in a seeded
downward direction with a smooth ramp over 500 steps; each instance at 0.9 x
its own critical step; FP32.  One benchmark step advances every instance by
one explicit time step (element forces -> node reduction -> central
difference with damping -> BCs) in one persistent kernel launch replayed
from a hipGraph, with the inputs resident in HBM.  Setup (pre-computation,
autotuning, graph capture) precedes the W warmup steps; K steps are timed.

Further measurements, reported under "extra" (each skippable):
  * cube64: the 64^3 cube as 1,572,864 tetrahedra and as 262,144 hexahedra
    (NH, compression, FP32), one persistent launch of K steps per mesh;
  * models: the 64^3 cubes with each material model of Table 3 (NH, TI, OT,
    MR): time per step, overhead over NH, and the ratio to the same step with
    the classical TLED force;
  * multi: k = 1, 2, 4, 8 compression cases per launch on the 64^3 cubes
    (djtled_step_multi): time per step and element-steps/s over cases;
  * anp: the average-nodal-pressure step (Sec. 7) on the 64^3 cubes next to
    the element-pressure step;
  * realtime (--realtime): step time over cube sizes and the model sizes
    for one step per 33.3 ms / 2 ms (Sec. 5.5), checked at the 2 ms size;
  * relaxation: the ~1.2M-tet transversely isotropic ellipsoid relaxed to
    r <= 1e-3 in FP32 and finished to r <= 1e-6 in FP64;
  * mlp: the full-size surrogate network's training and inference kernels;
  * warm start: surrogate trained on the GPU from relaxation steady states
    of a ~6000-tet ellipsoid; steps, device and wall time to 1e-3 relative
    displacement error from the prediction vs from rest with the best of a
    sweep of ramp lengths.

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported:
the library runs on a single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_2106_14189_amd", "csrc")
# sources of each measured kernel, and the committed counter summaries taken of it
KERNELS = {
    "batch": {"src": ["djtled_batch_kernels.hip", "djtled_device.h"],
              "traffic": os.path.join(ROOT, "profiles", "djtled_batch_config3_traffic.json")},
    "step": {"src": ["djtled_kernels.hip", "djtled_device.h"],
             "traffic": os.path.join(ROOT, "profiles", "djtled_step_cube64_t4_traffic.json")},
}
METRIC = "DJ-TLED element-steps/sec + HBM GB/s; warm-start vs plain time-to-1e-3"


def _src_sha(kernel: str) -> str:
    """sha256 of a kernel's sources (its kernel file and the device header)."""
    h = hashlib.sha256()
    for f in KERNELS[kernel]["src"]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def _traffic(kernel: str, steps: int):
    """HBM bytes of `steps` steps from committed rocprofv3 PMC counters
    (FETCH_SIZE + WRITE_SIZE per step, calibrated on a plain copy), or None if
    the kernel's sources changed since they were taken."""
    try:
        t = json.load(open(KERNELS[kernel]["traffic"]))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != _src_sha(kernel):
        return None
    return (t["fetch_bytes_per_step"] + t["write_bytes_per_step"]) * steps


def _copy_calib(torch) -> int:
    """Copies a 256 MiB buffer 4 times: a plain copy kernel of known size whose
    rocprofv3 FETCH_SIZE / WRITE_SIZE readings calibrate the byte counters."""
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    n = x.numel() * 4
    del x, y
    return n


def host_info() -> dict:
    """Host CPU model and core counts (as lscpu / nproc would report them)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc, "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _oracle_leg(spec, n_steps: int, omp: bool) -> tuple[int, float]:
    """(element-steps, seconds) of the FP64 oracle stepping each instance of
    spec from rest by n_steps steps of its own load (construction untimed)."""
    import numpy as np

    import oracle

    es, secs = 0, 0.0
    for m, mat, ld, alpha in spec:
        ora = oracle.Oracle(m.X, m.conn, mat.E, mat.nu, model=mat.model, rho=mat.rho, eta_ratio=mat.eta_ratio,
                            fibre=mat.fibre, hg_kappa=mat.hg_kappa, omp=omp)
        dt = 0.9 * ora.dt_crit
        t_ramp = -ld.t_ramp * dt if ld.t_ramp < 0 else ld.t_ramp
        u, up = np.zeros((m.n_nodes, 3)), np.zeros((m.n_nodes, 3))
        t0 = time.perf_counter()
        rc, done, _ = ora.run(u, up, n_steps, dt, alpha, ld.bc_node, ld.bc_mask, ld.bc_target, ramp=ld.ramp,
                              t_ramp=t_ramp)
        secs += time.perf_counter() - t0
        assert rc == 0 and done == n_steps, (rc, done)
        es += m.n_elems * n_steps
        del ora
    return es, secs


def cpu_baseline(spec, n_steps: int, every: int = 16) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the batch: every
    `every`-th instance stepped n_steps from rest, single-threaded and with its
    element loop on all host cores (the OpenMP build of the same source)."""
    import oracle

    sample = spec[::every]
    n_el = sum(m.n_elems for m, _, _, _ in sample)
    es1, s1 = _oracle_leg(sample, n_steps, omp=False)
    esn, sn = _oracle_leg(sample, n_steps, omp=True)
    nthr = oracle.threads(omp=True)
    what = (f"{len(sample)} of the {len(spec)} instances (every {every}th; {n_el} elements) x {n_steps} steps "
            f"from rest; FP64 C oracle, gcc -O2")
    return {"value": esn / sn, "unit": "element-steps/s", "cores": nthr, "kind": "oracle",
            "sample": what + f"; element loop on {nthr} OpenMP threads", "seconds": round(sn, 2),
            "single_thread": {"value": es1 / s1, "unit": "element-steps/s", "cores": 1, "kind": "oracle",
                              "sample": what + "; one thread", "seconds": round(s1, 2)},
            "host": host_info()}


def copy_ceiling(nbytes: int = 2 << 30, reps: int = 10) -> dict:
    """Achievable HBM bandwidth on this GPU in the same run: a device-to-device
    copy of nbytes (read + write), timed with HIP events."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return {"GBps": 2.0 * nbytes / (ms / 1e3) / 1e9, "bytes_copied": nbytes, "ms": ms}


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q))


def bench_cube64(log, K: int, Wm: int, variant: int = -1, meshes: str = "both") -> dict:
    """The 64^3 compression cube as 1,572,864 T4 and as 262,144 H8 (NH, FP32,
    E ~ U[2, 6] kPa, permuted): K steps of each mesh in one persistent launch
    after Wm warmup steps; per-mesh kernel time (HIP events on the launch
    stream), algorithmic bytes and, for T4, the committed counter traffic."""
    import torch
    from paper_2106_14189_amd import solver
    from paper_2106_14189_amd import workloads as W
    elems = {"both": [W.T4, W.H8], "t4": [W.T4], "h8": [W.H8]}[meshes]
    out = {"workload": "cube64_" + "+".join("t4" if e == W.T4 else "h8" for e in elems) + "_nh_fp32_compression",
           "steps": K, "warmup": Wm}
    tot_es, tot_s = 0, 0.0
    for elem in elems:
        wl = W.config1(elem)
        tag = "t4" if elem == W.T4 else "h8"
        kw = {} if variant < 0 else {"variant": variant}
        sv = solver.from_workload(wl, **kw)
        i = sv.info()
        ld = wl.loads
        ls = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, 1000 * i["dt"])
        u, up = sv.zeros(), sv.zeros()
        st, step = sv.step(u, up, Wm, ls)
        assert st.code == 0, st
        st, step = sv.step(u, up, K, ls, step0=step)
        torch.cuda.synchronize()
        assert st.code == 0 and st.steps_done == K, st
        assert bool(torch.isfinite(u).all())
        km = st.kernel_ms
        tot_es += i["n_elems"] * K
        tot_s += km / 1e3
        out[tag] = {"elems": i["n_elems"], "nodes": i["n_nodes"], "kernel_ms_per_step": km / K,
                    "element_steps_per_s": i["n_elems"] * K / (km / 1e3), "bytes_per_step": i["bytes_per_step"],
                    "bytes_per_element_step": i["bytes_per_step"] / i["n_elems"],
                    "effective_GBps": i["bytes_per_step"] * K / (km / 1e3) / 1e9,
                    "frac_of_hbm_peak": i["bytes_per_step"] * K / (km / 1e3) / 1e9 / HBM_PEAK_GBPS,
                    "counter_traffic_bytes_per_step": (_traffic("step", 1) if elem == W.T4 else None),
                    "dt": i["dt"], "grid": i["grid_blocks"], "chunks": i["n_chunks"],
                    "chunk_elems": i["chunk_elems"], "variant": i["variant"]}
        ls.close()
        sv.close()
        log(f"cube64 {tag}: {out[tag]}")
    out["element_steps_per_s_both"] = tot_es / tot_s
    return out


def bench_models(log, steps: int = 500) -> dict:
    """The four material models of Table 3 on the config-1 cubes (T4 and H8,
    FP32, automatic kernel variant): kernel time per step, the overhead of
    TI, OT and MR over NH (Table 7 reports these overheads on the paper's
    GPU), and the same step with the classical TLED force (Eq. 4) for the
    DJ-TLED / TLED time ratio (Table 5 reports it on the paper's CPU).
    Fibre and C01 inputs as workloads.uniform_material draws them."""
    import numpy as np
    import torch
    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W
    out = {}
    for elem in (W.T4, W.H8):
        wl = W.config1(elem)
        tag = "t4" if elem == W.T4 else "h8"
        ms = {}
        for model, name in ((W.NH, "nh"), (W.TI, "ti"), (W.OT, "ot"), (W.MR, "mr")):
            mat = W.uniform_material(wl.mesh.n_elems, wl.material.E, 0.45, 1000.0, model=model,
                                     rng=np.random.default_rng(11 + model))
            for form, suffix in (("jacobian", ""), ("classical", "_classical")):
                sv = S.Solver(wl.mesh.X, wl.mesh.conn, mat.E, mat.nu, model=model, rho=mat.rho,
                              eta_ratio=mat.eta_ratio, fibre=mat.fibre, eta_b_ratio=mat.eta_b_ratio,
                              fibre_b=mat.fibre_b, c01=mat.c01, hg_kappa=mat.hg_kappa, alpha=wl.alpha,
                              formulation=form)
                info = sv.info()
                ld = wl.loads
                ls = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, 1000 * info["dt"])
                u, up = sv.zeros(), sv.zeros()
                st, step = sv.step(u, up, 50, ls)
                st, step = sv.step(u, up, steps, ls, step0=step)
                torch.cuda.synchronize()
                assert st.code == 0 and st.steps_done == steps, st
                key = name + suffix
                ms[key] = st.kernel_ms / steps
                out[f"{tag}_{key}_kernel_us_per_step"] = ms[key] * 1e3
                out[f"{tag}_{key}_element_steps_per_s"] = info["n_elems"] / (ms[key] / 1e3)
                if not suffix:
                    out[f"{tag}_{name}_bytes_per_step"] = info["bytes_per_step"]
                    out[f"{tag}_{name}_effective_GBps"] = info["bytes_per_step"] / (ms[key] / 1e3) / 1e9
                    out[f"{tag}_variant"] = info["variant"]
                sv.close()
            out[f"{tag}_{name}_ratio_jacobian_over_classical"] = ms[name] / ms[name + "_classical"]
        for name in ("ti", "ot", "mr"):
            out[f"{tag}_{name}_overhead_vs_nh"] = ms[name] / ms["nh"] - 1.0
        log(f"models {tag}: " + ", ".join(f"{k} {v * 1e3:.1f} us" for k, v in ms.items()))
    out["workload"] = "cube64_t4+h8_fp32_compression_nh/ti/ot/mr"
    out["steps"] = steps
    return out


def bench_realtime(log) -> dict:
    """Real-time sizing (Sec. 5.5): kernel time per explicit step of the
    compression cube (NH, FP32, automatic variant) over a range of sizes, a
    least-squares line t = a + b E over the sizes with E >= 1M elements, the
    element counts at which one step takes 33.3 ms (30 Hz visual feedback) and
    2 ms (500 Hz haptic feedback), and a measurement at the 2 ms size."""
    import numpy as np
    import torch
    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W

    def measure(elem, n):
        mesh = W.cube_mesh(n, 0.1 / n, elem, jitter=0.05, seed=7, permute=True)
        E = np.random.default_rng(n).uniform(2000.0, 6000.0, mesh.n_elems)
        try:
            sv = S.Solver(mesh.X, mesh.conn, E, 0.45, alpha=37.0)
        except Exception as e:  # beyond the automatic variant's chunk list: the 512-workgroup variant
            log(f"realtime n={n}: {e}; variant 0")
            sv = S.Solver(mesh.X, mesh.conn, E, 0.45, alpha=37.0, variant=0)
        info = sv.info()
        ld = W.compression_loads(mesh, -0.2, W.RAMP_SMOOTH, 1000 * info["dt"])
        ls = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, ld.t_ramp)
        u, up = sv.zeros(), sv.zeros()
        st, step = sv.step(u, up, 20, ls)
        est = st.kernel_ms / 20
        k = int(min(2000, max(20, 30.0 / max(est, 1e-3))))
        st, step = sv.step(u, up, k, ls, step0=step)
        torch.cuda.synchronize()
        assert st.code == 0, st
        row = {"n": n, "elems": info["n_elems"], "nodes": info["n_nodes"], "dofs": 3 * info["n_nodes"],
               "steps": k, "us_per_step": st.kernel_ms / k * 1e3, "variant": info["variant"]}
        sv.close()
        del mesh
        log(f"realtime {'t4' if elem == W.T4 else 'h8'} {row}")
        return row

    out = {"workload": "cube_t4/h8_nh_fp32_compression_sizes"}
    for elem, tag, sizes in ((W.T4, "t4", (8, 16, 24, 32, 48, 64, 96, 128, 160)),
                             (W.H8, "h8", (8, 16, 32, 48, 64, 96, 128, 192, 256))):
        rows = [measure(elem, n) for n in sizes]
        big = [r for r in rows if r["elems"] >= 1_000_000]
        x = np.array([r["elems"] for r in big], float)
        y = np.array([r["us_per_step"] for r in big]) * 1e-6
        b, a = np.polyfit(x, y, 1)
        pred = {hz: (1.0 / hz - a) / b for hz in (30, 500)}
        # measured point past the fitted 500 Hz size; the 500 Hz size is then
        # interpolated between measured points, and the 30 Hz size (beyond this
        # host-side mesh generator) extrapolated with the slope of the two largest
        per = 6 if elem == W.T4 else 1
        n500 = int(round((pred[500] / per) ** (1.0 / 3.0)))
        check = measure(elem, n500)
        pts = sorted(rows + [check], key=lambda r: r["elems"])
        ex = np.array([r["elems"] for r in pts], float)
        ey = np.array([r["us_per_step"] for r in pts]) * 1e-6
        e500 = float(np.interp(2e-3, ey, ex)) if ey[-1] >= 2e-3 else None
        slope = (ey[-1] - ey[-2]) / (ex[-1] - ex[-2])
        e30 = float(ex[-1] + (1.0 / 30 - ey[-1]) / slope)
        out[tag] = {"sizes": rows, "fit_s_per_step": {"a": a, "b_per_element": b},
                    "fit_elements_at_30Hz": pred[30], "fit_elements_at_500Hz": pred[500], "check": check,
                    "elements_at_500Hz_measured": e500, "elements_at_30Hz_extrapolated": e30,
                    "min_us_per_step": min(r["us_per_step"] for r in rows)}
    return out


def bench_multi(log, steps: int = 300) -> dict:
    """Several load cases per launch (djtled_step_multi) on the config-1 cubes
    (automatic kernel variant): k compression cases of different strain share
    each step's grid barrier; kernel time per step and element-steps/s
    counting every case (k = 1: the single-case kernel)."""
    import torch
    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W
    out = {"workload": "cube64_t4+h8_nh_fp32_compression_k_cases", "steps": steps}
    for elem, variant in ((W.T4, -1), (W.T4, 2), (W.H8, -1)):
        wl = W.config1(elem)
        sv = S.from_workload(wl, variant=variant)
        info = sv.info()
        tag = ("t4" if elem == W.T4 else "h8") + ("" if variant < 0 else f"_v{variant}")
        out[f"{tag}_variant"] = info["variant"]
        per = {}
        for k in (1, 2, 4, 8):
            lss = []
            for i in range(k):
                ld = W.compression_loads(wl.mesh, -0.2 + 0.01 * i, W.RAMP_SMOOTH, 1000 * info["dt"])
                lss.append(sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, ld.t_ramp))
            U, UP = sv.zeros_multi(k), sv.zeros_multi(k)
            st, step, _, _ = sv.step_multi(U, UP, 20, lss)
            st, step, _, _ = sv.step_multi(U, UP, steps, lss, step0=step)
            torch.cuda.synchronize()
            assert st.code == 0 and st.steps_done == steps, st
            us = st.kernel_ms / steps * 1e3
            per[k] = us
            out[f"{tag}_k{k}_kernel_us_per_step"] = us
            out[f"{tag}_k{k}_element_steps_per_s"] = k * info["n_elems"] / (us * 1e-6)
            for ls in lss:
                ls.close()
        for k in (2, 4, 8):
            out[f"{tag}_k{k}_per_case_over_k1"] = per[k] / k / per[1]
        log(f"multi {tag}: " + ", ".join(f"k={k} {v:.1f} us ({v / k:.1f} per case)" for k, v in per.items()))
        sv.close()
    return out


def bench_anp(log, steps: int = 300) -> dict:
    """The average-nodal-pressure step (Sec. 7; formulation nodal_pressure)
    on the 64^3 compression cubes, T4 and H8, NH, FP32: kernel time per step
    next to the element-pressure step of the same mesh (the ANP step makes a
    second element pass and a second grid barrier per step)."""
    import torch
    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W
    out = {"workload": "cube64_t4+h8_nh_fp32_compression_nodal_pressure", "steps": steps}
    for elem in (W.T4, W.H8):
        wl = W.config1(elem)
        tag = "t4" if elem == W.T4 else "h8"
        for form in ("jacobian", "nodal_pressure"):
            sv = S.from_workload(wl, formulation=form)
            info = sv.info()
            ld = wl.loads
            ls = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, 1000 * info["dt"])
            u, up = sv.zeros(), sv.zeros()
            st, step = sv.step(u, up, 20, ls)
            st, step = sv.step(u, up, steps, ls, step0=step)
            torch.cuda.synchronize()
            assert st.code == 0 and st.steps_done == steps, st
            out[f"{tag}_{form}_us_per_step"] = st.kernel_ms / steps * 1e3
            out[f"{tag}_{form}_bytes_per_step"] = info["bytes_per_step"]
            out[f"{tag}_{form}_effective_GBps"] = info["bytes_per_step"] * steps / (st.kernel_ms / 1e3) / 1e9
            ls.close()
            sv.close()
        out[f"{tag}_anp_over_standard"] = out[f"{tag}_nodal_pressure_us_per_step"] / out[f"{tag}_jacobian_us_per_step"]
        log(f"anp {tag}: {out[f'{tag}_jacobian_us_per_step']:.1f} us standard, "
            f"{out[f'{tag}_nodal_pressure_us_per_step']:.1f} us nodal pressure")
    return out


def bench_relaxation(log, ramps=(0.0, 0.05, 0.1, 0.2, 0.4)) -> dict:
    """The ~1.2M-tet TI ellipsoid: FP32 dynamic relaxation to r <= 1e-3 (above
    its FP32 rounding floor) for each load-ramp length in `ramps` (0: the load
    applied at once; residual checks start when the ramp is complete), then
    the fastest converged run finished in FP64 to r <= 1e-6."""
    import torch
    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W
    wl = W.config2()
    ld = wl.loads
    ce = wl.extra["check_every"]
    out = {"workload": wl.name, "elements": wl.mesh.n_elems, "nodes": wl.mesh.n_nodes, "check_every": ce,
           "fp32_sweep": {}}
    s32 = S.from_workload(wl, precision="fp32")
    best = None
    for tr in ramps:
        ls = s32.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, tr)
        u, up = s32.zeros(), s32.zeros()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, step = s32.step(u, up, 400000, ls, relax=True, tol=1e-3, check_every=ce, raise_on_error=False)
        torch.cuda.synchronize()
        ls.close()
        row = {"code": st.code, "steps": st.steps_done, "residual": st.residual, "kernel_ms": st.kernel_ms,
               "wall_ms": (time.perf_counter() - t0) * 1e3,
               "ramp_steps": int(round(tr / s32.info()["dt"])),
               "element_steps_per_s": wl.mesh.n_elems * st.steps_done / max(st.kernel_ms / 1e3, 1e-12)}
        out["fp32_sweep"][f"{tr:g}"] = row
        log(f"relaxation t_ramp {tr:g} s: {row}")
        if st.code == 1 and (best is None or st.steps_done < best[1]):
            best = (tr, st.steps_done, u, up, step)
    assert best is not None, out
    tr, _, u, up, step = best
    out.update(t_ramp=tr, fp32_steps=out["fp32_sweep"][f"{tr:g}"]["steps"],
               fp32_kernel_ms=out["fp32_sweep"][f"{tr:g}"]["kernel_ms"],
               fp32_element_steps_per_s=out["fp32_sweep"][f"{tr:g}"]["element_steps_per_s"])
    s64 = S.from_workload(wl, precision="fp64")
    ls64 = s64.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, tr)
    u64, up64 = u.double(), up.double()
    t0 = time.perf_counter()
    st64, _ = s64.step(u64, up64, 400000, ls64, step0=step, relax=True, tol=1e-6, check_every=ce)
    torch.cuda.synchronize()
    out.update(fp64_steps=st64.steps_done, fp64_residual=st64.residual, fp64_kernel_ms=st64.kernel_ms,
               fp64_wall_ms=(time.perf_counter() - t0) * 1e3, converged=st64.code == 1)
    ls64.close()
    s32.close()
    s64.close()
    log(f"relaxation: {out}")
    return out


def bench_mlp(log) -> dict:
    """Surrogate network at the full config-4 size (16 -> 512 -> 512 -> 3N,
    3N = 638,757 outputs of the ~213k-node ellipsoid): one training step
    (forward, loss, backward, Adam) at batch 256 and one inference at batch 1,
    timed with HIP events.  FLOPs: 2 B (16 H + H^2 + H n_out) forward, three
    times that for a training step's products."""
    import torch
    from paper_2106_14189_amd.mlp import SurrogateMLP
    n_out, H, B = 3 * 212919, 512, 256
    net = SurrogateMLP(16, H, n_out, seed=0)
    P = torch.rand((B, 16), device="cuda")
    U = torch.randn((B, net.ld_out), device="cuda") * 0.1
    for _ in range(2):
        net.loss_grad(P, U, want_loss=False)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        net.loss_grad(P, U, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    lg_ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        net.adam_step(1e-4)
    e1.record()
    torch.cuda.synchronize()
    adam_ms = e0.elapsed_time(e1) / reps
    Y = torch.empty((B, net.ld_out), device="cuda")
    net.forward(P, out=Y)
    e0.record()
    for _ in range(reps):
        net.forward(P, out=Y)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    del Y
    P1 = P[:1].contiguous()
    net.forward(P1)
    e0.record()
    for _ in range(reps):
        net.forward(P1)
    e1.record()
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1) / reps
    fwd = 2.0 * B * (16 * H + H * H + H * n_out)
    out = {"n_out": n_out, "batch": B, "loss_grad_ms": lg_ms, "adam_ms": adam_ms, "forward_ms": fwd_ms,
           "inference_ms_batch1": inf_ms, "forward_GBps_W3": 2.0 * H * net.ld_out / (fwd_ms / 1e3) / 1e9,
           "train_products_TFLOPs": 3 * fwd / (lg_ms / 1e3) / 1e12,
           "inference_GBps_W3": 2.0 * H * net.ld_out / (inf_ms / 1e3) / 1e9}
    log(f"mlp: {out}")
    return out


def bench_warm_start(log) -> dict:
    from paper_2106_14189_amd import warmstart
    from paper_2106_14189_amd import workloads as W
    wl = W.config2(target_elems=6000)
    r = warmstart.experiment(wl.mesh, wl.material, wl.alpha, n_train=512, n_test=16, seed=4, relax_steps=6000,
                             t_ramp=0.4, hidden=512, epochs=150, batch=64, lr=1e-3, log=log)
    r["workload"] = "ellipsoid6k_t4_ti_fp32_patch_loads"
    return r


def bench_warm_start_full(log, n_train: int = 1024, n_test: int = 32) -> dict:
    """The warm-start pipeline on the full ~1.2M-tet ellipsoid: training
    states from single-context FP32 relaxations to r <= 1e-3 (load ramped over
    0.05 s, the fastest converging ramp of the relaxation sweep), held-out
    references finished in FP64 to r <= 1e-6, the network trained on the GPU,
    and warm vs tuned cold starts (ramp lengths 0 - 0.4 s) to 1e-3 relative
    displacement error."""
    from paper_2106_14189_amd import warmstart
    from paper_2106_14189_amd import workloads as W
    wl = W.config2()
    r = warmstart.experiment(wl.mesh, wl.material, wl.alpha, n_train=n_train, n_test=n_test, seed=4, relax_steps=0,
                             t_ramp=0.05, hidden=512, epochs=100, batch=64, lr=1e-3, single=True, tol_train=1e-3,
                             chunk=100, log=log)
    r["workload"] = "ellipsoid1200k_t4_ti_fp32_patch_loads"
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="oracle steps per sampled instance for cpu_baseline (0: skip)")
    ap.add_argument("--batch-variant", type=int, default=-1, help="batch kernel variant (-1: autotune)")
    ap.add_argument("--variant", type=int, default=-1, help="cube64 kernel variant (-1: per-mesh default)")
    ap.add_argument("--mesh", choices=["both", "t4", "h8"], default="both", help="cube64 meshes")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after the run, copy a 256 MiB buffer 4 times (calibrates rocprofv3 byte counters)")
    ap.add_argument("--no-cube", action="store_true", help="skip the 64^3 cube measurement")
    ap.add_argument("--no-models", action="store_true", help="skip the four-material-model measurement")
    ap.add_argument("--no-multi", action="store_true", help="skip the several-load-cases measurement")
    ap.add_argument("--no-anp", action="store_true", help="skip the average-nodal-pressure step measurement")
    ap.add_argument("--no-relax", action="store_true", help="skip the ellipsoid relaxation measurement")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start measurement")
    ap.add_argument("--no-mlp", action="store_true", help="skip the full-size network timing")
    ap.add_argument("--no-extra", action="store_true", help="skip every measurement under extra")
    ap.add_argument("--realtime", action="store_true",
                    help="also measure step time over cube sizes up to ~60M elements (real-time sizing)")
    ap.add_argument("--warm-full", action="store_true",
                    help="also run the warm-start pipeline on the full ellipsoid (several GPU-minutes)")
    ap.add_argument("--only", choices=["cube64", "models", "multi", "anp", "realtime", "relaxation", "mlp",
                                       "warm_start", "warm_start_full"],
                    help="run this one measurement alone (no headline line; for profiling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: --gpus {args.gpus} requested; this DJ-TLED library runs on one GPU only "
              f"(multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import math

    import torch

    from paper_2106_14189_amd import solver as S
    from paper_2106_14189_amd import workloads as W

    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    K, Wm = args.steps, args.warmup
    extras = (("cube64", args.no_cube, lambda lg: bench_cube64(lg, K, Wm, args.variant, args.mesh)),
              ("models", args.no_models, bench_models),
              ("multi", args.no_multi, bench_multi),
              ("anp", args.no_anp, bench_anp),
              ("realtime", not args.realtime, bench_realtime),
              ("relaxation", args.no_relax, bench_relaxation),
              ("mlp", args.no_mlp, bench_mlp), ("warm_start", args.no_warm, bench_warm_start),
              ("warm_start_full", not args.warm_full, bench_warm_start_full))
    if args.only:
        r = dict((n, f) for n, _, f in extras)[args.only](log)
        torch.cuda.synchronize()
        out = {"only": args.only, args.only: r}
        if args.copy_calib:
            out["copy_calib_bytes"] = _copy_calib(torch)
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    spec = W.config3()
    ins = [S.Instance(m.X, m.conn, mat.E, mat.nu, model=mat.model, rho=mat.rho, eta_ratio=mat.eta_ratio,
                      fibre=mat.fibre, hg_kappa=mat.hg_kappa, bc_node=ld.bc_node, bc_mask=ld.bc_mask,
                      bc_target=ld.bc_target, ramp=ld.ramp, t_ramp=ld.t_ramp, alpha=al) for m, mat, ld, al in spec]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = S.Batch(ins, autotune=args.batch_variant < 0, variant=args.batch_variant)
    del ins
    t_build = time.perf_counter() - t0
    info = b.info()
    log(f"batch: {info['n_inst']} instances, {info['n_elems']} elements, variant {info['variant']}, "
        f"chunk {info['chunk_elems']}, {info['n_items']} chunks on {info['grid_blocks']} workgroups, "
        f"{info['steps_per_launch']} steps per launch")
    # setup: capture the K-step and W-step graphs, then start from rest
    for n in ([K, Wm] if Wm > 0 else [K]):
        st = b.run(n)
        assert st.code == 0, st
    b.reset()
    if Wm > 0:
        st = b.run(Wm)
        assert st.code == 0 and st.steps_done == Wm, st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.run(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert st.code == 0 and st.steps_done == K and st.kernel_ms > 0, st
    info = b.info()
    lat = b.stats()
    bps = info["bytes_per_step"]
    spl = info["steps_per_launch"] if info["steps_per_launch"] > 0 else K
    launches = math.ceil(K / spl)
    # HIP events on the launch stream around the replayed graph: the
    # persistent launches of the run and their flag-reset kernels
    k_s = st.kernel_ms / 1e3
    achieved = bps * K / k_s / 1e9
    traffic = _traffic("batch", K)
    ceiling = copy_ceiling()
    cfg = {"workload": "batch256_boxes_5k-200k_t4h8_nhti_fp32", "instances": info["n_inst"],
           "elements": info["n_elems"], "nodes": info["n_nodes"], "precision": "fp32", "steps_timed": K,
           "kernel_ms": st.kernel_ms, "kernel_ms_per_step": st.kernel_ms / K,
           "element_steps_per_s_kernel": info["n_elems"] * K / k_s,
           "bytes_per_step": bps, "bytes_per_element_step": bps / info["n_elems"],
           "instance_latency_ms_p50": _pct(lat, 50), "instance_latency_ms_p99": _pct(lat, 99),
           "graph": info["graph"],
           "autotune": {"variant": info["variant"], "chunk_elems": info["chunk_elems"],
                        "steps_per_launch": info["steps_per_launch"], "candidates": info["tune_candidates"],
                        "tune_ms": info["tune_ms"]},
           "grid": info["grid_blocks"], "block": info["block_threads"], "chunks": info["n_items"],
           "host_build_s": t_build, "host_gen_s": t_gen}
    out = {
        "metric": METRIC,
        "value": info["n_elems"] * K / wall,
        "unit": "element-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": wall / K * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None if traffic is None else traffic / launches,
                     "kernel": "k_batch_step (persistent fused DJ-TLED step of the whole batch)",
                     "bytes_per_step": bps, "steps_per_launch": min(spl, K), "launches": launches,
                     "bytes_per_launch": bps * min(spl, K), "launch_ms_avg": st.kernel_ms / launches,
                     "copy_ceiling_GBps": ceiling["GBps"], "frac_of_copy_ceiling": achieved / ceiling["GBps"]},
    }
    b.close()
    del b
    torch.cuda.synchronize()
    if args.copy_calib:
        out["copy_calib_bytes"] = _copy_calib(torch)
    out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps) if args.cpu_steps > 0 else None
    del spec
    extra = {}
    for name, skip, fn in extras:
        if skip or (args.no_extra and name not in ("realtime", "warm_start_full")):
            continue
        try:
            extra[name] = fn(log)
        except Exception as e:  # reported, not hidden: the main line stays valid
            extra[name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.synchronize()
        log(f"{name}: {json.dumps(extra[name])[:400]}")
    out["extra"] = extra
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
