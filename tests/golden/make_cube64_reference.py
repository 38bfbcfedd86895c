"""Writes the FP64 oracle's state after the full 1000-step run of the 64^3
compression cube (1,572,864 tetrahedra and 262,144 hexahedra), for the GPU
parity test of the full-size run.

Calls only the oracle (test infrastructure) and the seeded input generators;
nothing here touches the GPU library.  The run follows Eq. 13 (central
differences with mass-proportional damping) with the critical step of Eq. 14
(dt = 0.9 dt_crit), the load ramped smoothly over the 1000 steps.  Stored per
mesh (cube64_<t4|h8>_u1000.npz): a fingerprint of the inputs, dt, the
oracle's max-norm and 2-norm of the whole final field, and the final
displacement of 8192 seeded sample nodes.  The all-cores build of the oracle
is used only to make this faster: its forces and runs equal the serial
build's bit for bit (pinned in tests/test_oracle.py).

    python tests/golden/make_cube64_reference.py [t4] [h8]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2106_14189_amd import workloads as W  # noqa: E402

N_SAMPLE = 8192
N_STEPS = 1000


def fingerprint(wl) -> str:
    """sha256 over the inputs that define the run (mesh, material, loads)."""
    h = hashlib.sha256()
    for a in (wl.mesh.X, wl.mesh.conn, np.asarray(wl.material.E, np.float64), np.asarray(wl.material.nu, np.float64),
              wl.loads.bc_node, wl.loads.bc_mask, wl.loads.bc_target,
              np.array([wl.material.rho, wl.material.hg_kappa, wl.alpha, wl.loads.ramp], np.float64)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def path_for(tag: str) -> str:
    return os.path.join(HERE, f"cube64_{tag}_u{N_STEPS}.npz")


def sample_nodes(n_nodes: int) -> np.ndarray:
    return np.sort(np.random.default_rng(20210614).choice(n_nodes, size=N_SAMPLE, replace=False)).astype(np.int32)


def make(tag: str) -> None:
    elem = W.T4 if tag == "t4" else W.H8
    wl = W.config1(elem)
    m, mat, ld = wl.mesh, wl.material, wl.loads
    ora = oracle.Oracle(m.X, m.conn, mat.E, mat.nu, rho=mat.rho, hg_kappa=mat.hg_kappa, omp=True)
    dt = 0.9 * ora.dt_crit
    u, up = np.zeros((m.n_nodes, 3)), np.zeros((m.n_nodes, 3))
    t0 = time.perf_counter()
    rc, done, _ = ora.run(u, up, N_STEPS, dt, wl.alpha, ld.bc_node, ld.bc_mask, ld.bc_target, ramp=ld.ramp,
                          t_ramp=N_STEPS * dt)
    assert rc == 0 and done == N_STEPS, (rc, done)
    nodes = sample_nodes(m.n_nodes)
    np.savez(path_for(tag), fingerprint=np.array(fingerprint(wl)), dt=np.array(dt), steps=np.array(N_STEPS),
             umax=np.array(np.abs(u).max()), unorm=np.array(np.linalg.norm(u)), nodes=nodes, u=u[nodes])
    print(f"{tag}: {m.n_elems} elements, {N_STEPS} steps in {time.perf_counter() - t0:.1f} s "
          f"on {oracle.threads(True)} threads; max|u| = {np.abs(u).max():.6e}", flush=True)


if __name__ == "__main__":
    for tag in (sys.argv[1:] or ["t4", "h8"]):
        make(tag)
