"""djtled_forces_noalloc, the allocation-free variant of djtled_forces (its
scratch is a fixed device array of the library), called through the C ABI:
its output must equal djtled_forces' bit for bit (same kernels, same order),
on two calls in a row, the second on a smaller context, and a context whose
scratch need exceeds the fixed array must be refused."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2106_14189_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, elem, prec, seed):
    from paper_2106_14189_amd import solver as S
    rng = np.random.default_rng(seed)
    mesh = W.cube_mesh(n, 0.1 / n, elem, jitter=0.05, seed=seed, permute=True)
    E = rng.uniform(2000.0, 6000.0, mesh.n_elems)
    sv = S.Solver(mesh.X, mesh.conn, E, 0.45, precision=prec)
    dt = torch.float32 if prec == "fp32" else torch.float64
    u = torch.tensor(mesh.X * 0.05 * np.array([0.3, -0.2, -1.0]) + 1e-4 * rng.normal(size=mesh.X.shape),
                     dtype=dt, device="cuda")
    return sv, u


def _noalloc(sv, u):
    from paper_2106_14189_amd import _lib as L
    f = torch.full_like(u, float("nan"))
    rc = L.lib.djtled_forces_noalloc(sv.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, f


def test_noalloc_forces_equal_forces_on_two_calls():
    from paper_2106_14189_amd import _lib as L
    assert torch.cuda.is_available()
    # first call: the larger context; second call: a smaller one (the array keeps the first call's contents)
    for n, elem, prec in ((12, W.T4, "fp32"), (5, W.H8, "fp64")):
        say(f"noalloc: {n}^3 {'T4' if elem == W.T4 else 'H8'} {prec}")
        sv, u = _case(n, elem, prec, seed=n)
        ref = sv.forces(u)
        rc, f = _noalloc(sv, u)
        torch.cuda.synchronize()
        assert rc == L.DJ_OK, L.lib.djtled_last_error().decode()
        assert torch.isfinite(f).all()
        assert torch.equal(f, ref), (f - ref).abs().max().item()
        sv.close()


def test_noalloc_refuses_a_context_beyond_the_fixed_scratch():
    """96^3-voxel cube (5.3M tetrahedra) in FP64 with small workgroup tiles:
    its node copies and partial sums need more than the fixed 64 MiB, so the
    call is refused before any launch and the output is left untouched."""
    from paper_2106_14189_amd import _lib as L
    from paper_2106_14189_amd import solver as S
    mesh = W.cube_mesh(96, 0.1 / 96, W.T4, jitter=0.05, seed=3, permute=True)
    sv = S.Solver(mesh.X, mesh.conn, 3000.0, 0.45, precision="fp64", chunk_elems=192)
    inf = sv.info()
    need = 3 * 8 * (inf["n_copies"] + max(inf["n_shared_copies"], 1))
    say(f"  {inf['n_copies']} copies, {inf['n_shared_copies']} shared -> {need / 2**20:.1f} MiB")
    assert need > 64 << 20
    u = torch.zeros((mesh.n_nodes, 3), dtype=torch.float64, device="cuda")
    rc, f = _noalloc(sv, u)
    torch.cuda.synchronize()
    assert rc == L.DJ_ERR_UNSUPPORTED
    assert "fixed scratch" in L.lib.djtled_last_error().decode()
    assert torch.isnan(f).all()  # nothing was written
    sv.close()
