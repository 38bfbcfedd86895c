"""The surrogate MLP's BF16 MFMA kernels against the float64 oracle.

* GEMM (all four operand layouts, ragged sizes, split K, the one-row-tile
  shape of the output layer): exact BF16 inputs,
  so the only difference is FP32 summation: |C_gpu - C_ref| <= 1e-5 sum_k |A||B|.
* forward (batches of 1 and 2 take streaming products per layer; batches up
  to 256 with H <= 512 the persistent W3 kernels; others the tiled GEMM),
  loss and every gradient against the oracle with the same BF16
  roundings emulated: relative Frobenius error <= 1e-2 (an FP32-order
  difference can flip a BF16 rounding, or a ReLU mask at zero).
* Adam: one step against the oracle's step on the same gradients, <= 1e-5.
* training reduces the loss of a smooth synthetic map by 10x.
"""
import ctypes
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2106_14189_amd import _lib as L
    from paper_2106_14189_amd import mlp
    return L, mlp


def _bf(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16)


@pytest.mark.parametrize("M_,N_,K_,ak,bk,splits", [(200, 300, 100, 1, 1, 1), (129, 77, 64, 0, 1, 1),
                                                    (256, 130, 40, 1, 0, 1), (70, 512, 515, 0, 0, 1),
                                                    (33, 260, 2000, 1, 0, 7), (1, 1000, 512, 1, 1, 1),
                                                    (200, 8300, 72, 1, 1, 1), (250, 8200, 40, 0, 0, 1),
                                                    (130, 8192, 100, 1, 0, 2)])
def test_gemm_layouts(M, M_, N_, K_, ak, bk, splits):
    L, _ = M
    rng = np.random.default_rng(M_ + N_ + K_)
    A = rng.normal(size=(M_, K_))
    B = rng.normal(size=(K_, N_))
    Ab, Bb = _bf(A), _bf(B)
    A64, B64 = Ab.double().numpy(), Bb.double().numpy()
    lda = (K_ if ak else M_ + 5) + 7 & ~7  # padded leading dimensions
    ldb = (K_ if bk else N_ + 3) + 7 & ~7
    Ad = torch.zeros((M_ if ak else K_, lda), dtype=torch.bfloat16)
    if ak:
        Ad[:, :K_] = Ab
    else:
        Ad[:, :M_] = Ab.T
    Bd = torch.zeros((N_ if bk else K_, ldb), dtype=torch.bfloat16)
    if bk:
        Bd[:, :K_] = Bb.T
    else:
        Bd[:, :N_] = Bb
    Ad, Bd = Ad.cuda(), Bd.cuda()
    C = torch.full((splits, M_, N_), float("nan"), dtype=torch.float32, device="cuda")
    z = L.lib.djtled_mlp_gemm_test(M_, N_, K_, ctypes.c_void_p(Ad.data_ptr()), lda, ak, ctypes.c_void_p(Bd.data_ptr()),
                                   ldb, bk, ctypes.c_void_p(C.data_ptr()), N_, splits, None)
    assert z >= 1
    torch.cuda.synchronize()
    Cg = C[:z].sum(0).double().cpu().numpy()
    ref = A64 @ B64
    bound = np.abs(A64) @ np.abs(B64)
    err = np.abs(Cg - ref) / bound
    say(f"M={M_} N={N_} K={K_} A{'k' if ak else 'm'} B{'k' if bk else 'n'} splits={z}: max err/bound {err.max():.2e}")
    assert np.isfinite(Cg).all() and err.max() <= 1e-5


def _net(mlp, n_in, H, n_out, seed):
    net = mlp.SurrogateMLP(n_in, H, n_out, seed=seed)
    rng = np.random.default_rng(seed)
    w = {"W1": rng.normal(size=(n_in, H)) * 0.4, "b1": rng.normal(size=H) * 0.1,
         "W2": rng.normal(size=(H, H)) * (1.5 / H) ** 0.5, "b2": rng.normal(size=H) * 0.1,
         "W3": np.zeros((net.ld_out, H)), "b3": np.zeros(net.ld_out)}
    w["W3"][:n_out] = rng.normal(size=(n_out, H)) * (1.0 / H) ** 0.5
    w["b3"][:n_out] = rng.normal(size=n_out) * 0.1
    net.set_weights({k: torch.from_numpy(v) for k, v in w.items()})
    prm = {k: (v[:n_out] if k in ("W3", "b3") else v) for k, v in w.items()}
    return net, prm


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("B,H,n_out", [(70, 64, 1001), (256, 512, 4227), (200, 512, 8500), (1, 512, 9001),
                                       (2, 64, 300), (1, 2048, 333), (300, 64, 777), (33, 520, 250),
                                       (96, 256, 65000)])
def test_forward_loss_and_gradients_match_oracle(M, B, H, n_out):
    L, mlp = M
    net, prm = _net(mlp, 16, H, n_out, seed=B)
    rng = np.random.default_rng(B + 1)
    P = rng.uniform(-1, 1, size=(B, 16))
    U = rng.normal(size=(B, n_out)) * 0.5
    Pd = torch.from_numpy(P).float().cuda()
    Ud = torch.zeros((B, net.ld_out), dtype=torch.float32, device="cuda")
    Ud[:, :n_out] = torch.from_numpy(U).float()
    Y = net.forward(Pd)[:, :n_out].double().cpu().numpy()
    Yo, _ = omlp.forward(prm, P.astype(np.float32), emulate_bf16=True)
    ey = _rel(Y, Yo)
    loss = net.loss_grad(Pd, Ud)
    lo, go = omlp.loss_grad(prm, P.astype(np.float32), U.astype(np.float32), emulate_bf16=True)
    say(f"B={B} H={H} n_out={n_out}: forward {ey:.2e}, loss {loss:.6e} vs {lo:.6e}")
    assert ey <= 1e-2
    assert abs(loss - lo) <= 1e-3 * lo
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        g = net.g[k].double().cpu().numpy()
        if k in ("W3", "b3"):
            assert np.abs(g[n_out:]).max() == 0.0  # padded outputs carry no gradient
            g = g[:n_out]
        e = _rel(g, go[k])
        say(f"  d{k}: rel error {e:.2e}")
        assert e <= 1e-2


def test_adam_step_matches_oracle(M):
    L, mlp = M
    net, prm = _net(mlp, 16, 64, 300, seed=5)
    rng = np.random.default_rng(9)
    gr = {k: rng.normal(size=v.shape) * 1e-3 for k, v in prm.items()}
    for k, v in gr.items():
        net.g[k].zero_()
        net.g[k][: v.shape[0]] = torch.from_numpy(v).float()
    gr = {k: net.g[k][: v.shape[0]].double().cpu().numpy() for k, v in gr.items()}
    w0 = {k: net.w[k][: v.shape[0]].double().cpu().numpy() for k, v in prm.items()}
    m = {k: np.zeros_like(v) for k, v in w0.items()}
    v = {k: np.zeros_like(x) for k, x in w0.items()}
    ref = {k: x.copy() for k, x in w0.items()}
    for t in (1, 2):
        net.adam_step(1e-3)
        omlp.adam(ref, gr, m, v, t, 1e-3)
    for k in ref:
        got = net.w[k][: ref[k].shape[0]].double().cpu().numpy()
        # FP32 weights: the step is exact to a few units in the last place of w
        tol = 1e-5 * np.abs(ref[k] - w0[k]).max() + 4 * 2.0 ** -24 * np.abs(w0[k]).max()
        assert np.abs(got - ref[k]).max() <= tol, k
    wb = net.wb["W2"].float().cpu().numpy()
    np.testing.assert_array_equal(wb, omlp.bf16(net.w["W2"].cpu().numpy()).astype(np.float32))


def test_training_reduces_loss(M):
    L, mlp = M
    rng = np.random.default_rng(4)
    n_out, n = 600, 512
    P = rng.uniform(-1, 1, size=(n, 16))
    basis = rng.normal(size=(16, n_out)) / 4
    U = np.tanh(P @ basis) + 0.3 * (P[:, :1] ** 2)
    net = mlp.SurrogateMLP(16, 256, n_out, seed=1)
    Pd = torch.from_numpy(P).float().cuda()
    Ud = torch.zeros((n, net.ld_out), dtype=torch.float32, device="cuda")
    Ud[:, :n_out] = torch.from_numpy(U).float()
    losses = net.fit(Pd, Ud, epochs=60, batch=64, lr=2e-3, log=say)
    say(f"loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.1 * losses[0]
