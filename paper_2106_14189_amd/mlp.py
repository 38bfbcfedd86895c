"""Surrogate MLP of the learned warm start (binding of ``include/djtled_mlp.h``).

PyTorch tensors hold the parameters, gradients, Adam moments and the
workspace (device memory only); every product, the loss, the backward pass
and the Adam update run in libdjtled.so's BF16 MFMA kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class SurrogateMLP:
    """p (n_in) -> relu(W1) -> relu(W2) -> W3 -> u (n_out), on one GPU."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, n_in: int, n_hidden: int, n_out: int, device=0, seed: int = 0):
        torch.cuda.init()
        self.n_in, self.n_hidden, self.n_out = int(n_in), int(n_hidden), int(n_out)
        # rows of Y, U and the output gradient start on 256-byte boundaries
        self.ld_out = (self.n_out + 63) // 64 * 64
        self.device = torch.device("cuda", device)
        g = torch.Generator().manual_seed(seed)
        H, O = self.n_hidden, self.ld_out
        shapes = {"W1": (n_in, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (O, H), "b3": (O,)}
        self.shapes = shapes
        w = {
            "W1": torch.randn(shapes["W1"], generator=g) * (2.0 / n_in) ** 0.5,
            "b1": torch.zeros(H),
            "W2": torch.randn(shapes["W2"], generator=g) * (2.0 / H) ** 0.5,
            "b2": torch.zeros(H),
            "W3": torch.randn(shapes["W3"], generator=g) * (1.0 / H) ** 0.5 * 0.1,
            "b3": torch.zeros(O),
        }
        w["W3"][self.n_out:] = 0.0
        self.w = {k: v.to(self.device, torch.float32).contiguous() for k, v in w.items()}
        self.wb = {k: torch.empty(shapes[k], dtype=torch.bfloat16, device=self.device) for k in ("W1", "W2", "W3")}
        self.g = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.m1 = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.m2 = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.t = 0
        self._ws = None
        self._ws_batch = 0
        L.check(L.lib.djtled_mlp_sync_bf16(ctypes.byref(self.desc()), _stream(None)), "djtled_mlp_sync_bf16")

    def desc(self) -> L.djtled_mlp:
        w, wb = self.w, self.wb
        return L.djtled_mlp(self.n_in, self.n_hidden, self.n_out, self.ld_out, _p(w["W1"]), _p(w["b1"]), _p(w["W2"]),
                            _p(w["b2"]), _p(w["W3"]), _p(w["b3"]), _p(wb["W1"]), _p(wb["W2"]), _p(wb["W3"]))

    @staticmethod
    def _grads(d) -> L.djtled_mlp_grads:
        return L.djtled_mlp_grads(*[_p(d[k]) for k in SurrogateMLP.NAMES])

    def set_weights(self, w: dict):
        """Copy FP32 master weights (shapes as self.shapes) and refresh the BF16 copies."""
        for k, v in w.items():
            self.w[k].copy_(torch.as_tensor(v, dtype=torch.float32))
        L.check(L.lib.djtled_mlp_sync_bf16(ctypes.byref(self.desc()), _stream(None)), "djtled_mlp_sync_bf16")

    def _workspace(self, batch: int):
        if self._ws is None or batch > self._ws_batch:
            n = ctypes.c_size_t()
            L.check(L.lib.djtled_mlp_workspace_size(ctypes.byref(self.desc()), int(batch), ctypes.byref(n)),
                    "djtled_mlp_workspace_size")
            self._ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
            self._ws_batch = batch
        return self._ws

    def _check_rows(self, t, cols, name):
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous() or t.dim() != 2 \
                or t.shape[1] != cols:
            raise ValueError(f"{name} must be a contiguous float32 [batch x {cols}] tensor on {self.device}")

    def forward(self, P: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Y [batch x ld_out] (columns >= n_out are not written)."""
        self._check_rows(P, self.n_in, "P")
        B = P.shape[0]
        if out is None:
            out = torch.empty((B, self.ld_out), dtype=torch.float32, device=self.device)
        self._check_rows(out, self.ld_out, "out")
        ws = self._workspace(B)
        L.check(L.lib.djtled_mlp_forward(ctypes.byref(self.desc()), B, _p(P), _p(out), _p(ws), ws.numel(),
                                         _stream(stream)), "djtled_mlp_forward")
        return out

    def loss_grad(self, P: torch.Tensor, U: torch.Tensor, stream=None, want_loss: bool = True) -> float:
        """Fills self.g; U is [batch x ld_out] (columns >= n_out ignored)."""
        self._check_rows(P, self.n_in, "P")
        self._check_rows(U, self.ld_out, "U")
        B = P.shape[0]
        ws = self._workspace(B)
        loss = ctypes.c_double(float("nan"))
        gr = self._grads(self.g)
        L.check(L.lib.djtled_mlp_loss_grad(ctypes.byref(self.desc()), B, _p(P), _p(U), ctypes.byref(gr),
                                           ctypes.byref(loss) if want_loss else None, _p(ws), ws.numel(),
                                           _stream(stream)), "djtled_mlp_loss_grad")
        return loss.value

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        self.t += 1
        g, m1, m2 = self._grads(self.g), self._grads(self.m1), self._grads(self.m2)
        L.check(L.lib.djtled_mlp_adam(ctypes.byref(self.desc()), ctypes.byref(g), ctypes.byref(m1), ctypes.byref(m2),
                                      self.t, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
                "djtled_mlp_adam")

    def fit(self, P: torch.Tensor, U: torch.Tensor, epochs: int, batch: int, lr: float, lr_final: float | None = None,
            seed: int = 0, log=None) -> list:
        """Minibatch Adam over (P, U) with a cosine learning-rate decay; returns the epoch losses."""
        n = P.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        lr_final = lr * 0.05 if lr_final is None else lr_final
        steps = epochs * ((n + batch - 1) // batch)
        losses, it = [], 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(self.device)
            tot = 0.0
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                Pb, Ub = P.index_select(0, idx).contiguous(), U.index_select(0, idx).contiguous()
                frac = it / max(steps - 1, 1)
                lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + torch.cos(torch.tensor(frac * 3.141592653589793)).item())
                tot += self.loss_grad(Pb, Ub) * len(idx)
                self.adam_step(lr_t)
                it += 1
            losses.append(tot / n)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {losses[-1]:.4e}")
        return losses
