"""Surrogate-MLP oracle: TEST INFRASTRUCTURE ONLY.

Plain NumPy (float64) forward pass, mean-squared-error loss, hand-derived
backward pass and Adam step of the warm-start network
    H1 = relu(P W1 + b1),  H2 = relu(H1 W2 + b2),  Y = H2 W3^T + b3,
    loss = mean over (rows, outputs) of (Y - U)^2.
The paper proposes data-driven acceleration only as future work (Sec. 8)
and fixes no network, so these are the textbook definitions: backpropagation
through affine maps and ReLU, and Adam (Kingma and Ba, 2015, Algorithm 1).

``emulate_bf16=True`` rounds, to BF16 (round to nearest even, through FP32),
exactly the tensors the GPU path stores in BF16 -- the input, the weight
copies, both activations and the three back-propagated signals -- and keeps
every sum in float64, so the GPU result differs only by its FP32 summation
order.  Pins (tests/test_oracle_mlp.py): gradients equal central finite
differences of the float64 loss; Adam's first step equals -lr g / (|g| + eps).
Only tests, the smoke check and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest BF16 value (ties to even), via FP32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(prm: dict, P, emulate_bf16: bool = False):
    """Returns (Y, cache).  prm: W1 [n_in x H], b1, W2 [H x H], b2, W3 [n_out x H], b3."""
    e = emulate_bf16
    Pb = _r(P, e)
    W1, W2, W3 = (_r(prm[k], e) for k in ("W1", "W2", "W3"))
    H1 = _r(np.maximum(Pb @ W1 + prm["b1"], 0.0), e)
    H2 = _r(np.maximum(H1 @ W2 + prm["b2"], 0.0), e)
    Y = H2 @ W3.T + prm["b3"]
    return Y, dict(Pb=Pb, W1=W1, W2=W2, W3=W3, H1=H1, H2=H2)


def loss_grad(prm: dict, P, U, emulate_bf16: bool = False):
    """Mean-squared error and its gradient with respect to every parameter."""
    e = emulate_bf16
    Y, c = forward(prm, P, e)
    B, n_out = Y.shape
    D = Y - U
    loss = float(np.mean(D * D))
    dY = _r(2.0 * D / (B * n_out), e)            # d loss / d Y
    g = {"W3": dY.T @ c["H2"], "b3": dY.sum(axis=0)}
    dZ2 = _r((dY @ c["W3"]) * (c["H2"] > 0), e)    # through the output layer and ReLU
    g["W2"] = c["H1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = _r((dZ2 @ c["W2"].T) * (c["H1"] > 0), e)
    g["W1"] = c["Pb"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, g


def loss_only(prm: dict, P, U) -> float:
    Y, _ = forward(prm, P, False)
    return float(np.mean((Y - U) ** 2))


def adam(prm: dict, g: dict, m: dict, v: dict, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place (bias-corrected moments, step number t >= 1)."""
    for k in prm:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        prm[k] = prm[k] - lr * mh / (np.sqrt(vh) + eps)
