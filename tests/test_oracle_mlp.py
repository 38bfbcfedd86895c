"""Pins of the surrogate-MLP oracle against what the mathematics fixes:
finite differences of the float64 loss, a library BF16 rounding, and the
closed form of Adam's first steps."""
import numpy as np
import pytest

from oracle import mlp


def _params(rng, n_in=3, H=8, n_out=5, scale=0.5):
    return {"W1": scale * rng.normal(size=(n_in, H)), "b1": 0.1 * rng.normal(size=H),
            "W2": scale * rng.normal(size=(H, H)), "b2": 0.1 * rng.normal(size=H),
            "W3": scale * rng.normal(size=(n_out, H)), "b3": 0.1 * rng.normal(size=n_out)}


def test_gradients_equal_finite_differences():
    rng = np.random.default_rng(0)
    prm = _params(rng)
    P = rng.normal(size=(4, 3))
    U = rng.normal(size=(4, 5))
    loss, g = mlp.loss_grad(prm, P, U)
    assert loss == pytest.approx(mlp.loss_only(prm, P, U), rel=1e-15)
    h = 1e-6
    for k, w in prm.items():
        fd = np.zeros_like(w)
        for idx in np.ndindex(w.shape):
            wp = {kk: vv.copy() for kk, vv in prm.items()}
            wm = {kk: vv.copy() for kk, vv in prm.items()}
            wp[k][idx] += h
            wm[k][idx] -= h
            fd[idx] = (mlp.loss_only(wp, P, U) - mlp.loss_only(wm, P, U)) / (2 * h)
        np.testing.assert_allclose(g[k], fd, rtol=1e-6, atol=1e-9, err_msg=k)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5e-3, 3.14159, 65504.0, 1e-30,
                     -1 - 2 ** -8])
    rng = np.random.default_rng(1)
    vals = np.concatenate([vals, rng.normal(size=1000) * 10.0 ** rng.uniform(-6, 6, 1000)])
    ref = torch.from_numpy(vals.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(vals), ref)
    assert mlp.bf16(np.array([1 + 2 ** -8]))[0] == 1.0            # tie -> even
    assert mlp.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(2)
    prm = _params(rng)
    g = {k: rng.normal(size=v.shape) for k, v in prm.items()}
    m = {k: np.zeros_like(v) for k, v in prm.items()}
    v = {k: np.zeros_like(w) for k, w in prm.items()}
    p0 = {k: w.copy() for k, w in prm.items()}
    lr, eps = 1e-3, 1e-8
    mlp.adam(prm, g, m, v, 1, lr, eps=eps)
    for k in prm:  # bias-corrected first moments are g and g^2
        np.testing.assert_allclose(prm[k] - p0[k], -lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-12)
    mlp.adam(prm, g, m, v, 2, lr, eps=eps)  # constant gradient: the same step again
    for k in prm:
        np.testing.assert_allclose(prm[k] - p0[k], -2 * lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-9)


def test_bf16_emulation_stays_close_to_float64():
    rng = np.random.default_rng(3)
    prm = _params(rng, n_in=16, H=64, n_out=40, scale=0.2)
    P = rng.uniform(-1, 1, size=(32, 16))
    U = rng.normal(size=(32, 40))
    l64, g64 = mlp.loss_grad(prm, P, U)
    lbf, gbf = mlp.loss_grad(prm, P, U, emulate_bf16=True)
    assert abs(lbf - l64) / l64 < 2e-2
    for k in g64:  # BF16 has 8 significant bits; a few ReLU masks may flip
        assert np.linalg.norm(gbf[k] - g64[k]) <= 5e-2 * np.linalg.norm(g64[k]), k
