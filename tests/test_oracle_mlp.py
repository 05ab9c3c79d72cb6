"""Pins for the oracle's MLP: central differences of the loss, a closed form
for the last layer alone, and Adam's first step."""
import numpy as np

from oracle import mlp

R = np.random.default_rng(17)


def _setup(F=7, H=5, K=3, B=6):
    p = R.standard_normal(mlp.nparams(F, H, K)) * 0.5
    X = R.standard_normal((B, F))
    T = R.standard_normal((B, K))
    mask = (R.uniform(size=(B, K)) > 0.3).astype(float)
    mask[0, 0] = 1.0
    return p, X, T, mask, F, H, K


def test_gradient_central_differences():
    p, X, T, mask, F, H, K = _setup()
    g = mlp.grad(p, X, T, mask, F, H, K)
    h = 1e-6
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T, mask, F, H, K) - mlp.loss(p - e, X, T, mask, F, H, K)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd))


def test_last_layer_closed_form():
    """With W1 = I-like positive paths fixed, the output is linear in (W3, b3):
    y = h2 W3 + b3, so the loss gradient w.r.t. b3 is 2 sum(mask (y - t)) / sum(mask)."""
    p, X, T, mask, F, H, K = _setup()
    h1, h2, y = mlp.forward(p, X, F, H, K)
    g = mlp.grad(p, X, T, mask, F, H, K)
    db3 = g[-K:]
    assert np.allclose(db3, 2 * np.sum(mask * (y - T), axis=0) / mask.sum(), rtol=1e-12)
    dW3 = g[-K - H * K:-K].reshape(H, K)
    assert np.allclose(dW3, h2.T @ (2 * mask * (y - T) / mask.sum()), rtol=1e-12)


def test_adam_first_step_is_sign_step():
    """On the first step the bias-corrected update is lr * g / (|g| + eps)."""
    p = R.standard_normal(10)
    g = R.standard_normal(10)
    q, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01, eps=1e-12)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
