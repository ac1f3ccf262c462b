"""Pins of the cost-MLP oracle: a hand-written numpy forward pass, central
finite differences of its MSE gradient, and the Adam update's first-step
closed form (lr * sign(g) for |g| >> eps)."""
import numpy as np

from oracle import mlp


def _data(seed=0, rows=50):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, size=mlp.N_PARAMS)
    norm = np.r_[rng.normal(0, 1, 8), rng.uniform(0.5, 2, 8), rng.uniform(-3, -1, 8), rng.uniform(1, 3, 8)]
    x = rng.normal(0, 2, size=(rows, 8))
    t = rng.normal(0, 1, size=rows)
    return w, norm, x, t


def test_forward_matches_numpy():
    w, norm, x, _ = _data()
    W1, b1 = w[:256].reshape(32, 8), w[256:288]
    W2, b2 = w[288:1312].reshape(32, 32), w[1312:1344]
    W3, b3 = w[1344:1376], w[1376]
    xn = (np.clip(x, norm[16:24], norm[24:32]) - norm[:8]) / norm[8:16]
    h1 = np.maximum(xn @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    np.testing.assert_allclose(mlp.forward(w, norm, x).numpy(), h2 @ W3 + b3, rtol=1e-12)


def test_gradient_matches_central_differences():
    w, norm, x, t = _data(1)
    loss, g = mlp.mse_and_grad(w, norm, x, t)
    rng = np.random.default_rng(2)
    for k in rng.choice(mlp.N_PARAMS, 120, replace=False):
        e = np.zeros_like(w)
        e[k] = 1e-6
        fd = (mlp.mse_and_grad(w + e, norm, x, t)[0] - mlp.mse_and_grad(w - e, norm, x, t)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(3)
    g = rng.normal(size=100)
    w1, m, v = mlp.adam(np.zeros(100), np.zeros(100), np.zeros(100), g, 1, 1e-3)
    # update = lr g / (|g| + eps): relative deviation eps / |g|
    np.testing.assert_allclose(w1, -1e-3 * np.sign(g), rtol=1e-8 / np.abs(g).min() * 1.01)
