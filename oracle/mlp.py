"""CPU oracle of the per-tile cost MLP -- TEST INFRASTRUCTURE ONLY.

Plain PyTorch CPU in float64.  Network: clamp the 8 features to [low, high]
and standardise them with (mean, std) (norm = mean, std, low, high, 8 each),
Linear 8->32, ReLU, Linear 32->32, ReLU, Linear 32->1.  Loss:
mean squared error.  Optimiser: Adam (Kingma & Ba) with beta = (0.9, 0.999),
eps = 1e-8.  Weights are one flat vector: W1[32][8], b1[32], W2[32][32],
b2[32], W3[32], b3.
"""
from __future__ import annotations

import numpy as np
import torch

N_PARAMS = 1377


def unpack(w: torch.Tensor):
    W1 = w[0:256].reshape(32, 8)
    b1 = w[256:288]
    W2 = w[288:1312].reshape(32, 32)
    b2 = w[1312:1344]
    W3 = w[1344:1376]
    b3 = w[1376]
    return W1, b1, W2, b2, W3, b3


def forward(w, norm, x) -> torch.Tensor:
    return forward_t(torch.as_tensor(np.asarray(w, np.float64)), norm, x)


def mse_and_grad(w, norm, x, t):
    """(loss, dloss/dw) by torch autograd."""
    wt = torch.tensor(np.asarray(w, np.float64), requires_grad=True)
    y = forward_t(wt, norm, x)
    loss = torch.mean((y - torch.as_tensor(np.asarray(t, np.float64))) ** 2)
    loss.backward()
    return float(loss.item()), wt.grad.numpy().copy()


def forward_t(wt, norm, x):
    norm = torch.as_tensor(np.asarray(norm, np.float64))
    x = torch.as_tensor(np.asarray(x, np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(wt)
    xn = (torch.minimum(torch.maximum(x, norm[16:24]), norm[24:32]) - norm[:8]) / norm[8:16]
    h1 = torch.relu(xn @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def adam(w, m, v, g, step: int, lr: float, betas=(0.9, 0.999), eps=1e-8):
    """One Adam update in float64; returns (w, m, v)."""
    b1, b2 = betas
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    bc1 = 1 - b1 ** step
    bc2 = 1 - b2 ** step
    w = w - (lr / bc1) * m / (np.sqrt(v) / np.sqrt(bc2) + eps)
    return w, m, v
