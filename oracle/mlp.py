"""FP64 reference of the truncation scorer network (test infrastructure only).

Network: f (160) -> z1 = W1 f + b1 (128) -> h1 = GELU(z1) -> z2 = W2 h1 + b2
(128) -> h2 = GELU(z2) -> y = W3 h2 + b3 (1), with the exact GELU
GELU(x) = x * Phi(x), Phi the standard normal CDF.  Loss: mean squared error
over a batch.  Plain numpy matrix products, no fusion; the gradients are
pinned against central finite differences in the CPU tests.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_H = 160, 128


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def init_params(seed: int = 0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, 1 / math.sqrt(N_IN), (N_H, N_IN)),
        "b1": np.zeros(N_H),
        "W2": rng.normal(0, 1 / math.sqrt(N_H), (N_H, N_H)),
        "b2": np.zeros(N_H),
        "W3": rng.normal(0, 1 / math.sqrt(N_H), (1, N_H)),
        "b3": np.zeros(1),
    }


def forward(p, F):
    """F: (B, 160).  Returns y (B,) and the cache for backward."""
    z1 = F @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (F, z1, h1, z2, h2)


def loss_and_grads(p, F, target):
    """MSE loss and its gradients with respect to every parameter."""
    y, (F, z1, h1, z2, h2) = forward(p, F)
    B = F.shape[0]
    r = y - target
    loss = float(np.mean(r * r))
    dy = (2.0 / B) * r[:, None]           # (B,1)
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dh2 = dy @ p["W3"]                    # (B,128)
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = dz1.T @ F
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every parameter in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def to_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
