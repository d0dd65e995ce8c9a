"""Pins of the FP64 scorer-network reference (oracle/mlp.py): gradients
against central finite differences, GELU against its definition by
quadrature, Adam against a hand-derived first step."""

import math

import numpy as np
from scipy import integrate

from oracle import mlp


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    for k in p:
        p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)
    F = rng.normal(size=(7, mlp.N_IN))
    t = rng.normal(size=7)
    _, g = mlp.loss_and_grads(p, F, t)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(p, F, t)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(p, F, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[i]) <= 1e-7 + 1e-6 * abs(fd), (k, i, fd, g[k].reshape(-1)[i])


def test_gelu_is_x_times_normal_cdf():
    for x in (-3.0, -0.7, 0.0, 0.4, 2.5):
        cdf, _ = integrate.quad(lambda u: math.exp(-0.5 * u * u) / math.sqrt(2 * math.pi), -math.inf, x)
        assert abs(mlp.gelu(np.array([x]))[0] - x * cdf) <= 1e-12
        # derivative by central difference
        h = 1e-6
        fd = (mlp.gelu(np.array([x + h]))[0] - mlp.gelu(np.array([x - h]))[0]) / (2 * h)
        assert abs(fd - mlp.gelu_grad(np.array([x]))[0]) <= 1e-8


def test_adam_first_step_moves_by_lr_times_sign():
    # after one step with bias correction, the update is lr * g / (|g| + eps)
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 0.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    mlp.adam_step(p, g, m, v, 1, lr=0.01)
    expect = np.array([1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8), 0.5])
    assert np.allclose(p["w"], expect, atol=1e-12)


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is halfway between two bf16 values: ties go to the even one (1.0)
    assert mlp.to_bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp.to_bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    vals = np.array([0.1, -3.3, 1e-3, 257.0])
    r = mlp.to_bf16(vals)
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8)
