"""Pins for the FP64 selector-network reference (no GPU)."""
import math

import numpy as np

from oracle import mlp


def _data(B=16, seed=0):
    g = np.random.default_rng(seed)
    X = g.normal(size=(B, mlp.N_IN))
    Y = np.stack([g.integers(0, 4, B), g.integers(0, 3, B), g.integers(0, 3, B)], axis=1)
    return X, Y


def test_zero_weights_loss_closed_form():
    X, Y = _data()
    theta = np.zeros(mlp.N_PARAM)
    assert mlp.loss(theta, X, Y) == np.float64(math.log(4) + 2 * math.log(3)).item() or \
        abs(mlp.loss(theta, X, Y) - (math.log(4) + 2 * math.log(3))) < 1e-14


def test_gradient_matches_finite_differences():
    X, Y = _data(B=24, seed=3)
    theta = np.random.default_rng(1).normal(scale=0.5, size=mlp.N_PARAM)
    g = mlp.grad(theta, X, Y)
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(len(theta)):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (mlp.loss(theta + e, X, Y) - mlp.loss(theta - e, X, Y)) / (2 * h)
    err = np.abs(num - g).max() / max(np.abs(num).max(), 1e-12)
    assert err <= 1e-6


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=0.1)
    assert np.allclose(th, -0.1 * np.sign(g), rtol=1e-4)


def test_training_reduces_loss():
    X, Y = _data(B=32, seed=5)
    theta = np.random.default_rng(2).normal(scale=0.1, size=mlp.N_PARAM)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, Y)
    for t in range(1, 301):
        theta, m, v = mlp.adam(theta, mlp.grad(theta, X, Y), m, v, t, lr=1e-2)
    assert mlp.loss(theta, X, Y) < 0.5 * l0
