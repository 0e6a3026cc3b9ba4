"""Pins of the FP64 warm-start network reference against definitions that do
not share its code: a neuron-by-neuron loop for the forward pass, central
finite differences for the gradient, closed forms of GELU and of AdamW."""
import math

import numpy as np
import pytest

from oracle import mlp

DIMS = (5, 4, 3, 6)


def rand_theta(dims, seed):
    return np.random.default_rng(seed).normal(0.0, 0.7, mlp.n_params(dims))


def test_parameter_layout():
    assert mlp.param_shapes(DIMS) == [(4, 5), (4,), (3, 4), (3,), (6, 3), (6,)]
    assert mlp.n_params((1024, 512, 512, 2112)) == 1024 * 512 + 512 + 512 * 512 + 512 + 512 * 2112 + 2112


def test_gelu_closed_forms():
    z = np.linspace(-6, 6, 241)
    # z Phi(z) - (-z) Phi(-z) = z (Phi(z) + Phi(-z)) = z
    np.testing.assert_allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    assert mlp.gelu(0.0) == 0.0 and mlp.gelu_prime(0.0) == 0.5
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-15 and abs(mlp.gelu(-10.0)) < 1e-20
    # Phi(1) from the error function table value erf(1/sqrt 2) = 0.682689492137086
    assert mlp.gelu(1.0) == pytest.approx(0.5 * (1 + 0.682689492137086), rel=1e-14)
    h = 1e-5
    np.testing.assert_allclose(mlp.gelu_prime(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=1e-8, atol=1e-9)


def test_forward_matches_a_neuron_loop():
    theta = rand_theta(DIMS, 1)
    X = np.random.default_rng(2).normal(size=(3, DIMS[0]))
    Z, _ = mlp.forward(theta, DIMS, X)
    Ws = mlp.unpack(theta, DIMS)
    for b in range(3):
        h = list(X[b])
        for layer in range(3):
            W, c = Ws[2 * layer], Ws[2 * layer + 1]
            nxt = []
            for o in range(W.shape[0]):
                z = c[o] + sum(W[o, i] * h[i] for i in range(W.shape[1]))
                nxt.append(z * 0.5 * (1 + math.erf(z / math.sqrt(2))) if layer < 2 else z)
            h = nxt
        np.testing.assert_allclose(Z[b], h, rtol=1e-13, atol=1e-13)


def test_gradient_matches_central_differences():
    theta = rand_theta(DIMS, 3)
    rng = np.random.default_rng(4)
    X, T = rng.normal(size=(7, DIMS[0])), rng.normal(size=(7, DIMS[-1]))
    L, g = mlp.loss_and_grad(theta, DIMS, X, T)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(theta + e, DIMS, X, T)[0] - mlp.loss_and_grad(theta - e, DIMS, X, T)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-7 * np.max(np.abs(fd))
    # the loss is the plain mean of squared residuals
    Z, _ = mlp.forward(theta, DIMS, X)
    assert L == pytest.approx(np.mean((Z - T) ** 2), rel=1e-14)
    assert mlp.loss_and_grad(theta, DIMS, X, Z + 0.25)[0] == pytest.approx(0.0625, rel=1e-12)
    # output weights scale each output's share of the loss; the weighted
    # gradient is the weighted sum of single-output gradients
    om = np.array([0.0, 2.0, 1.0, 0.5, 3.0, 1.0])
    Lw, gw = mlp.loss_and_grad(theta, DIMS, X, T, weights=om)
    assert Lw == pytest.approx(np.mean(om * (Z - T) ** 2), rel=1e-14)
    parts = []
    for o in range(DIMS[-1]):
        e = np.zeros(DIMS[-1])
        e[o] = 1.0
        parts.append(om[o] * mlp.loss_and_grad(theta, DIMS, X, T, weights=e)[1])
    np.testing.assert_allclose(gw, np.sum(parts, axis=0), rtol=1e-10, atol=1e-14)


def test_adamw_closed_forms():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    lr, wd, eps = 0.01, 0.1, 1e-8
    p, m, v = theta.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 4):
        # constant gradient: bias-corrected moments are exactly g and g^2
        expect = p - lr * (g / (np.abs(g) + eps) + wd * p)
        p, m, v = mlp.adamw(p, g, m, v, t, lr, eps=eps, wd=wd)
        np.testing.assert_allclose(p, expect, rtol=1e-12)


def test_column_standardisation():
    rng = np.random.default_rng(5)
    A = rng.normal(3.0, 2.0, (200, 4))
    A[:, 2] = 7.0                      # constant column: floored sd
    A[0, 3] = -np.inf                  # clamped entry
    mu, sd = mlp.column_stats(A, clamp=mlp.T_CLAMP)
    S = mlp.standardise(A, mu, sd, clamp=mlp.T_CLAMP)
    np.testing.assert_allclose(S[:, [0, 1, 3]].mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(S[:, [0, 1, 3]].std(axis=0), 1.0, rtol=1e-12)
    assert sd[2] == mlp.SD_FLOOR and np.all(S[:, 2] == 0.0)
    assert np.isfinite(S).all()
