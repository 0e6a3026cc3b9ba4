"""FP64 reference for the warm-start network.  TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the GPU library shares no code with it.

The network is not part of the paper.  It maps a target spectrum y (n bins) to
a starting point of Algorithm 1, the scalings and weights (log u, log v, w)
the solver reaches for that target, so that the scaling loop starts near its
fixed point instead of at v = 1.  Everything below is the plain textbook
definition, in float64 NumPy:

* multilayer perceptron  x -> GELU(x W1^T + b1) -> GELU(. W2^T + b2) -> . W3^T + b3
  with weights W_l stored [out_l, in_l] row-major and the exact (erf) GELU,
  gelu(z) = z Phi(z), Phi the standard normal CDF;
* weighted mean squared error over every output of a minibatch,
  L = 1 / (B O) sum_b sum_o omega_o (z_bo - t_bo)^2 (omega = 1 unless given),
  and its gradient by the chain rule (backpropagation);
* AdamW (Loshchilov & Hutter, "Decoupled Weight Decay Regularization"):
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd p),
  with the decay applied to every parameter;
* per-column standardisation of inputs and targets with statistics of the
  training set: mean, and standard deviation floored at SD_FLOOR; targets are
  first clamped to [-T_CLAMP, T_CLAMP] (log u is -inf where no dictionary mass
  reaches a bin).

The flat parameter vector is [W1, b1, W2, b2, W3, b3].
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SD_FLOOR = 1e-6
T_CLAMP = 50.0


def param_shapes(dims):
    """[(out, in), (out,), ...] for layer widths dims = (in, h1, h2, out)."""
    shapes = []
    for a, b in zip(dims[:-1], dims[1:]):
        shapes += [(b, a), (b,)]
    return shapes


def n_params(dims):
    return int(sum(np.prod(s) for s in param_shapes(dims)))


def unpack(theta, dims):
    out, o = [], 0
    for s in param_shapes(dims):
        c = int(np.prod(s))
        out.append(np.asarray(theta[o:o + c], dtype=np.float64).reshape(s))
        o += c
    return out


def gelu(z):
    """z Phi(z) with Phi(z) = (1 + erf(z / sqrt 2)) / 2."""
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_prime(z):
    """Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(theta, dims, X):
    """Network output Z3 [B, out] for inputs X [B, in], plus the layer cache."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, dims)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Z3 = H2 @ W3.T + b3
    return Z3, (X, Z1, H1, Z2, H2)


def loss_and_grad(theta, dims, X, T, weights=None):
    """(Weighted) mean squared error over all outputs and its gradient (flat,
    as theta)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, dims)
    Z3, (X, Z1, H1, Z2, H2) = forward(theta, dims, X)
    T = np.asarray(T, dtype=np.float64)
    B, O = Z3.shape
    om = np.ones(O) if weights is None else np.asarray(weights, dtype=np.float64)
    R = Z3 - T
    L = float(np.sum(om * R * R) / (B * O))
    dZ3 = 2.0 * om * R / (B * O)
    dW3 = dZ3.T @ H2
    db3 = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ W3) * gelu_prime(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_prime(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
    return L, g


def adamw(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step (step count t >= 1); returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    theta = theta - lr * (mhat / (np.sqrt(vhat) + eps) + wd * theta)
    return theta, m, v


def column_stats(A, clamp=None):
    """Per-column mean and floored standard deviation (after the clamp)."""
    A = np.asarray(A, dtype=np.float64)
    if clamp is not None:
        A = np.clip(A, -clamp, clamp)
    mu = A.mean(axis=0)
    sd = np.maximum(np.sqrt(np.mean((A - mu) ** 2, axis=0)), SD_FLOOR)
    return mu, sd


def standardise(A, mu, sd, clamp=None):
    A = np.asarray(A, dtype=np.float64)
    if clamp is not None:
        A = np.clip(A, -clamp, clamp)
    return (A - mu) / sd


def predict(theta, dims, Y, in_mu, in_sd, out_mu, out_sd):
    """Raw-unit prediction: standardise y, run the network, undo the target
    standardisation."""
    Z3, _ = forward(theta, dims, standardise(Y, in_mu, in_sd))
    return Z3 * out_sd + out_mu
