"""Learned warm start: spectrum -> K non-negative subspace coefficients.

The paper has no learned component; this follows the design chosen for
the warm start:
  pool     adaptive average of each spectrum to 256 bins, bin i covering
           [floor(i N_k / 256), ceil((i + 1) N_k / 256))
  network  256 -> 128 GELU -> 128 GELU -> K softplus
           GELU(z) = z Phi(z) (exact erf form), softplus(z) = max(z,0) + log1p(e^-|z|)
  loss     mean squared error over the batch and the K outputs
  update   Adam (lr, beta1, beta2, eps) on the parameters

Parameter layout (row-major, the order used for flat parameter vectors):
  W1[256][128], b1[128], W2[128][128], b2[128], W3[128][K], b3[K].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN = 256
N_H = 128


def param_shapes(k: int):
    return [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, k), (k,)]


def n_params(k: int) -> int:
    return sum(int(np.prod(s)) for s in param_shapes(k))


def unflatten(theta, k: int):
    out, o = [], 0
    for s in param_shapes(k):
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], np.float64).reshape(s))
        o += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in params])


def pool_bounds(n_k: int, n_out: int = N_IN):
    lo = [(i * n_k) // n_out for i in range(n_out)]
    hi = [-((-(i + 1) * n_k) // n_out) for i in range(n_out)]
    return lo, hi


def pool(P, n_out: int = N_IN):
    P = np.asarray(P, np.float64)
    lo, hi = pool_bounds(P.shape[1], n_out)
    return np.stack([P[:, a:b].mean(axis=1) for a, b in zip(lo, hi)], axis=1)


def gelu(z):
    return z * 0.5 * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    Phi = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(params, x):
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    z3 = h2 @ W3 + b3
    return softplus(z3), (x, z1, h1, z2, h2, z3)


def loss_and_grad(params, x, target):
    W1, b1, W2, b2, W3, b3 = params
    y, (x, z1, h1, z2, h2, z3) = forward(params, x)
    n = y.size
    diff = y - target
    loss = float(np.sum(diff * diff) / n)
    dy = 2.0 * diff / n
    dz3 = dy * sigmoid(z3)
    dW3 = h2.T @ dz3
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ W3.T) * gelu_grad(z2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(theta, grad, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
