"""Per-channel reconstruction (eq. 5) with the prior h = 0.

With h = 0 and a constant noise deviation, eq. (5) reduces to
min_x ||V_j - A x||^2 for every subspace channel j independently.  It is
solved by CGLS (Bjorck's conjugate gradients on the normal equations),
x_0 = 0, a fixed number of iterations, each iteration one A and one A^T.
All K channels advance together but every scalar is per channel.
"""
from __future__ import annotations

import numpy as np

from .projector import backproject, project


def _cdot(a, b):
    """Per-channel inner product (sum over every axis but the last)."""
    return np.sum(a * b, axis=tuple(range(a.ndim - 1)))


def cgls(sino, n: int, n_iter: int, thetas=None, history: bool = False):
    """sino: [N_v][N_r][N_c][K]; returns x [N_r][N][N][K] (and the iterates'
    residual norms per channel if history)."""
    b = np.asarray(sino, np.float64)
    n_v = b.shape[0]
    k = b.shape[-1]
    x = np.zeros((b.shape[1], n, n, k))
    r = b.copy()
    s = backproject(r, n, thetas)
    p = s.copy()
    gamma = _cdot(s, s)
    res = [np.sqrt(_cdot(r, r))]
    for _ in range(n_iter):
        q = project(p, n_v, thetas)
        qq = _cdot(q, q)
        alpha = np.where(qq > 0, gamma / np.where(qq > 0, qq, 1.0), 0.0)
        x = x + alpha * p
        r = r - alpha * q
        s = backproject(r, n, thetas)
        gamma_new = _cdot(s, s)
        beta = np.where(gamma > 0, gamma_new / np.where(gamma > 0, gamma, 1.0), 0.0)
        p = s + beta * p
        gamma = gamma_new
        res.append(np.sqrt(_cdot(r, r)))
    if history:
        return x, np.array(res)
    return x
