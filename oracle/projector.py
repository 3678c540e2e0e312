"""The linear projection operator A of eq. (3)/(5), K channels at once.

The paper names A only as a linear map from a rasterised volume to a
rasterised sinogram.  Reading: parallel-beam Joseph interpolation written
as a closed-form footprint, so that the forward and the adjoint evaluate
the same matrix entries:

    a_{(v,c),(j,i)} = (1/w_v) * max(0, 1 - |d| / w_v)
    d   = s_c - (x_i cos t_v + y_j sin t_v)
    w_v = max(|cos t_v|, |sin t_v|)

with s_c = c - (N_c-1)/2, x_i = i - (N-1)/2, y_j = j - (N-1)/2 and image
size N = N_c.  For |cos| >= |sin| this is Joseph's rule (step along image
rows, linear interpolation between the two nearest columns, path length
1/|cos| per step); otherwise the roles of rows and columns swap.

Layouts: volume x[N_r][N][N][K] (slice r, image row j, column i, channel),
sinogram s[N_v][N_r][N_c][K].  Each detector row r sees slice r only.
"""
from __future__ import annotations

import math

import numpy as np


def angles(n_views: int) -> np.ndarray:
    return np.arange(n_views, dtype=np.float64) * (math.pi / n_views)


def _view_taps(theta: float, n: int, n_cols: int):
    """For one view: for every pixel (j, i), the (at most) two detector
    columns with non-zero weight and their weights; out-of-range columns
    get weight 0."""
    c, s = math.cos(theta), math.sin(theta)
    w = max(abs(c), abs(s))
    g = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    t = g[None, :] * c + g[:, None] * s            # [j][i]
    u = t + (n_cols - 1) / 2.0                      # detector index of the pixel centre
    c0 = np.floor(u)
    taps = []
    for cc in (c0, c0 + 1.0):
        d = (cc - (n_cols - 1) / 2.0) - t
        a = np.maximum(0.0, 1.0 - np.abs(d) / w) / w
        valid = (cc >= 0) & (cc < n_cols)
        taps.append((np.where(valid, cc, 0).astype(np.int64), np.where(valid, a, 0.0)))
    return taps


def project(x, n_views: int, thetas=None):
    """Forward projection s = A x for every slice and channel."""
    x = np.asarray(x, np.float64)
    n_r, n, n2, k = x.shape
    assert n == n2
    n_cols = n
    th = angles(n_views) if thetas is None else np.asarray(thetas, np.float64)
    s = np.zeros((len(th), n_r, n_cols, k))
    for v, theta in enumerate(th):
        for cidx, a in _view_taps(theta, n, n_cols):
            flat_c = cidx.ravel()
            flat_a = a.ravel()
            for r in range(n_r):
                xr = x[r].reshape(n * n, k)
                for ch in range(k):
                    s[v, r, :, ch] += np.bincount(flat_c, weights=flat_a * xr[:, ch], minlength=n_cols)
    return s


def backproject(s, n: int, thetas=None):
    """Adjoint x = A^T s for every slice and channel."""
    s = np.asarray(s, np.float64)
    n_v, n_r, n_cols, k = s.shape
    th = angles(n_v) if thetas is None else np.asarray(thetas, np.float64)
    x = np.zeros((n_r, n, n, k))
    for v, theta in enumerate(th):
        for cidx, a in _view_taps(theta, n, n_cols):
            # x[r, j, i, ch] += a[j, i] * s[v, r, cidx[j, i], ch]
            x += a[None, :, :, None] * s[v][:, cidx, :]
    return x


def dense_matrix(n: int, n_views: int, thetas=None):
    """Dense A (rows (v, c), columns (j, i)) evaluated entry by entry from
    the footprint formula; only for tiny n."""
    th = angles(n_views) if thetas is None else np.asarray(thetas, np.float64)
    g = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    A = np.zeros((len(th) * n, n * n))
    for v, theta in enumerate(th):
        c, s = math.cos(theta), math.sin(theta)
        w = max(abs(c), abs(s))
        for col in range(n):
            sc = col - (n - 1) / 2.0
            for j in range(n):
                for i in range(n):
                    d = sc - (g[i] * c + g[j] * s)
                    A[v * n + col, j * n + i] = max(0.0, 1.0 - abs(d) / w) / w
    return A
