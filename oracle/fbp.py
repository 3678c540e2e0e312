"""Filtered backprojection (FBP), K channels at once.  Test infrastructure:
the float64 reference the GPU path is checked against.

The paper uses FBP as the per-bin reconstruction of its baseline (DHR: one
FBP per wavelength bin) and as the cheaper alternative to MBIR in "FHR with
FBP" (subspace reconstruction by FBP of the K sinograms V), Section V and
Tables II and IV, without stating the filter.  Reading: the textbook
parallel-beam FBP with the band-limited ramp filter sampled at the detector
pitch (Ram-Lak),

    h[0] = 1/4,   h[d] = -1 / (pi^2 d^2) for odd d,   h[d] = 0 for even d != 0,

the inverse Fourier transform of |f| on |f| <= 1/2 (Kak and Slaney,
"Principles of Computerized Tomographic Imaging", ch. 3), applied to each
detector row by a linear (zero-padded, not circular) convolution over the
N_c columns:

    q[v][r][c][:] = sum_{c'} h[c - c'] s[v][r][c'][:],

then backprojected with the adjoint A^T of the projector, scaled by the
angular step pi / N_v of the views on [0, pi):

    x = (pi / N_v) A^T q.
"""
from __future__ import annotations

import math

import numpy as np

from .projector import backproject


def ramp_kernel(n_cols: int) -> np.ndarray:
    """h[d] for d = -(n_cols-1) .. n_cols-1 (index d + n_cols - 1)."""
    d = np.arange(-(n_cols - 1), n_cols, dtype=np.int64)
    h = np.zeros(d.shape, np.float64)
    h[d == 0] = 0.25
    odd = (d % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * d[odd].astype(np.float64) ** 2)
    return h


def ramp_filter(sino) -> np.ndarray:
    """q = h * s along the detector columns of every (view, row, channel)."""
    s = np.asarray(sino, np.float64)
    n_cols = s.shape[2]
    h = ramp_kernel(n_cols)
    c = np.arange(n_cols)
    H = h[(c[:, None] - c[None, :]) + n_cols - 1]   # H[c][c'] = h[c - c']
    return np.einsum("cd,vrdk->vrck", H, s)


def fbp(sino, n: int, thetas=None) -> np.ndarray:
    """sino [N_v][N_r][N_c][K] -> x [N_r][N][N][K]."""
    s = np.asarray(sino, np.float64)
    n_v = s.shape[0]
    return (math.pi / n_v) * backproject(ramp_filter(s), n, thetas)
