"""Subspace expansion (eq. 6) and the fast-material-decomposition tail.

  rehydrate        x^h = x^s (D^s)^T                     eq. (6)
  transform_matrix T_ij = mean of x^s_{n,j} over M_i     eq. (7)
  material_volumes x^m = argmin_{x>=0} ||x^s - x T||^2   eq. (8), row NNLS
  material_spectra D^m = D^s T^T                         eq. (9)
"""
from __future__ import annotations

import numpy as np

from .nnls import nnls_rows


def rehydrate(xs, D, vox=None, bins=None):
    """xs [N_x][K], D [N_k][K] -> x^h over the selected voxel and bin ranges."""
    xs = np.asarray(xs, np.float64)
    D = np.asarray(D, np.float64)
    if vox is not None:
        xs = xs[vox[0]:vox[1]]
    if bins is not None:
        D = D[bins[0]:bins[1]]
    return xs @ D.T


def transform_matrix(xs, masks):
    """masks: list of N_m index arrays (or boolean masks) over the N_x voxels."""
    xs = np.asarray(xs, np.float64)
    T = np.zeros((len(masks), xs.shape[1]))
    for i, m in enumerate(masks):
        sel = xs[m]
        T[i] = sel.sum(axis=0) / sel.shape[0]
    return T


def material_volumes(xs, T):
    """Row-wise min_{x>=0} ||x^s_n - x T||^2: Gram T T^T, right side T x^s_n."""
    xs = np.asarray(xs, np.float64)
    return nnls_rows(T @ T.T, xs @ T.T)


def material_spectra(D, T):
    return np.asarray(D, np.float64) @ np.asarray(T, np.float64).T
