"""Measures used to judge a decomposition.

  rel_obj      (f - f*) / f*, f* = the lowest objective reached for the
               instance (the absolute f/||p||^2 cannot reach 1e-4 on
               Poisson data: the noise floor sits far above it)
  canonical    NMF is unique only up to column permutation and positive
               scaling; D columns are scaled to unit l2 (V inversely) and
               ordered by matching a reference library (or by descending
               column norm of V when there is none)
  snr_db       eq. (11): 10 log10 of the mean over bins and materials of
               (mu_signal / sigma_noise)^2 over homogeneous regions
"""
from __future__ import annotations

import itertools

import numpy as np


def rel_obj(f, f_star):
    return (np.asarray(f, np.float64) - f_star) / f_star


def canonical(V, D, library=None):
    V = np.asarray(V, np.float64)
    D = np.asarray(D, np.float64)
    nrm = np.linalg.norm(D, axis=0)
    nrm = np.where(nrm > 0, nrm, 1.0)
    Dn = D / nrm
    Vn = V * nrm
    k = D.shape[1]
    if library is not None:
        Lb = np.asarray(library, np.float64)
        Lb = Lb / np.linalg.norm(Lb, axis=0)
        cos = Dn.T @ Lb
        best, best_s = None, -np.inf
        for perm in itertools.permutations(range(k)):
            sc = sum(cos[perm[m], m] for m in range(min(k, Lb.shape[1])))
            if sc > best_s:
                best, best_s = perm, sc
        order = list(best)
    else:
        order = list(np.argsort(-np.linalg.norm(Vn, axis=0), kind="stable"))
    return Vn[:, order], Dn[:, order]


def snr_db(recon, truth_regions):
    """recon [N_x][N_k]; truth_regions: list of index arrays, one per
    homogeneous region.  Mean over bins and regions of (mean/std)^2."""
    recon = np.asarray(recon, np.float64)
    vals = []
    for reg in truth_regions:
        sel = recon[reg]
        mu = sel.mean(axis=0)
        sd = sel.std(axis=0)
        vals.append((mu / np.where(sd > 0, sd, np.inf)) ** 2)
    return float(10 * np.log10(np.mean(vals)))
