"""Measures used to judge a decomposition.

  canonical    NMF is unique only up to column permutation and positive
               scaling; D columns are scaled to unit l2 (V inversely) and
               ordered by matching a reference library (or by descending
               column norm of V when there is none)
  snr_fhr      eq. (11): SNR of a hyperspectral reconstruction
  snr_fmd      eq. (12): SNR of material reconstructions
"""
from __future__ import annotations

import itertools

import numpy as np


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


def snr_fhr(recon, material_regions, background):
    """eq. (11), Section V-B: 10 log10 of the mean over bins k and materials
    m of (mu_{m,k} / sigma_k)^2, where mu_{m,k} is the mean of bin k over the
    voxels of material m's region and sigma_k the standard deviation of bin
    k over the background region (outside the sample).
      recon [N_x][N_k]; material_regions: one index array per material;
      background: index array.
    Reading: sigma is the population deviation (divisor n); log base 10 (dB)."""
    recon = np.asarray(recon, np.float64)
    sd = recon[background].std(axis=0, ddof=0)
    ratios = [(recon[reg].mean(axis=0) / sd) ** 2 for reg in material_regions]
    return float(10.0 * np.log10(np.mean(ratios)))


def snr_fmd(xm, material_regions, background):
    """eq. (12), Section V-B: 10 log10 of the mean over materials m of
    (mu_m / sigma_m)^2, where mu_m is the mean of material image m over its
    region and sigma_m the standard deviation of material image m over the
    background region.  xm [N_x][N_m]; regions as snr_fhr."""
    xm = np.asarray(xm, np.float64)
    ratios = [(xm[reg, m].mean() / xm[background, m].std(ddof=0)) ** 2 for m, reg in enumerate(material_regions)]
    return float(10.0 * np.log10(np.mean(ratios)))
