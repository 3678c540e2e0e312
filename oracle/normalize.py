"""-log normalisation (eq. 2) with the Appendix A offset correction.

Readings where the paper is silent:
  * the log is natural (eq. 10 inverts eq. 2 with an exponential);
  * counts are floored at `floor` (default 1) on both y and y^o, since
    -log(0) is undefined;
  * the offset b_{v,k} is the mean over background pixels B of the
    *unclipped* p (Appendix A, offset equation), subtracted before clipping;
  * p is clipped at 0 afterwards when `clip` is set, because the NMF of
    eq. (4) needs a non-negative matrix.
"""
from __future__ import annotations

import numpy as np


def normalize(y, yo, floor: float = 1.0, bg_mask=None, clip: bool = True):
    """Return (p [N_v*N_r*N_c][N_k], b [N_v][N_k] or None, sum(p^2)).

    y  : counts [N_v][N_r][N_c][N_k]
    yo : open beam [N_r][N_c][N_k]
    bg_mask : optional bool/uint8 [N_r][N_c], True on background pixels B.
    """
    y = np.asarray(y, dtype=np.float64)
    yo = np.asarray(yo, dtype=np.float64)
    n_v, n_r, n_c, n_k = y.shape
    assert yo.shape == (n_r, n_c, n_k)
    ratio = np.maximum(y, floor) / np.maximum(yo, floor)[None]
    p = -np.log(ratio)                                   # eq. (2)
    b = None
    if bg_mask is not None:
        m = np.asarray(bg_mask).astype(bool)
        assert m.shape == (n_r, n_c) and m.any()
        # Appendix A: b_{v,k} = (1/|B|) sum_{(r,c) in B} -log(y/y^o)
        b = np.zeros((n_v, n_k))
        for v in range(n_v):
            b[v] = p[v][m].sum(axis=0) / m.sum()
        p = p - b[:, None, None, :]
    if clip:
        p = np.maximum(p, 0.0)
    p = p.reshape(n_v * n_r * n_c, n_k)
    return p, b, float(np.sum(p * p))
