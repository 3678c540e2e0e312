"""Non-negative least squares in Gram form.

The row problems of the NMF (eq. 4, one factor held fixed) and of the
material estimate (eq. 8) are min_{v >= 0} ||p - D v||^2, equivalently
min_{v >= 0} 1/2 v^T G v - h^T v with G = D^T D and h = D^T p.

`nnls_gram` is the Lawson-Hanson active-set method written in Gram form
with an FP64 Cholesky solve on the passive set; `nnls_brute` enumerates
every support (tiny K) and keeps the one that satisfies the KKT
conditions.  For G positive definite the minimiser is unique, so both
return the same vector up to rounding.
"""
from __future__ import annotations

import itertools

import numpy as np


def _solve_passive(G, h, passive):
    idx = np.flatnonzero(passive)
    z = np.zeros_like(h)
    if idx.size:
        Gs = G[np.ix_(idx, idx)]
        L = np.linalg.cholesky(Gs)
        t = np.linalg.solve(L, h[idx])
        z[idx] = np.linalg.solve(L.T, t)
    return z


def nnls_gram(G, h, tol: float = 1e-12, max_iter: int = 200):
    """Lawson-Hanson active set for min_{v>=0} 1/2 v'Gv - h'v."""
    G = np.asarray(G, np.float64)
    h = np.asarray(h, np.float64)
    k = h.shape[0]
    scale = max(np.abs(h).max(), np.abs(G).max() * 1e-300, 1e-300)
    x = np.zeros(k)
    passive = np.zeros(k, bool)
    w = h - G @ x
    it = 0
    while it < max_iter:
        it += 1
        cand = np.where(~passive, w, -np.inf)
        j = int(np.argmax(cand))
        if not (cand[j] > tol * scale):
            break
        passive[j] = True
        while True:
            z = _solve_passive(G, h, passive)
            if np.all(z[passive] > 0):
                x = z
                break
            neg = passive & (z <= 0)
            alpha = np.min(x[neg] / (x[neg] - z[neg]))
            x = x + alpha * (z - x)
            passive &= x > tol * max(1.0, np.abs(x).max())
            x[~passive] = 0.0
        w = h - G @ x
    return x


def nnls_brute(G, h):
    """Exhaustive search over the 2^K supports (tiny K): the support whose
    unconstrained solution is positive and whose gradient on the
    complement is non-negative is the minimiser."""
    G = np.asarray(G, np.float64)
    h = np.asarray(h, np.float64)
    k = h.shape[0]
    best, best_f = np.zeros(k), 0.0
    for r in range(1, k + 1):
        for S in itertools.combinations(range(k), r):
            S = list(S)
            z = np.zeros(k)
            z[S] = np.linalg.solve(G[np.ix_(S, S)], h[S])
            if np.any(z[S] <= 0):
                continue
            f = 0.5 * z @ G @ z - h @ z
            if f < best_f:
                best, best_f = z, f
    return best


def nnls_rows(G, H):
    """Apply nnls_gram to every row of H (rows are right-hand sides h)."""
    H = np.asarray(H, np.float64)
    out = np.zeros_like(H)
    for i in range(H.shape[0]):
        out[i] = nnls_gram(G, H[i])
    return out
