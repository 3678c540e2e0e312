"""Per-channel MBIR reconstruction with a qGGMRF prior (eq. 5 with h != 0),
K channels at once.  Test infrastructure: the float64 reference the GPU path
is checked against.

Eq. (5) minimises, for every subspace channel j,

    f(x) = 1/(2 sigma_v^2) ||V_j - A x||^2 + h(x),

with h the q-generalised Gaussian MRF (qGGMRF) prior, whose parameters the
paper does not give.  Readings (all stated, none from the paper):

  * h(x) = sum over unordered neighbour pairs {s, r} of b_sr rho(x_s - x_r),
    the pairs being the 8-neighbourhood inside each slice (slices are
    reconstructed independently, as the parallel-beam data are), pixels
    outside the image omitted; b_sr = w1 for the 4 nearest neighbours and
    w1 / sqrt(2) for the 4 diagonal ones, w1 = 1 / (4 + 2 sqrt(2)), so that a
    pixel's 8 weights sum to 1;
  * rho is the standard qGGMRF potential with q = 2,

        rho(d) = |d|^p / (p sigma_x^p) * u / (1 + u),   u = |d / (T sigma_x)|^(2 - p),

    1 <= p <= 2, T > 0, sigma_x > 0 (per channel), sigma_v > 0 (per channel);
  * no positivity constraint (the subspace images are signed in general);
  * the optimiser is majorisation-minimisation with the symmetric-bound
    quadratic surrogate of rho (rho'(d) / d non-increasing in |d|):

        rho(d) <= rho(d') + a(d') (d^2 - d'^2),   a(d') = rho'(|d'|) / (2 |d'|),

    a(0) = 1 / (p T^(2-p) sigma_x^2) for p < 2 (1 / (4 sigma_x^2) at p = 2,
    where u = 1), so each outer iteration minimises the
    quadratic  1/(2 sigma_v^2) ||V - A x||^2 + sum b_sr a(x'_s - x'_r) (x_s - x_r)^2
    around the current x' by n_inner conjugate-gradient iterations on

        (A^T A + sigma_v^2 L) x = A^T V,   (L v)_s = 2 sum_r b_sr a_sr (v_s - v_r),

    started at x' (every CG step lowers the quadratic, the quadratic lies
    above f and touches it at x', so f never increases).

Layouts as in oracle.projector: x [N_r][N][N][K], sinogram [N_v][N_r][N][K].
"""
from __future__ import annotations

import math

import numpy as np

from .projector import backproject, project

W1 = 1.0 / (4.0 + 2.0 * math.sqrt(2.0))
W2 = W1 / math.sqrt(2.0)
# the 4 "forward" neighbour offsets (dj, di) of the 8-neighbourhood, each
# unordered pair once; the other 4 are their negatives
PAIRS = ((0, 1, W1), (1, 0, W1), (1, 1, W2), (1, -1, W2))


def _ch(v, k):
    return np.broadcast_to(np.asarray(v, np.float64).reshape(-1), (k,))


def rho(d, p: float, T: float, sigma_x):
    """qGGMRF potential (q = 2), elementwise; sigma_x broadcasts over the last axis."""
    a = np.abs(np.asarray(d, np.float64))
    u = (a / (T * sigma_x)) ** (2.0 - p)
    return a ** p / (p * sigma_x ** p) * u / (1.0 + u)


def rho_prime(d, p: float, T: float, sigma_x):
    """d rho / d d (odd in d)."""
    d = np.asarray(d, np.float64)
    a = np.abs(d)
    u = (a / (T * sigma_x)) ** (2.0 - p)
    with np.errstate(divide="ignore", invalid="ignore"):
        mag = a ** (p - 1.0) / sigma_x ** p * u / (1.0 + u) * (1.0 + (2.0 - p) / (p * (1.0 + u)))
    return np.sign(d) * np.where(a > 0, mag, 0.0)


def surrogate_coef(d, p: float, T: float, sigma_x):
    """a(d) = rho'(|d|) / (2 |d|), finite at d = 0 (q = 2)."""
    a = np.abs(np.asarray(d, np.float64))
    u = (a / (T * sigma_x)) ** (2.0 - p)
    return 1.0 / (2.0 * sigma_x ** 2 * T ** (2.0 - p)) / (1.0 + u) * (1.0 + (2.0 - p) / (p * (1.0 + u)))


def _pair_views(x, dj, di):
    """(x_s, x_r) over every pair with r = s + (dj, di) inside the image."""
    n = x.shape[1]
    js, je = max(0, -dj), n - max(0, dj)
    is_, ie = max(0, -di), n - max(0, di)
    return x[:, js:je, is_:ie], x[:, js + dj:je + dj, is_ + di:ie + di], (slice(js, je), slice(is_, ie)), \
        (slice(js + dj, je + dj), slice(is_ + di, ie + di))


def prior_cost(x, p: float, T: float, sigma_x):
    """h(x) per channel [K]."""
    x = np.asarray(x, np.float64)
    sx = _ch(sigma_x, x.shape[-1])
    h = np.zeros(x.shape[-1])
    for dj, di, w in PAIRS:
        xs, xr, _, _ = _pair_views(x, dj, di)
        h += w * rho(xs - xr, p, T, sx).sum(axis=(0, 1, 2))
    return h


def prior_grad(x, p: float, T: float, sigma_x):
    """grad h(x): sum over neighbours r of b_sr rho'(x_s - x_r)."""
    x = np.asarray(x, np.float64)
    sx = _ch(sigma_x, x.shape[-1])
    g = np.zeros_like(x)
    for dj, di, w in PAIRS:
        xs, xr, ss, rs = _pair_views(x, dj, di)
        t = w * rho_prime(xs - xr, p, T, sx)
        g[:, ss[0], ss[1]] += t
        g[:, rs[0], rs[1]] -= t
    return g


def prior_apply(anchor, v, p: float, T: float, sigma_x):
    """L v with the surrogate weights taken at `anchor`:
    (L v)_s = 2 sum_r b_sr a(anchor_s - anchor_r) (v_s - v_r)."""
    xa = np.asarray(anchor, np.float64)
    v = np.asarray(v, np.float64)
    sx = _ch(sigma_x, xa.shape[-1])
    out = np.zeros_like(v)
    for dj, di, w in PAIRS:
        as_, ar, ss, rs = _pair_views(xa, dj, di)
        vs, vr, _, _ = _pair_views(v, dj, di)
        t = 2.0 * w * surrogate_coef(as_ - ar, p, T, sx) * (vs - vr)
        out[:, ss[0], ss[1]] += t
        out[:, rs[0], rs[1]] -= t
    return out


def cost(x, sino, sigma_v, sigma_x, p: float, T: float, thetas=None):
    """f(x) per channel [K]."""
    x = np.asarray(x, np.float64)
    b = np.asarray(sino, np.float64)
    k = x.shape[-1]
    sv = _ch(sigma_v, k)
    res = b - project(x, b.shape[0], thetas)
    return 0.5 * np.sum(res * res, axis=(0, 1, 2)) / sv ** 2 + prior_cost(x, p, T, sigma_x)


def grad(x, sino, sigma_v, sigma_x, p: float, T: float, thetas=None):
    x = np.asarray(x, np.float64)
    b = np.asarray(sino, np.float64)
    n = x.shape[1]
    sv = _ch(sigma_v, x.shape[-1])
    return backproject(project(x, b.shape[0], thetas) - b, n, thetas) / sv ** 2 + prior_grad(x, p, T, sigma_x)


def _cdot(a, b):
    return np.sum(a * b, axis=tuple(range(a.ndim - 1)))


def mbir(sino, n: int, sigma_v, sigma_x, p: float, T: float, n_outer: int, n_inner: int, x0=None,
         thetas=None, history: bool = False):
    """Majorisation-minimisation with n_inner CG iterations per outer
    iteration (see the module docstring).  Returns x [N_r][N][N][K] (and the
    cost per channel after every outer iteration if history)."""
    b = np.asarray(sino, np.float64)
    n_v, n_r = b.shape[0], b.shape[1]
    k = b.shape[-1]
    s2 = _ch(sigma_v, k) ** 2
    x = np.zeros((n_r, n, n, k)) if x0 is None else np.array(x0, np.float64)
    costs = [cost(x, b, sigma_v, sigma_x, p, T, thetas)]
    for _ in range(n_outer):
        xa = x.copy()
        r = backproject(b - project(x, n_v, thetas), n, thetas) - s2 * prior_apply(xa, x, p, T, sigma_x)
        d = r.copy()
        rr = _cdot(r, r)
        for _ in range(n_inner):
            w = backproject(project(d, n_v, thetas), n, thetas) + s2 * prior_apply(xa, d, p, T, sigma_x)
            dw = _cdot(d, w)
            alpha = np.where(dw > 0, rr / np.where(dw > 0, dw, 1.0), 0.0)
            x = x + alpha * d
            r = r - alpha * w
            rr_new = _cdot(r, r)
            beta = np.where(rr > 0, rr_new / np.where(rr > 0, rr, 1.0), 0.0)
            d = r + beta * d
            rr = rr_new
        if history:
            costs.append(cost(x, b, sigma_v, sigma_x, p, T, thetas))
    return (x, np.array(costs)) if history else x
