"""Pins of the qGGMRF-MBIR oracle against what the mathematics fixes: closed
forms of the potential, finite differences of the potential and of the cost,
the surrogate's majorisation, a brute-force pair enumeration of the surrogate
Hessian, the least-squares limit of a vanishing prior, and the minimiser
found by an independent optimiser (scipy's L-BFGS-B)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import mbir as om
from oracle import projector as oprj

PARAMS = [(1.0, 1.0, 0.7), (1.2, 1.0, 1.0), (1.5, 0.3, 2.0), (2.0, 1.0, 0.5)]


@pytest.mark.parametrize("p,T,sx", PARAMS)
def test_rho_closed_forms(p, T, sx):
    d = np.array([0.0, 1e-3, 0.1, 0.5, 1.0, 3.0, 50.0])
    r = om.rho(d, p, T, sx)
    assert r[0] == 0.0
    np.testing.assert_array_equal(om.rho(-d, p, T, sx), r)            # even
    if p == 2.0:
        np.testing.assert_allclose(r, d * d / (4.0 * sx * sx), rtol=1e-15)   # u = 1
    if p < 2.0:
        # u = |d / (T sigma)|^(2-p): rho ~ d^2 / (p T^(2-p) sigma^2) as u -> 0 and
        # rho ~ |d|^p / (p sigma^p) as u -> infinity, relative errors about u and 1/u
        small, big = 1e-6 * T * sx, 1e8 * T * sx
        u_s, u_b = 1e-6 ** (2 - p), 1e8 ** (2 - p)
        assert abs(om.rho(small, p, T, sx) / (small ** 2 / (p * T ** (2 - p) * sx ** 2)) - 1.0) <= 2 * u_s
        assert abs(om.rho(big, p, T, sx) / (big ** p / (p * sx ** p)) - 1.0) <= 2 / u_b


@pytest.mark.parametrize("p,T,sx", PARAMS)
def test_rho_prime_is_the_derivative(p, T, sx):
    for d in (-2.3, -0.4, -0.01, 0.02, 0.3, 1.7, 9.0):
        h = 1e-6 * max(1.0, abs(d))
        fd = (om.rho(d + h, p, T, sx) - om.rho(d - h, p, T, sx)) / (2 * h)
        assert abs(om.rho_prime(d, p, T, sx) - fd) <= 1e-6 * max(1.0, abs(fd)), d
    assert om.rho_prime(0.0, p, T, sx) == 0.0
    # the surrogate coefficient is rho'(|d|) / (2 |d|), with the finite limit at 0
    for d in (0.01, 0.4, 3.0):
        assert math.isclose(om.surrogate_coef(d, p, T, sx), om.rho_prime(d, p, T, sx) / (2 * d), rel_tol=1e-12)
    a0 = 1.0 / (p * T ** (2 - p) * sx ** 2) if p < 2.0 else 1.0 / (4.0 * sx ** 2)   # u -> 0, or u = 1 at p = 2
    assert math.isclose(om.surrogate_coef(0.0, p, T, sx), a0, rel_tol=1e-12)


@pytest.mark.parametrize("p,T,sx", PARAMS)
def test_surrogate_majorises_and_touches(p, T, sx):
    g = np.random.Generator(np.random.PCG64(1))
    d0 = g.normal(0, 2 * sx, 300)
    d = g.normal(0, 2 * sx, 300)
    a = om.surrogate_coef(d0, p, T, sx)
    upper = om.rho(d0, p, T, sx) + a * (d * d - d0 * d0)
    assert np.all(om.rho(d, p, T, sx) <= upper + 1e-12 * (1 + np.abs(upper)))
    np.testing.assert_allclose(om.rho(-d0, p, T, sx), om.rho(d0, p, T, sx) + a * 0.0, rtol=1e-15)


def test_prior_apply_matches_brute_force_pairs():
    # The surrogate prior sum_{pairs} b a(anchor) (v_s - v_r)^2 enumerated
    # pixel by pixel over the 8-neighbourhood (each unordered pair once): its
    # gradient 2 sum b a (v_s - v_r) is L v.
    g = np.random.Generator(np.random.PCG64(2))
    n_r, n, k = 2, 5, 3
    xa = g.normal(0, 1, (n_r, n, n, k))
    v = g.normal(0, 1, (n_r, n, n, k))
    p, T, sx = 1.2, 0.8, np.array([0.5, 1.0, 2.0])
    ref = np.zeros_like(v)
    for r in range(n_r):
        for j in range(n):
            for i in range(n):
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        if (dj, di) == (0, 0) or not (0 <= j + dj < n and 0 <= i + di < n):
                            continue
                        b = om.W1 if dj == 0 or di == 0 else om.W1 / math.sqrt(2.0)
                        a = om.surrogate_coef(xa[r, j, i] - xa[r, j + dj, i + di], p, T, sx)
                        ref[r, j, i] += 2 * b * a * (v[r, j, i] - v[r, j + dj, i + di])
    np.testing.assert_allclose(om.prior_apply(xa, v, p, T, sx), ref, rtol=1e-13, atol=1e-13)
    # 8 weights per interior pixel sum to 1
    assert math.isclose(4 * om.W1 + 4 * om.W1 / math.sqrt(2.0), 1.0, rel_tol=1e-15)
    # L is symmetric and annihilates constants
    u = g.normal(0, 1, v.shape)
    lu, lv = om.prior_apply(xa, u, p, T, sx), om.prior_apply(xa, v, p, T, sx)
    np.testing.assert_allclose(np.sum(u * lv, axis=(0, 1, 2)), np.sum(lu * v, axis=(0, 1, 2)), rtol=1e-12)
    assert np.abs(om.prior_apply(xa, np.ones_like(v), p, T, sx)).max() <= 1e-14


def test_cost_gradient_is_the_derivative():
    g = np.random.Generator(np.random.PCG64(3))
    n, nv, k = 6, 8, 2
    x = g.normal(0, 1, (1, n, n, k))
    b = g.normal(0, 1, (nv, 1, n, k))
    sv, sx, p, T = np.array([0.7, 1.3]), np.array([0.4, 1.1]), 1.2, 1.0
    gr = om.grad(x, b, sv, sx, p, T)
    for (j, i, c) in ((0, 0, 0), (2, 3, 1), (5, 5, 0), (3, 1, 1)):
        e = np.zeros_like(x)
        e[0, j, i, c] = 1e-6
        fd = (om.cost(x + e, b, sv, sx, p, T)[c] - om.cost(x - e, b, sv, sx, p, T)[c]) / 2e-6
        assert abs(gr[0, j, i, c] - fd) <= 1e-5 * max(1.0, abs(fd))


def _problem(seed, n=8, nv=12, k=2):
    g = np.random.Generator(np.random.PCG64(seed))
    xt = np.zeros((1, n, n, k))
    xt[0, 2:6, 2:5, 0] = 1.0
    xt[0, 1:4, 3:7, k - 1] += 0.5
    b = oprj.project(xt, nv) + 0.05 * g.standard_normal((nv, 1, n, k))
    return b, n


def test_mm_decreases_the_cost_and_reaches_the_lbfgs_minimiser():
    b, n = _problem(4)
    sv, sx, p, T = np.array([0.1, 0.2]), np.array([0.3, 0.2]), 1.2, 1.0
    x, costs = om.mbir(b, n, sv, sx, p, T, n_outer=60, n_inner=8, history=True)
    assert np.all(np.diff(costs, axis=0) <= 1e-12 * np.abs(costs[:-1]))      # never increases
    for c in range(2):
        def f(z, c=c):
            xx = np.zeros((1, n, n, 2))
            xx[..., c] = z.reshape(1, n, n)
            return om.cost(xx, b, sv, sx, p, T)[c], om.grad(xx, b, sv, sx, p, T)[..., c].ravel()
        res = optimize.minimize(f, np.zeros(n * n), jac=True, method="L-BFGS-B",
                                options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
        z = res.x.reshape(1, n, n)
        assert np.linalg.norm(x[..., c] - z) <= 1e-5 * np.linalg.norm(z), c
        assert costs[-1, c] <= res.fun * (1 + 1e-10)


def test_vanishing_prior_gives_least_squares():
    # sigma_x -> infinity: h -> 0 and the minimiser is the least-squares
    # solution of the dense system (overdetermined: 24 views of an 8 x 8 image).
    b, n = _problem(5, nv=24, k=1)
    x = om.mbir(b, n, 1.0, 1e9, 1.2, 1.0, n_outer=3, n_inner=200)
    A = oprj.dense_matrix(n, 24)
    ref, *_ = np.linalg.lstsq(A, b[:, 0, :, 0].ravel(), rcond=None)
    assert np.linalg.norm(x[0, :, :, 0].ravel() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_quadratic_prior_is_one_linear_solve():
    # p = 2: rho(d) = d^2 / (4 sigma_x^2) for every d, the surrogate is exact
    # and one outer iteration with enough CG steps lands on the solution of
    # (A^T A + sigma_v^2 L) x = A^T b, L the constant-weight graph Laplacian.
    b, n = _problem(6, k=1)
    sv, sx = 0.3, 0.5
    x = om.mbir(b, n, sv, sx, 2.0, 1.0, n_outer=1, n_inner=300)
    A = oprj.dense_matrix(n, 12)
    L = np.zeros((n * n, n * n))
    for dj, di, w in om.PAIRS:
        for j in range(n):
            for i in range(n):
                jj, ii = j + dj, i + di
                if 0 <= jj < n and 0 <= ii < n:
                    s, r = j * n + i, jj * n + ii
                    c = 2 * w / (4 * sx * sx)
                    L[s, s] += c
                    L[r, r] += c
                    L[s, r] -= c
                    L[r, s] -= c
    ref = np.linalg.solve(A.T @ A + sv * sv * L, A.T @ b[:, 0, :, 0].ravel())
    assert np.linalg.norm(x[0, :, :, 0].ravel() - ref) <= 1e-9 * np.linalg.norm(ref)
