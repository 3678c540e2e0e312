"""Pins for the projector oracle (A of eq. 3/5) and the CGLS oracle (eq. 5, h = 0)."""
import math

import numpy as np
import pytest
from scipy.sparse.linalg import lsqr

from oracle import projector as prj
from oracle.cgls import cgls


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


@pytest.mark.parametrize("n,n_views", [(8, 7), (9, 12), (16, 30)])
def test_adjoint_identity(n, n_views):
    g = _rng(n)
    x = g.standard_normal((2, n, n, 3))
    y = g.standard_normal((n_views, 2, n, 3))
    lhs = np.sum(prj.project(x, n_views) * y)
    rhs = np.sum(x * prj.backproject(y, n))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_dense_matches_matrix_free():
    n, nv = 7, 9
    A = prj.dense_matrix(n, nv)
    g = _rng(2)
    x = g.standard_normal((1, n, n, 1))
    s = prj.project(x, nv)
    np.testing.assert_allclose(s[:, 0, :, 0].ravel(), A @ x[0, :, :, 0].ravel(), rtol=1e-13, atol=1e-13)
    y = g.standard_normal((nv, 1, n, 1))
    xb = prj.backproject(y, n)
    np.testing.assert_allclose(xb[0, :, :, 0].ravel(), A.T @ y[:, 0, :, 0].ravel(), rtol=1e-13, atol=1e-13)


def test_theta0_column_sums_theta90_row_sums():
    n = 12
    g = _rng(3)
    x = g.standard_normal((1, n, n, 1))
    s = prj.project(x, 2)          # views 0 and 90 degrees
    np.testing.assert_allclose(s[0, 0, :, 0], x[0, :, :, 0].sum(axis=0), rtol=1e-15, atol=1e-14)
    np.testing.assert_allclose(s[1, 0, :, 0], x[0, :, :, 0].sum(axis=1), rtol=1e-12, atol=1e-12)


def test_single_pixel_impulse_triangle():
    # one pixel at (x0, y0): its projection at angle t is the triangle of
    # half-width w and height 1/w centred at x0 cos t + y0 sin t.
    n = 15
    x = np.zeros((1, n, n, 1))
    j, i = 9, 4
    x[0, j, i, 0] = 1.0
    th = np.array([0.3, 1.0, 2.2])
    s = prj.project(x, 3, thetas=th)
    for v, t in enumerate(th):
        w = max(abs(math.cos(t)), abs(math.sin(t)))
        centre = (i - (n - 1) / 2) * math.cos(t) + (j - (n - 1) / 2) * math.sin(t)
        sc = np.arange(n) - (n - 1) / 2
        ref = np.maximum(0, 1 - np.abs(sc - centre) / w) / w
        np.testing.assert_allclose(s[v, 0, :, 0], ref, rtol=1e-15, atol=1e-15)


def _disk_area_fractions(n, R, q=64):
    # exact area of the disk inside each pixel by 1D quadrature of the chord
    g = np.arange(n) - (n - 1) / 2
    frac = np.zeros((n, n))
    for i in range(n):
        xs = g[i] - 0.5 + (np.arange(q) + 0.5) / q
        for j in range(n):
            lo, hi = g[j] - 0.5, g[j] + 0.5
            h = np.sqrt(np.maximum(R * R - xs * xs, 0))
            frac[j, i] = np.mean(np.clip(np.minimum(hi, h) - np.maximum(lo, -h), 0, None))
    return frac


def test_disk_theta0_equals_strip_area():
    # At theta = 0 the projection is a column sum; for exact pixel area
    # fractions of a disk that is the strip integral of the chord
    # 2 sqrt(R^2 - t^2): F(s + 1/2) - F(s - 1/2), F(t) = t sqrt(R^2-t^2) + R^2 asin(t/R).
    n, R = 24, 9.3
    x = np.zeros((1, n, n, 1))
    x[0, :, :, 0] = _disk_area_fractions(n, R, q=4096)
    s = prj.project(x, 1)[0, 0, :, 0]

    def F(t):
        t = np.clip(t, -R, R)
        return t * np.sqrt(R * R - t * t) + R * R * np.arcsin(t / R)
    sc = np.arange(n) - (n - 1) / 2
    ref = F(sc + 0.5) - F(sc - 0.5)
    np.testing.assert_allclose(s, ref, atol=2e-5 * R)


def test_disk_chord_first_order_convergence():
    # Same disk at every angle: A f approaches the chord 2 sqrt(R^2 - s^2);
    # the maximum error (over rays well inside the disk) shrinks with R.
    errs = []
    for R in (8.0, 16.0, 32.0):
        n = int(2 * R + 6)
        x = np.zeros((1, n, n, 1))
        x[0, :, :, 0] = _disk_area_fractions(n, R, q=32)
        s = prj.project(x, 8)[:, 0, :, 0]
        sc = np.arange(n) - (n - 1) / 2
        chord = 2 * np.sqrt(np.maximum(R * R - sc * sc, 0))
        inner = np.abs(sc) < 0.7 * R
        errs.append(np.max(np.abs(s[:, inner] - chord[inner])) / (2 * R))
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[2] < 0.01


def test_linearity_and_channels():
    n, nv = 10, 6
    g = _rng(5)
    x1 = g.standard_normal((2, n, n, 3))
    x2 = g.standard_normal((2, n, n, 3))
    a, b = 1.7, -0.4
    np.testing.assert_allclose(prj.project(a * x1 + b * x2, nv),
                               a * prj.project(x1, nv) + b * prj.project(x2, nv), rtol=1e-12, atol=1e-12)
    full = prj.project(x1, nv)
    for ch in range(3):
        np.testing.assert_allclose(full[..., ch:ch + 1], prj.project(x1[..., ch:ch + 1], nv), rtol=1e-15, atol=0)


def test_cgls_matches_lsqr_and_residual_monotone():
    # CGLS and LSQR generate the same Krylov iterates in exact arithmetic.
    n, nv = 8, 10
    A = prj.dense_matrix(n, nv)
    g = _rng(6)
    b = g.standard_normal((nv, 1, n, 1))
    for it in (1, 3, 8):
        x = cgls(b, n, it)
        ref = lsqr(A, b[:, 0, :, 0].ravel(), atol=0, btol=0, conlim=0, iter_lim=it)[0]
        np.testing.assert_allclose(x[0, :, :, 0].ravel(), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    _, hist = cgls(b, n, 20, history=True)
    assert np.all(np.diff(hist[:, 0]) <= 1e-12 * hist[0, 0])


def test_cgls_consistent_data_converges():
    n, nv = 6, 12
    g = _rng(7)
    xt = g.standard_normal((1, n, n, 2))
    b = prj.project(xt, nv)
    x = cgls(b, n, 200)
    np.testing.assert_allclose(x, xt, rtol=1e-8, atol=1e-8)
