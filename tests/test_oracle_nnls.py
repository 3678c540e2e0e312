"""Pins for the NNLS oracle: KKT, brute force, scipy, interior solve."""
import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls

from oracle.nnls import nnls_brute, nnls_gram, nnls_rows


def _problem(seed, n=30, k=5):
    g = np.random.Generator(np.random.PCG64(seed))
    D = g.uniform(0, 1, (n, k))
    p = g.standard_normal(n) + 0.3
    return D, p


@pytest.mark.parametrize("seed", range(20))
def test_kkt_and_bruteforce_and_scipy(seed):
    k = 1 + seed % 6
    D, p = _problem(seed, k=k)
    G, h = D.T @ D, D.T @ p
    v = nnls_gram(G, h)
    g = G @ v - h
    scale = np.abs(h).max()
    assert np.all(v >= 0)
    assert np.all(g >= -1e-12 * scale)
    assert np.all(np.abs(v * g) <= 1e-12 * scale * max(1, np.abs(v).max()))
    np.testing.assert_allclose(v, nnls_brute(G, h), rtol=1e-12, atol=1e-12)
    ref, _ = scipy_nnls(D, p)
    np.testing.assert_allclose(v, ref, rtol=1e-10, atol=1e-10)


def test_interior_equals_unconstrained():
    g = np.random.Generator(np.random.PCG64(7))
    D = g.uniform(0, 1, (40, 4))
    v_true = g.uniform(0.5, 2, 4)
    p = D @ v_true
    v = nnls_gram(D.T @ D, D.T @ p)
    np.testing.assert_allclose(v, np.linalg.lstsq(D, p, rcond=None)[0], rtol=1e-12)
    np.testing.assert_allclose(v, v_true, rtol=1e-10)


def test_all_negative_rhs_gives_zero():
    G = np.eye(3) * 2.0
    assert np.all(nnls_gram(G, -np.ones(3)) == 0)


def test_rows():
    D, _ = _problem(3, k=4)
    g = np.random.Generator(np.random.PCG64(9))
    H = g.standard_normal((6, 4))
    out = nnls_rows(D.T @ D, H)
    for i in range(6):
        np.testing.assert_allclose(out[i], nnls_brute(D.T @ D, H[i]), rtol=1e-12, atol=1e-12)
