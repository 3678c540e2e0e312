"""Pins for the -log normalisation oracle (eq. 2, eq. 10, Appendix A)."""
import numpy as np

from oracle.normalize import normalize


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_noiseless_inverse_of_eq10():
    # eq. (10) y = y^o e^{-p} inverted by eq. (2): p is recovered exactly.
    g = _rng(0)
    p = g.uniform(0, 2, (3, 2, 5, 7))
    yo = g.uniform(100, 1000, (2, 5, 7))
    y = yo[None] * np.exp(-p)
    got, b, ss = normalize(y, yo, floor=0.0, clip=False)
    np.testing.assert_allclose(got, p.reshape(-1, 7), rtol=1e-14, atol=1e-14)
    assert b is None
    np.testing.assert_allclose(ss, np.sum(p * p), rtol=1e-15)


def test_offset_recovery_appendix_a():
    # Appendix A: with a dosage mismatch alpha_{v,k} the true projection is
    # p = -log(alpha y / y^o), i.e. the detector sees y = y^o e^{-p} / alpha.
    # On background pixels p = 0, so the offset b = mean_B -log(y/y^o)
    # equals log(alpha), and subtracting it recovers p.
    g = _rng(1)
    n_v, n_r, n_c, n_k = 4, 3, 6, 5
    p = g.uniform(0.1, 2, (n_v, n_r, n_c, n_k))
    bg = np.zeros((n_r, n_c), bool)
    bg[:, :2] = True
    p[:, bg, :] = 0.0
    yo = g.uniform(200, 900, (n_r, n_c, n_k))
    alpha = g.uniform(0.7, 1.4, (n_v, n_k))
    y = yo[None] * np.exp(-p) / alpha[:, None, None, :]
    got, b, _ = normalize(y, yo, floor=0.0, bg_mask=bg, clip=False)
    np.testing.assert_allclose(b, np.log(alpha), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(got, p.reshape(-1, n_k), rtol=1e-13, atol=1e-13)


def test_floor_and_clip():
    y = np.array([0, 5, 20, 10], float).reshape(1, 1, 1, 4)
    yo = np.array([10, 0, 10, 10], float).reshape(1, 1, 4)
    p, _, _ = normalize(y, yo, floor=1.0, clip=False)
    np.testing.assert_allclose(p[0], [np.log(10.0), -np.log(5.0), -np.log(2.0), 0.0], rtol=1e-15)
    pc, _, ss = normalize(y, yo, floor=1.0, clip=True)
    np.testing.assert_allclose(pc[0], [np.log(10.0), 0, 0, 0], rtol=1e-15)
    assert abs(ss - np.log(10.0) ** 2) <= 1e-15 * ss


def test_paper_datapoint_count():
    # The paper's size example: a 512 x 512 x 1200 radiograph holds 3.146e8 values.
    assert abs(512 * 512 * 1200 - 3.146e8) / 3.146e8 < 1e-3
