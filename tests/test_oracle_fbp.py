"""Pins of the FBP oracle (ramp filter + scaled adjoint) against what the
mathematics fixes: the band-limited ramp's inverse Fourier transform, the
linear (non-circular) convolution, and the reconstruction of a disk from its
analytic parallel-beam projections."""
import math

import numpy as np
from scipy import integrate

from oracle import fbp as ofbp
from oracle import projector as oprj


def test_ramp_kernel_is_the_band_limited_ramp():
    # h[t] = int_{-1/2}^{1/2} |f| cos(2 pi f t) df, evaluated by quadrature.
    n = 24
    h = ofbp.ramp_kernel(n)
    assert h.shape == (2 * n - 1,)
    for t in range(0, 13):
        q, _ = integrate.quad(lambda f: abs(f) * math.cos(2.0 * math.pi * f * t), -0.5, 0.5, limit=400)
        assert abs(h[t + n - 1] - q) <= 1e-12, t
        assert h[n - 1 - t] == h[n - 1 + t]  # even kernel


def test_ramp_filter_is_a_linear_convolution():
    # An impulse at column c0 gives h[c - c0] on every column, with no
    # wrap-around from the other end (a circular filter would add it).
    n, c0 = 20, 3
    s = np.zeros((1, 1, n, 2))
    s[0, 0, c0, 0] = 1.0
    s[0, 0, n - 1, 1] = 2.0
    q = ofbp.ramp_filter(s)
    h = ofbp.ramp_kernel(n)
    for c in range(n):
        assert abs(q[0, 0, c, 0] - h[c - c0 + n - 1]) <= 1e-15
        assert abs(q[0, 0, c, 1] - 2.0 * h[c - (n - 1) + n - 1]) <= 1e-15


def _disk_sino(n, n_views, radius, value):
    s = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    p = np.where(np.abs(s) < radius, 2.0 * value * np.sqrt(np.maximum(radius * radius - s * s, 0.0)), 0.0)
    return np.broadcast_to(p[None, None, :], (n_views, 1, n)).copy()


def test_fbp_reconstructs_disks():
    # Centred disks (radius 30 of value 1, radius 20 of value 2.5) from their
    # analytic projections 2 v sqrt(R^2 - s^2) over 180 views: the interior
    # is recovered to 1 % and the outside stays near 0.  A wrong angular
    # scale, a dropped centre tap or a circular filter fail this.
    n, n_views = 96, 180
    sino = np.stack([_disk_sino(n, n_views, 30.0, 1.0), _disk_sino(n, n_views, 20.0, 2.5)], axis=-1)
    x = ofbp.fbp(sino, n)
    g = np.arange(n) - (n - 1) / 2.0
    rr = np.sqrt(g[None, :] ** 2 + g[:, None] ** 2)
    for ch, (radius, value) in enumerate(((30.0, 1.0), (20.0, 2.5))):
        img = x[0, :, :, ch]
        inner = img[rr < radius - 3]
        outer = img[(rr > radius + 3) & (rr < n / 2 - 2)]
        assert abs(inner.mean() - value) <= 0.01 * value, (ch, inner.mean())
        assert inner.std() <= 0.02 * value
        assert abs(outer.mean()) <= 0.01 * value


def test_fbp_uses_the_projector_adjoint_scaled_by_the_angular_step():
    g = np.random.Generator(np.random.PCG64(3))
    s = g.standard_normal((12, 2, 16, 3))
    th = oprj.angles(12)
    ref = (math.pi / 12) * oprj.backproject(ofbp.ramp_filter(s), 16, th)
    assert np.allclose(ofbp.fbp(s, 16), ref, rtol=0, atol=1e-13)
