"""GPU filtered backprojection (hsn_fbp) against the float64 oracle."""
import math

import numpy as np
import pytest

from oracle import fbp as ofbp
from tests.gpu_util import rel_fro, show, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,n_views,k,n_r,angles", [(24, 30, 3, 2, None), (37, 11, 1, 3, None), (64, 60, 4, 2, None),
                                                    (50, 13, 5, 1, [0.0, 0.2, 0.7, 1.1, 1.5, 1.9, 2.2, 2.5, 2.8,
                                                                    2.9, 3.0, 3.05, 3.1]),
                                                    (19, 7, 8, 2, None)])
def test_fbp_parity(hsn, n, n_views, k, n_r, angles):
    import torch
    g = np.random.Generator(np.random.PCG64(n * 7 + k))
    th = None if angles is None else np.array(angles)
    s = g.standard_normal((n_views, n_r, n, k))
    show("fbp", n=n, n_views=n_views, k=k, n_r=n_r)
    x = hsn.hsn_fbp(to_dev(s, torch.float32), n_views, n_r, n, k, angles=th).cpu().numpy()
    assert rel_fro(x, ofbp.fbp(s, n, thetas=th)) <= 1e-5


def test_fbp_reads_bins_of_a_wider_row(hsn):
    # ld > k: k consecutive bins out of rows of ld floats (the DHR use: 8
    # bins of p at a time) give the same values as a contiguous copy.
    import torch
    g = np.random.Generator(np.random.PCG64(21))
    n, n_views, n_r, ld, b0, k = 40, 24, 3, 20, 6, 5
    rows = to_dev(g.standard_normal((n_views * n_r * n, ld)), torch.float32)
    show("fbp strided", ld=ld, b0=b0, k=k)
    x1 = hsn.hsn_fbp(rows[:, b0:], n_views, n_r, n, k, ld=ld)
    x2 = hsn.hsn_fbp(rows[:, b0:b0 + k].contiguous(), n_views, n_r, n, k)
    assert torch.equal(x1, x2)


def test_fbp_reconstructs_a_disk(hsn):
    import torch
    n, n_views, radius = 128, 180, 40.0
    sc = np.arange(n) - (n - 1) / 2.0
    p = np.where(np.abs(sc) < radius, 2.0 * np.sqrt(np.maximum(radius ** 2 - sc ** 2, 0.0)), 0.0)
    s = np.broadcast_to(p[None, None, :, None], (n_views, 1, n, 1)).copy()
    x = hsn.hsn_fbp(to_dev(s, torch.float32), n_views, 1, n, 1).cpu().numpy()[0, :, :, 0]
    g = np.arange(n) - (n - 1) / 2.0
    rr = np.sqrt(g[None, :] ** 2 + g[:, None] ** 2)
    show("fbp disk", inner=float(x[rr < radius - 3].mean()))
    assert abs(x[rr < radius - 3].mean() - 1.0) <= 0.01
    assert abs(x[(rr > radius + 3) & (rr < n / 2 - 2)].mean()) <= 0.01


def test_fbp_mid_config_slices(hsn):
    # 4 slices of the mid reconstruction shape (128 x 128, 60 views, K = 4).
    import torch
    g = np.random.Generator(np.random.PCG64(22))
    s = g.uniform(0, 1, (60, 4, 128, 4))
    x = hsn.hsn_fbp(to_dev(s, torch.float32), 60, 4, 128, 4).cpu().numpy()
    assert rel_fro(x, ofbp.fbp(s, 128)) <= 1e-5


def test_fbp_rejects_bad_arguments(hsn):
    import torch
    s = torch.zeros((4, 1, 16, 2), device="cuda")
    with pytest.raises(hsn.HsnError):
        hsn.hsn_fbp(s, 4, 1, 16, 2, ld=1)
    big = torch.zeros((2, 1, 2048, 8), device="cuda")
    with pytest.raises(hsn.HsnError):
        hsn.hsn_fbp(big, 2, 1, 2048, 8)
