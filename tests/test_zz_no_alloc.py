"""The no-allocation normalisation (hsn_normalize_noalloc) against
hsn_normalize, through the C ABI: two calls in a row on one context, the
second with a smaller input, each equal bit for bit to the allocating entry
point (same kernels, same summation order), with and without the bfloat16
copy, the offset and the bias."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import show

pytestmark = pytest.mark.gpu


def _counts(shape, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    n_v, n_r, n_c, n_k = shape
    y = torch.from_numpy(g.integers(0, 4000, shape, dtype=np.uint16).view(np.int16)).cuda()
    yo = torch.from_numpy(g.integers(1000, 6000, (n_r, n_c, n_k), dtype=np.uint16).view(np.int16)).cuda()
    return y, yo


@pytest.mark.parametrize("mask", [False, True])
def test_noalloc_normalize_matches_allocating_entry(hsn, mask):
    for shape, seed in (((12, 3, 20, 1000), 1), ((5, 2, 7, 96), 2)):   # the second call is smaller
        y, yo = _counts(shape, seed)
        n_v, n_r, n_c, n_k = shape
        bg = None
        if mask:
            bg = torch.zeros((n_r, n_c), dtype=torch.uint8, device="cuda")
            bg[:, :3] = 1
        show("noalloc normalize", shape=shape, mask=mask)
        p0, pb0, b0, ss0, e0 = hsn.hsn_normalize(y, yo, bg_mask=bg, want_bf16=True, want_offset=mask, want_bias=True)
        p1 = torch.full_like(p0, 7.0)
        pb1 = torch.full_like(pb0, 7)
        b1 = torch.empty((n_v, n_k), dtype=torch.float32, device="cuda") if mask else None
        ss1 = torch.empty((), dtype=torch.float64, device="cuda")
        e1 = torch.empty((), dtype=torch.float64, device="cuda")
        hsn.hsn_normalize_noalloc(y, yo, p=p1, p_bf16=pb1, bg_mask=bg, offset_b=b1, sumsq=ss1, bf16_bias=e1)
        torch.cuda.synchronize()
        assert torch.equal(p0[:, :n_k], p1[:, :n_k]) and torch.equal(pb0, pb1)
        assert float(ss0) == float(ss1) and float(e0) == float(e1)
        if mask:
            assert torch.equal(b0, b1)
        # float32 output only (another thread layout than with the padded
        # bfloat16 rows, so its own allocating counterpart)
        p3, _, _, ss3 = hsn.hsn_normalize(y, yo, bg_mask=bg, want_offset=mask)
        p2 = torch.empty_like(p0)
        ss2 = torch.empty((), dtype=torch.float64, device="cuda")
        hsn.hsn_normalize_noalloc(y, yo, p=p2, bg_mask=bg, offset_b=b1, sumsq=ss2)
        assert torch.equal(p3[:, :n_k], p2[:, :n_k]) and float(ss2) == float(ss3)


def test_noalloc_normalize_rejects_mask_without_offset(hsn):
    y, yo = _counts((2, 1, 4, 16), 3)
    bg = torch.ones((1, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(hsn.HsnError):
        hsn.hsn_normalize_noalloc(y, yo, p=torch.empty((8, 16), device="cuda"), bg_mask=bg)
