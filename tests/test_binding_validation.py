"""The Python binding rejects tensors the kernels would misread (wrong
dtype, shape, layout, host memory) with ValueError before any library call.
CPU only: every case here is refused before a device is touched."""
import os

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if not os.path.exists(os.path.join(ROOT, "paper_2410_22500_amd", "libhsn.so")):
    pytest.skip("libhsn.so not built", allow_module_level=True)

from paper_2410_22500_amd import hsn  # noqa: E402


def _nmf(**kw):
    n_p, n_k, k = 40, 24, 3
    args = dict(p=torch.zeros(n_p, 24), p_bf16=None, n_k=n_k, V=torch.zeros(n_p, k), D=torch.zeros(n_k, k))
    args.update(kw)
    return hsn.hsn_subspace_nmf(args.pop("p"), args.pop("p_bf16"), args.pop("n_k"), args.pop("V"), args.pop("D"),
                                **args)


def test_nmf_rejects_wrong_dtype_shape_layout_and_host_memory():
    with pytest.raises(ValueError, match="V must have dtype"):
        _nmf(V=torch.zeros(40, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="D must have shape"):
        _nmf(D=torch.zeros(23, 3))
    with pytest.raises(ValueError, match="D must be contiguous"):
        _nmf(D=torch.zeros(3, 24).t())
    with pytest.raises(ValueError, match="V must be contiguous"):
        _nmf(V=torch.zeros(40, 5)[:, :3])
    with pytest.raises(ValueError, match="p must have shape"):
        _nmf(p=torch.zeros(39, 24))
    with pytest.raises(ValueError, match="p must be a 2-D array of rows"):
        _nmf(p=torch.zeros(24, 40).t())
    with pytest.raises(ValueError, match="p and p_bf16 rows must hold"):
        _nmf(p=torch.zeros(40, 32)[:, :20])
    with pytest.raises(ValueError, match="p_bf16 must have dtype"):
        _nmf(p_bf16=torch.zeros(40, 32))
    with pytest.raises(ValueError, match="must live on a GPU"):
        _nmf()
    # a pitched view of wider rows is a valid p (unit column stride, pitch >= width)
    with pytest.raises(ValueError, match="must live on a GPU"):
        _nmf(p=torch.zeros(40, 32)[:, :24])


def test_normalize_and_projector_arguments():
    y = torch.zeros(4, 2, 8, 16, dtype=torch.int16)
    with pytest.raises(ValueError, match="y_open must have shape"):
        hsn.hsn_normalize(y, torch.zeros(2, 8, 15, dtype=torch.int16))
    with pytest.raises(ValueError, match="y must have dtype"):
        hsn.hsn_normalize(y.to(torch.int32), torch.zeros(2, 8, 16, dtype=torch.int16))
    with pytest.raises(ValueError, match="bg_mask must have"):
        hsn.hsn_normalize(y, torch.zeros(2, 8, 16, dtype=torch.int16), bg_mask=torch.zeros(2, 8))
    with pytest.raises(ValueError, match="x must have shape"):
        hsn.hsn_project(torch.zeros(2, 8, 7, 3), 10)
    with pytest.raises(ValueError, match="x must be contiguous"):
        hsn.hsn_project(torch.zeros(2, 8, 8, 6)[..., :3], 10)
    with pytest.raises(ValueError, match="out must have shape"):
        hsn.hsn_backproject(torch.zeros(10, 2, 8, 3), out=torch.zeros(2, 8, 8, 4))
    with pytest.raises(ValueError, match="sino must be contiguous"):
        hsn.hsn_cgls(torch.zeros(10, 2, 8, 6)[..., ::2], 3)


def test_fbp_extent_and_other_entry_points():
    # 10 views x 1 slice x 8 columns of 4-bin rays at a pitch of 16 floats
    # read (80 - 1) * 16 + 4 floats
    with pytest.raises(ValueError, match="fewer than"):
        hsn.hsn_fbp(torch.zeros(79 * 16 + 3), 10, 1, 8, 4, ld=16)
    with pytest.raises(ValueError, match="must live on a GPU"):
        hsn.hsn_fbp(torch.zeros(79 * 16 + 4), 10, 1, 8, 4, ld=16)
    with pytest.raises(ValueError, match="D must have shape"):
        hsn.hsn_rehydrate(torch.zeros(10, 3), torch.zeros(5, 4))
    with pytest.raises(ValueError, match="labels must have dtype"):
        hsn.hsn_fmd(torch.zeros(10, 3), torch.zeros(10, dtype=torch.int64), 2, torch.zeros(5, 3))
    with pytest.raises(ValueError, match="p_bf16 must have dtype"):
        hsn.hsn_mlp_pool(torch.zeros(4, 32), 32)
    with pytest.raises(ValueError, match="library must have shape"):
        hsn.hsn_canonicalize(torch.zeros(10, 3), torch.zeros(5, 3), library=torch.zeros(5, 2))
    with pytest.raises(ValueError, match=r"problems\[1\].D must have shape"):
        hsn.hsn_subspace_nmf_batched([(torch.zeros(4, 8), 8, torch.zeros(4, 2), torch.zeros(8, 2), 0.0),
                                      (torch.zeros(4, 8), 8, torch.zeros(4, 2), torch.zeros(8, 3), 0.0)])
