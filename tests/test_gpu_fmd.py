"""GPU parity of the fast-material-decomposition tail (Alg. 2, eq. 7-9)
against the FP64 oracle, and the Appendix B identity on exact data.

Both sides start from the same float32 x^s and D^s and compute in float64,
so the only differences are summation order and the final float32
rounding: T and D^m are held to 1e-6 relative, x^m (row NNLS with Gram
T T^T, same active sets) to 1e-5."""
import numpy as np
import pytest
import torch

from oracle import expand as oexp
from tests.gpu_util import rel_fro, show

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n_m,n_x,n_k", [(4, 3, 5000, 300), (6, 5, 20001, 1024), (3, 3, 777, 64), (8, 8, 4096, 2000)])
def test_fmd_matches_oracle(hsn, k, n_m, n_x, n_k):
    g = np.random.Generator(np.random.PCG64(k * 10 + n_m))
    xs = g.uniform(0, 2, (n_x, k)).astype(np.float32)
    labels = g.integers(-1, n_m, n_x).astype(np.int32)
    Ds = g.uniform(0.1, 1, (n_k, k)).astype(np.float32)
    masks = [labels == i for i in range(n_m)]
    T = oexp.transform_matrix(xs.astype(np.float64), masks)
    xm = oexp.material_volumes(xs.astype(np.float64), T)
    Dm = oexp.material_spectra(Ds.astype(np.float64), T)
    show("fmd", k=k, n_m=n_m, n_x=n_x)
    Tg, xmg, Dmg = hsn.hsn_fmd(torch.from_numpy(xs).cuda(), torch.from_numpy(labels).cuda(), n_m,
                               torch.from_numpy(Ds).cuda())
    tol = 1e-5
    show("  err", T=rel_fro(Tg.cpu().numpy(), T), xm=rel_fro(xmg.cpu().numpy(), xm),
         Dm=rel_fro(Dmg.cpu().numpy(), Dm), tol=tol)
    assert rel_fro(Tg.cpu().numpy(), T) <= 1e-6
    assert rel_fro(Dmg.cpu().numpy(), Dm) <= 1e-6
    assert rel_fro(xmg.cpu().numpy(), xm) <= tol
    assert np.all(xmg.cpu().numpy() >= 0)


def test_fmd_appendix_b_identity(hsn):
    # Pure-material voxels define T exactly; mixtures are recovered exactly
    # and D^m = D^s T^T reproduces the material spectra (Appendix B).
    g = np.random.Generator(np.random.PCG64(7))
    k, n_m, n_k = 4, 4, 500
    T_true = g.uniform(0.2, 1.0, (n_m, k))
    Dm_true = g.uniform(0.1, 1.0, (n_k, n_m))
    Ds = np.ascontiguousarray(np.linalg.lstsq(T_true, Dm_true.T, rcond=None)[0].T)  # D^s with D^s T^T = D^m
    pure = np.repeat(np.arange(n_m), 50)
    mix = g.uniform(0, 1, (2000, n_m)) * (g.uniform(0, 1, (2000, n_m)) > 0.4)
    x_true = np.concatenate([np.eye(n_m)[pure], mix])
    xs = x_true @ T_true
    labels = np.concatenate([pure, -np.ones(2000, int)]).astype(np.int32)
    Tg, xmg, Dmg = hsn.hsn_fmd(torch.from_numpy(xs.astype(np.float32)).cuda(), torch.from_numpy(labels).cuda(), n_m,
                               torch.from_numpy(Ds.astype(np.float32)).cuda())
    show("fmd appendix B", T=rel_fro(Tg.cpu().numpy(), T_true), xm=rel_fro(xmg.cpu().numpy(), x_true),
         Dm=rel_fro(Dmg.cpu().numpy(), Dm_true))
    assert rel_fro(Tg.cpu().numpy(), T_true) <= 1e-6
    assert rel_fro(xmg.cpu().numpy(), x_true) <= 1e-4
    assert rel_fro(Dmg.cpu().numpy(), Dm_true) <= 1e-5


def test_fmd_rejects_bad_sizes(hsn):
    xs = torch.zeros((10, 9), device="cuda")
    with pytest.raises(hsn.HsnError):
        hsn.hsn_fmd(xs, torch.zeros(10, dtype=torch.int32, device="cuda"), 2, torch.zeros((5, 9), device="cuda"))
