"""GPU qGGMRF-MBIR (hsn_mbir) against the float64 oracle: the same
majorisation-minimisation steps element by element for a few CG iterations
(float32 CG amplifies rounding, so longer runs are checked by the cost and
the distance to the converged minimiser)."""
import numpy as np
import pytest

from oracle import mbir as om
from oracle import projector as oprj
from tests.gpu_util import rel_fro, show, to_dev

pytestmark = pytest.mark.gpu


def _sino(n, n_views, n_r, k, seed, noise=0.05):
    g = np.random.Generator(np.random.PCG64(seed))
    x = np.zeros((n_r, n, n, k))
    for c in range(k):
        j0, i0 = g.integers(1, n // 2, 2)
        x[:, j0:j0 + n // 3, i0:i0 + n // 3, c] = 1.0 + 0.5 * c
    b = oprj.project(x, n_views) + noise * g.standard_normal((n_views, n_r, n, k))
    return b.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,n_views,n_r,k,p,T,outer,inner", [
    (16, 12, 2, 1, 1.2, 1.0, 1, 3), (16, 12, 2, 3, 1.2, 1.0, 2, 2), (19, 9, 1, 8, 1.0, 0.5, 1, 3),
    (24, 30, 2, 4, 2.0, 1.0, 1, 3), (17, 16, 3, 5, 1.5, 2.0, 2, 1)])
def test_mbir_steps_match_oracle(hsn, n, n_views, n_r, k, p, T, outer, inner):
    import torch
    b = _sino(n, n_views, n_r, k, n + k)
    sv = np.linspace(0.05, 0.2, k)
    sx = np.linspace(0.3, 0.8, k)
    show("mbir steps", n=n, n_views=n_views, n_r=n_r, k=k, p=p, T=T, outer=outer, inner=inner)
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, p=p, T=T, n_outer=outer, n_inner=inner).cpu().numpy()
    ref = om.mbir(b, n, sv, sx, p, T, outer, inner)
    assert rel_fro(x, ref) <= 1e-5


def test_mbir_converges_to_the_minimiser(hsn):
    # Parameters for which the oracle's iterations converge within 20 x 6
    # (to 3e-6): 30 x 6 GPU iterations land on the minimiser of the cost
    # (the oracle's 300 x 10 result) to float32 accuracy.
    import torch
    n, n_views, n_r, k = 16, 18, 2, 2
    b = _sino(n, n_views, n_r, k, 3)
    sv, sx, p, T = np.array([0.3, 0.5]), np.array([0.3, 0.4]), 1.2, 1.0
    show("mbir converge")
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, p=p, T=T, n_outer=30, n_inner=6).cpu().numpy()
    ref = om.mbir(b, n, sv, sx, p, T, 300, 10)
    f_gpu = om.cost(x.astype(np.float64), b, sv, sx, p, T)
    f_ref = om.cost(ref, b, sv, sx, p, T)
    show("mbir converge", rel=rel_fro(x, ref), f_gpu=f_gpu, f_ref=f_ref)
    assert np.all(f_gpu <= f_ref * (1 + 1e-5))
    assert rel_fro(x, ref) <= 1e-4


def test_mbir_mid_geometry_slices(hsn):
    # 2 slices of the mid reconstruction shape (128 x 128, 60 views, K = 4)
    # through the LDS-staged operators.
    import torch
    b = _sino(128, 60, 2, 4, 7)
    sv, sx = np.array([0.1, 0.1, 0.2, 0.2]), np.array([0.5, 1.0, 0.5, 1.0])
    show("mbir mid", shape=hsn.hsn_projector_launch_info(60, 2, 128, 4))
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, p=1.2, T=1.0, n_outer=1, n_inner=3).cpu().numpy()
    ref = om.mbir(b, 128, sv, sx, 1.2, 1.0, 1, 3)
    assert rel_fro(x, ref) <= 1e-5


def test_mbir_bench_shape_all_slices(hsn):
    # The benchmark's MBIR launch: all 16 slices of the mid reconstruction
    # (the CG scalars couple the slices, so the whole volume is compared),
    # per-channel parameters, started from a non-zero image.
    import torch
    b = _sino(128, 60, 16, 4, 11)
    g = np.random.Generator(np.random.PCG64(12))
    x0 = (0.1 * g.standard_normal((16, 128, 128, 4))).astype(np.float32)
    sv, sx = np.array([0.05, 0.1, 0.2, 0.4]), np.array([0.3, 0.5, 0.7, 0.9])
    show("mbir bench shape", shape=hsn.hsn_projector_launch_info(60, 16, 128, 4))
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, p=1.2, T=1.0, n_outer=1, n_inner=2,
                     x0=to_dev(x0)).cpu().numpy()
    ref = om.mbir(b, 128, sv, sx, 1.2, 1.0, 1, 2, x0=x0.astype(np.float64))
    assert rel_fro(x, ref) <= 1e-5


def test_mbir_warm_start_and_zero_iterations(hsn):
    import torch
    n, n_views, n_r, k = 16, 12, 1, 2
    b = _sino(n, n_views, n_r, k, 9)
    sv, sx = 0.1, 0.5
    x0 = om.mbir(b, n, sv, sx, 1.2, 1.0, 2, 3)
    x0_32 = x0.astype(np.float32)
    same = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, n_outer=0, n_inner=5, x0=to_dev(x0_32))
    assert np.array_equal(same.cpu().numpy(), x0_32)
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, n_outer=1, n_inner=2, x0=to_dev(x0_32)).cpu().numpy()
    ref = om.mbir(b, n, sv, sx, 1.2, 1.0, 1, 2, x0=x0_32.astype(np.float64))
    assert rel_fro(x, ref) <= 1e-5


def test_mbir_custom_angles_tiny_image(hsn):
    # An image smaller than one 16 x 16 stencil tile (n = 5), one channel,
    # uneven view angles.
    import torch
    th = np.array([0.0, 0.3, 0.9, 1.4, 1.6, 2.2, 2.9])
    g = np.random.Generator(np.random.PCG64(31))
    x = g.uniform(0, 1, (2, 5, 5, 1))
    b = (oprj.project(x, 7, thetas=th) + 0.02 * g.standard_normal((7, 2, 5, 1))).astype(np.float32)
    show("mbir tiny angles")
    # one outer x 3 CG iterations: the element-wise bar of the other step tests (float32 CG
    # amplifies rounding with more steps; longer runs are checked at the minimiser)
    xg = hsn.hsn_mbir(to_dev(b), 0.1, 0.4, p=1.1, T=0.7, n_outer=1, n_inner=3, angles=th).cpu().numpy()
    ref = om.mbir(b.astype(np.float64), 5, 0.1, 0.4, 1.1, 0.7, 1, 3, thetas=th)
    assert rel_fro(xg, ref) <= 1e-5


def test_mbir_quadratic_prior_solves_the_linear_system(hsn):
    # p = 2: the surrogate is exact, so enough CG steps give the solution of
    # (A^T A + sigma_v^2 L) x = A^T b with the constant-weight Laplacian,
    # formed densely here (float32 CG: 1e-4).
    import torch
    n, nv = 10, 14
    b = _sino(n, nv, 1, 1, 5)
    sv, sx = 0.3, 0.5
    show("mbir quadratic")
    x = hsn.hsn_mbir(to_dev(b, torch.float32), sv, sx, p=2.0, T=1.0, n_outer=1, n_inner=100).cpu().numpy()
    A = oprj.dense_matrix(n, nv)
    L = np.zeros((n * n, n * n))
    for dj, di, w in om.PAIRS:
        for j in range(n):
            for i in range(n):
                jj, ii = j + dj, i + di
                if 0 <= jj < n and 0 <= ii < n:
                    s_, r_ = j * n + i, jj * n + ii
                    c = 2 * w / (4 * sx * sx)
                    L[s_, s_] += c
                    L[r_, r_] += c
                    L[s_, r_] -= c
                    L[r_, s_] -= c
    ref = np.linalg.solve(A.T @ A + sv * sv * L, A.T @ b[:, 0, :, 0].ravel())
    assert rel_fro(x[0, :, :, 0].ravel(), ref) <= 1e-4


def test_mbir_rejects_bad_arguments(hsn):
    import torch
    s = torch.zeros((4, 1, 16, 2), device="cuda")
    for kw in (dict(p=0.5), dict(p=2.5), dict(T=0.0), dict(sigma_v=0.0), dict(sigma_x=-1.0), dict(n_outer=-1)):
        args = dict(sigma_v=0.1, sigma_x=0.5)
        args.update(kw)
        with pytest.raises(hsn.HsnError):
            hsn.hsn_mbir(s, **args)
    with pytest.raises(ValueError):
        hsn.hsn_mbir(s, [0.1, 0.2, 0.3], 0.5)
