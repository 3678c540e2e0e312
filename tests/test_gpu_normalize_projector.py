"""GPU parity: -log normalisation (eq. 2, Appendix A), projector A / A^T,
CGLS (eq. 5, h = 0) and subspace expansion (eq. 6) against the FP64 oracle.

Float32 tolerances: normalisation elementwise |d| <= 1e-5 max(|p|, rms p);
operators 1e-5 relative Frobenius (float32 sums of <= 2N taps)."""
import math

import numpy as np
import pytest

import synth
from oracle import cgls as ocgls
from oracle import expand as oexp
from oracle import projector as oprj
from oracle.normalize import normalize as onorm
from tests.gpu_util import bf16_rne, rel_fro, show, to_dev

pytestmark = pytest.mark.gpu


def _check_p(p_gpu, p_ref):
    p_gpu = np.asarray(p_gpu, np.float64)
    rms = math.sqrt(np.mean(p_ref * p_ref))
    bound = 1e-5 * np.maximum(np.abs(p_ref), rms)
    bad = np.abs(p_gpu - p_ref) > bound
    assert not bad.any(), f"{bad.sum()} elements off; worst {np.max(np.abs(p_gpu - p_ref) / bound)}"


@pytest.mark.parametrize("flt", [False, True])
def test_normalize_tiny_config(hsn, flt):
    sc = synth.config_scan("tiny")
    show("normalize tiny", flt=flt)
    y = sc.y.astype(np.float32) if flt else sc.y
    p_ref, _, ss_ref = onorm(sc.y, sc.yo)
    p, pb, _, ss = hsn.hsn_normalize(to_dev(y), to_dev(sc.yo), want_bf16=True)
    n_k = sc.n_bins
    pg = p[:, :n_k].cpu().numpy()
    _check_p(pg, p_ref)
    bits = pb.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(bits[:, :n_k], bf16_rne(pg))
    assert np.all(bits[:, n_k:] == 0)
    assert abs(ss.item() - ss_ref) <= 1e-6 * ss_ref


@pytest.mark.parametrize("n_k", [37, 64])
def test_normalize_ragged_floor_offset_noclip(hsn, n_k):
    # Zero counts, a background mask and no clip; 37 bins (not a multiple of
    # 8: the general kernel) and 64 bins (whole 8-bin chunks: the uint16 fast
    # kernel with the offset and the bfloat16 copy).
    g = np.random.Generator(np.random.PCG64(5))
    n_v, n_r, n_c = 7, 3, 10
    yo = g.poisson(500, (n_r, n_c, n_k)).astype(np.uint16)
    y = g.poisson(300, (n_v, n_r, n_c, n_k)).astype(np.uint16)
    y[0, 0, 0, :5] = 0
    yo[1, 2, 3:6] = 0
    mask = np.zeros((n_r, n_c), np.uint8)
    mask[:, :3] = 1
    show("normalize ragged", n_k=n_k)
    p_ref, b_ref, ss_ref = onorm(y, yo, floor=1.0, bg_mask=mask.astype(bool), clip=False)
    p, pb, b, ss = hsn.hsn_normalize(to_dev(y), to_dev(yo), bg_mask=to_dev(mask), clip=False, want_bf16=True,
                                     want_offset=True)
    _check_p(p[:, :n_k].cpu().numpy(), p_ref)
    assert rel_fro(b.cpu().numpy(), b_ref) <= 1e-6
    assert abs(ss.item() - ss_ref) <= 1e-6 * ss_ref


@pytest.mark.parametrize("n_k,mask", [(1024, False), (64, True), (2000, True)])
def test_normalize_fast_kernel_matches_general(hsn, n_k, mask):
    # 16-byte aligned uint16 counts in whole 8-bin chunks take the fast
    # kernel; the same open beam at an odd address takes the general one
    # (scalar loads).  Same rows per block and summation order: the same p,
    # offset, pooled rows and sum of squares, bit for bit.
    import torch
    g = np.random.Generator(np.random.PCG64(n_k + 3))
    n_v, n_r, n_c = 3, 4, 5
    y = torch.from_numpy(g.integers(0, 4000, (n_v, n_r, n_c, n_k), dtype=np.uint16).view(np.int16)).cuda()
    yo_h = torch.from_numpy(g.integers(1000, 6000, (n_r, n_c, n_k), dtype=np.uint16).view(np.int16))
    yo = yo_h.cuda()
    yo_odd = torch.zeros(n_r * n_c * n_k + 1, dtype=torch.int16, device="cuda")[1:].view(n_r, n_c, n_k)
    yo_odd.copy_(yo)
    assert yo_odd.data_ptr() % 16 != 0
    bg = torch.from_numpy((g.random((n_r, n_c)) < 0.3).astype(np.uint8)).cuda() if mask else None
    if bg is not None:
        bg[0, 0] = 1
    show("normalize fast vs general", n_k=n_k, mask=mask)
    p0, pb0, pooled0, b0, ss0, e0 = hsn.hsn_normalize_pooled(y, yo, hsn.PREC_BF16, bg_mask=bg, want_offset=mask,
                                                              want_bf16=True, want_bias=True)
    p1, pb1, pooled1, b1, ss1, e1 = hsn.hsn_normalize_pooled(y, yo_odd, hsn.PREC_BF16, bg_mask=bg, want_offset=mask,
                                                              want_bf16=True, want_bias=True)
    assert torch.equal(p0[:, :n_k], p1[:, :n_k]) and torch.equal(pooled0, pooled1)
    assert torch.equal(pb0, pb1) and pb0.shape[1] >= n_k   # the padded bfloat16 copy, pad columns zero
    assert not torch.any(pb0[:, n_k:])
    assert float(ss0) == float(ss1) and float(e0) == float(e1)
    if mask:
        assert torch.equal(b0, b1)


def test_normalize_mid_config_sampled_rows(hsn):
    # Full mid-size scan (16 slices, 60 views, 128 columns, 1024 bins) in the
    # launch shape the benchmark uses; the oracle recomputes sampled rows.
    sc = synth.config_scan("mid")
    show("normalize mid", n_p=sc.n_p)
    p, pb, _, ss = hsn.hsn_normalize(to_dev(sc.y), to_dev(sc.yo), want_bf16=True)
    rows = np.random.Generator(np.random.PCG64(0)).choice(sc.n_p, 3000, replace=False)
    yr = sc.y.reshape(-1, sc.n_bins)[rows]
    pix = rows % (sc.n_rows * sc.n_cols)
    yor = sc.yo.reshape(-1, sc.n_bins)[pix]
    ratio = np.maximum(yr.astype(np.float64), 1) / np.maximum(yor.astype(np.float64), 1)
    p_ref = np.maximum(-np.log(ratio), 0)       # eq. (2) with floor 1 and clip, row by row
    _check_p(p[rows].cpu().numpy(), p_ref)
    bits = pb[rows].cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(bits, bf16_rne(p[rows].cpu().numpy()))


@pytest.mark.parametrize("n_k,shape,prec,mask", [(1024, (3, 4, 5), 1, False), (2000, (2, 3, 4), 0, True),
                                                 (300, (2, 2, 7), 1, True), (37, (1, 3, 3), 0, False),
                                                 (256, (5, 1, 9), 1, False),
                                                 (1024, (2, 3, 4), 0, True)])
def test_normalize_pooled_matches_separate_calls(hsn, n_k, shape, prec, mask):
    # The fused pass writes the same p, p_bf16 and offset as hsn_normalize,
    # and pooled rows equal to pooling its p_bf16 with hsn_mlp_pool, bit for
    # bit; the sum of squares agrees to float64 rounding (another order).
    import torch
    g = np.random.Generator(np.random.PCG64(n_k))
    n_v, n_r, n_c = shape
    y = torch.from_numpy(g.integers(0, 4000, (n_v, n_r, n_c, n_k), dtype=np.uint16).view(np.int16)).cuda()
    yo = torch.from_numpy(g.integers(1000, 6000, (n_r, n_c, n_k), dtype=np.uint16).view(np.int16)).cuda()
    bg = torch.from_numpy((g.random((n_r, n_c)) < 0.3).astype(np.uint8)).cuda() if mask else None
    if bg is not None:
        bg[0, 0] = 1
    show("normalize pooled", n_k=n_k, shape=shape, prec=prec, mask=mask)
    p0, pb0, b0, ss0 = hsn.hsn_normalize(y, yo, bg_mask=bg, want_bf16=True, want_offset=mask)
    p1, pb1, pooled, b1, ss1 = hsn.hsn_normalize_pooled(y, yo, prec, bg_mask=bg, want_bf16=True, want_offset=mask)
    assert torch.equal(p0[:, :n_k], p1[:, :n_k]) and torch.equal(pb0, pb1)  # p's pad columns are not written
    if mask:
        assert torch.equal(b0, b1)
    assert abs(float(ss0) - float(ss1)) <= 1e-12 * abs(float(ss0))
    ref = hsn.hsn_mlp_pool(pb0, n_k, prec)
    assert torch.equal(pooled, ref)
    # pooled rows alone (no p, no p_bf16)
    _, _, pooled2, _, _ = hsn.hsn_normalize_pooled(y, yo, prec, bg_mask=bg, want_f32=False)
    assert torch.equal(pooled2, ref)


@pytest.mark.parametrize("n,n_views,k,n_r", [(16, 12, 1, 2), (17, 9, 3, 1), (32, 30, 4, 3), (24, 8, 8, 2),
                                             (33, 7, 5, 1)])
def test_projector_parity_and_adjoint(hsn, n, n_views, k, n_r):
    import torch
    g = np.random.Generator(np.random.PCG64(n * 100 + k))
    x = g.standard_normal((n_r, n, n, k))
    y = g.standard_normal((n_views, n_r, n, k))
    show("projector", n=n, n_views=n_views, k=k)
    s_gpu = hsn.hsn_project(to_dev(x, torch.float32), n_views).cpu().numpy()
    x_gpu = hsn.hsn_backproject(to_dev(y, torch.float32)).cpu().numpy()
    assert rel_fro(s_gpu, oprj.project(x, n_views)) <= 1e-5
    assert rel_fro(x_gpu, oprj.backproject(y, n)) <= 1e-5
    lhs = float(np.sum(s_gpu.astype(np.float64) * y))
    rhs = float(np.sum(x.astype(np.float64) * x_gpu))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(x) * np.linalg.norm(y)


def test_projector_alpha_beta_and_angles(hsn):
    import torch
    g = np.random.Generator(np.random.PCG64(9))
    n, k = 20, 2
    th = np.array([0.0, math.pi / 4, math.pi / 2, 2.0, 3.0])
    x = g.standard_normal((2, n, n, k))
    s0 = g.standard_normal((5, 2, n, k))
    out = to_dev(s0, torch.float32)
    hsn.hsn_project(to_dev(x, torch.float32), 5, angles=th, alpha=0.5, beta=-2.0, out=out)
    ref = 0.5 * oprj.project(x, 5, thetas=th) - 2.0 * s0
    assert rel_fro(out.cpu().numpy(), ref) <= 1e-5


def test_projector_mid_config_shape(hsn):
    # 16 slices of 128 x 128, 60 views, K = 4: the reconstruction shape of the mid workload.
    import torch
    g = np.random.Generator(np.random.PCG64(11))
    x = g.uniform(0, 1, (16, 128, 128, 4))
    show("projector mid")
    s = hsn.hsn_project(to_dev(x, torch.float32), 60).cpu().numpy()
    assert rel_fro(s, oprj.project(x, 60)) <= 1e-5
    y = g.standard_normal((60, 16, 128, 4))
    xb = hsn.hsn_backproject(to_dev(y, torch.float32)).cpu().numpy()
    assert rel_fro(xb, oprj.backproject(y, 128)) <= 1e-5


# Geometries for the launch-shape checks: n * k not a multiple of 4 (scalar
# staging), n not a multiple of 64, view groups padded at both
# orientations, custom angles mixing flat and steep views, one slice; for
# k >= 5 (two staged parts) n a multiple of 4 (grouped float4 copies) and
# not (scalar copies), with both parts' read widths (k = 5, 6, 7, 8).
_SHAPES = [(37, 11, 3, 3, None), (64, 60, 4, 9, None), (50, 13, 5, 2, None),
           (24, 6, 8, 1, [0.0, 0.3, 1.2, 1.9, 2.6, 3.0]), (128, 9, 1, 8, None), (19, 5, 7, 2, None),
           (40, 9, 6, 3, None), (42, 7, 6, 2, None), (64, 12, 5, 3, None)]


@pytest.mark.parametrize("n,n_views,k,n_r,angles", _SHAPES)
def test_projector_launch_shapes_bitwise(hsn, n, n_views, k, n_r, angles):
    # The LDS-staged kernels evaluate every ray and voxel with the arithmetic
    # of the gather kernels; a tap outside the image reads a staged zero
    # where the gather kernel applies weight 0.  With one copy of the ray set
    # per block (split 1) every launch shape must give the same float32
    # values bit for bit; more copies only reorder the sum along each ray.
    import torch
    g = np.random.Generator(np.random.PCG64(n * 31 + k))
    th = None if angles is None else np.array(angles)
    x = to_dev(g.standard_normal((n_r, n, n, k)), torch.float32)
    y = to_dev(g.standard_normal((n_views, n_r, n, k)), torch.float32)
    try:
        hsn.hsn_projector_set_launch(-1, 0, -1, 0)
        assert hsn.hsn_projector_launch_info(n_views, n_r, n, k, angles=th) == (0, 0, 0, 0)
        s_ref = hsn.hsn_project(x, n_views, angles=th).cpu().numpy()
        x_ref = hsn.hsn_backproject(y, angles=th).cpu().numpy()
        assert rel_fro(s_ref, oprj.project(x.cpu().numpy().astype(np.float64), n_views, thetas=th)) <= 1e-5
        assert rel_fro(x_ref, oprj.backproject(y.cpu().numpy().astype(np.float64), n, thetas=th)) <= 1e-5
        for vb in (1, 2, 4):
            for split in (1, 2, 4, 16):
                hsn.hsn_projector_set_launch(vb, split, -1, 0)
                info = hsn.hsn_projector_launch_info(n_views, n_r, n, k, angles=th)
                show("project lds", n=n, n_views=n_views, k=k, n_r=n_r, shape=info)
                assert info[0] == vb and info[1] <= split
                s = hsn.hsn_project(x, n_views, angles=th).cpu().numpy()
                if info[1] == 1:
                    np.testing.assert_array_equal(s, s_ref)
                else:
                    assert rel_fro(s, s_ref) <= 1e-6
        for vpt in (1, 2, 4):
            for nt in (64, 256, 1024):
                hsn.hsn_projector_set_launch(-1, 0, vpt, nt)
                info = hsn.hsn_projector_launch_info(n_views, n_r, n, k, angles=th)
                show("backproject lds", n=n, n_views=n_views, k=k, n_r=n_r, shape=info)
                assert info[2] in (1, vpt)  # several voxels per thread need whole image rows per block
                xb = hsn.hsn_backproject(y, angles=th).cpu().numpy()
                np.testing.assert_array_equal(xb, x_ref)
    finally:
        hsn.hsn_projector_set_launch(0, 0, 0, 0)


def test_projector_launch_knob_errors_and_auto(hsn):
    for bad in ((3, 0, 0, 0), (0, 3, 0, 0), (0, 0, 3, 0), (0, 0, 0, 100), (-2, 0, 0, 0)):
        with pytest.raises(hsn.HsnError):
            hsn.hsn_projector_set_launch(*bad)
    # defaults: LDS-staged kernels at the benchmark shapes
    for geo in ((60, 16, 128, 4), (120, 256, 256, 5)):
        va, sp, vx, nt = hsn.hsn_projector_launch_info(*geo)
        show("auto launch", geo=geo, shape=(va, sp, vx, nt))
        assert va in (1, 2, 4) and sp >= 1 and vx in (1, 2, 4) and 64 <= nt <= 1024
    # a staged row beyond the LDS budget: gather kernels
    assert hsn.hsn_projector_launch_info(4, 1, 2048, 8) == (0, 0, 0, 0)


def test_projector_full_config_slices(hsn):
    # Two slices of the full reconstruction shape (256 x 256, 120 views,
    # K = 5) through the default (LDS-staged) launch against the oracle.
    import torch
    g = np.random.Generator(np.random.PCG64(14))
    x = g.uniform(0, 1, (2, 256, 256, 5))
    show("projector full slices", shape=hsn.hsn_projector_launch_info(120, 2, 256, 5))
    s = hsn.hsn_project(to_dev(x, torch.float32), 120).cpu().numpy()
    assert rel_fro(s, oprj.project(x, 120)) <= 1e-5
    y = g.standard_normal((120, 2, 256, 5))
    xb = hsn.hsn_backproject(to_dev(y, torch.float32)).cpu().numpy()
    assert rel_fro(xb, oprj.backproject(y, 256)) <= 1e-5


def test_cgls_launch_shapes_agree(hsn):
    # The fused sums of squares come from one partial per block, so launch
    # shapes differ in summation order only: the iterates agree to float32
    # rounding.
    import torch
    g = np.random.Generator(np.random.PCG64(15))
    n, nv, k = 40, 24, 5
    b = to_dev(g.standard_normal((nv, 3, n, k)), torch.float32)
    try:
        hsn.hsn_projector_set_launch(-1, 0, -1, 0)
        x0 = hsn.hsn_cgls(b, 4).cpu().numpy()
        for shape in ((1, 1, 1, 64), (2, 4, 2, 256), (4, 16, 4, 1024), (0, 0, 0, 0)):
            hsn.hsn_projector_set_launch(*shape)
            show("cgls launch", shape=shape)
            x = hsn.hsn_cgls(b, 4).cpu().numpy()
            assert rel_fro(x, x0) <= 1e-5
    finally:
        hsn.hsn_projector_set_launch(0, 0, 0, 0)


def test_cgls_parity(hsn):
    # The operator applications are pinned to 1e-5 above.  The CGLS
    # recursion itself amplifies rounding: on this instance a 1e-10 relative
    # perturbation of the A outputs moves the float64 x_20 by 2.5e-4 and
    # float32 arithmetic (emulated on the CPU from the oracle's operators)
    # moves it by 2e-2, with a 12-16% larger residual.  So: the first
    # iterates are compared directly (1e-5), and at 20 iterations the GPU
    # result must be a valid CGLS iterate -- non-increasing residuals and a
    # true residual ||b - A x|| (evaluated by the float64 oracle) within 25%
    # of the float64 oracle's.
    import torch
    g = np.random.Generator(np.random.PCG64(12))
    n, nv, k = 24, 30, 3
    xt = g.uniform(0, 1, (2, n, n, k))
    b = oprj.project(xt, nv) + 0.01 * g.standard_normal((nv, 2, n, k))
    bd = to_dev(b, torch.float32)
    for it in (1, 2, 3):
        x_ref = ocgls.cgls(b, n, it)
        x = hsn.hsn_cgls(bd, it).cpu().numpy()
        show("cgls", it=it, rel=rel_fro(x, x_ref))
        assert rel_fro(x, x_ref) <= 1e-5
    x_ref, res_ref = ocgls.cgls(b, n, 20, history=True)
    x, res = hsn.hsn_cgls(bd, 20, resid=True)
    x = x.cpu().numpy().astype(np.float64)
    res = res.cpu().numpy()
    r = b - oprj.project(x, nv)
    true_res = np.sqrt(np.sum(r * r, axis=(0, 1, 2)))
    show("cgls 20", x_rel=rel_fro(x, x_ref), true_res=true_res / res_ref[-1])
    assert np.all(true_res <= 1.25 * res_ref[-1])
    np.testing.assert_allclose(res[:4], res_ref[:4], rtol=1e-5)
    assert np.all(np.diff(res, axis=0) <= 1e-6 * res_ref[0])


def test_rehydrate_parity(hsn):
    import torch
    g = np.random.Generator(np.random.PCG64(13))
    for k in (1, 4, 5, 8):
        xs = g.standard_normal((1000, k))
        D = g.uniform(0, 1, (700, k))
        out = hsn.hsn_rehydrate(to_dev(xs, torch.float32), to_dev(D, torch.float32), vox=(3, 997), bins=(11, 690))
        ref = oexp.rehydrate(xs, D, vox=(3, 997), bins=(11, 690))
        assert rel_fro(out.cpu().numpy(), ref) <= 1e-6
