"""Parity at the full workload's size (256 slices x 256 x 256, 120 views,
2000 bins, K = 5), in the launch configuration the benchmark times, on
outputs the float64 oracle can compute one at a time: sampled rows of p and
of the network's pooled input, sampled rows of V after one ANLS round, the
non-negative least-squares optimality of sampled rows of D, and sampled
slices of A x and A^T s over the whole 256-slice volume (slices are
independent, the launch plan depends on their number)."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp
from oracle import nnls as onnls
from oracle import projector as oprj
from oracle.normalize import normalize as onorm
from tests.gpu_util import bf16_rne, rel_fro, show, to_dev

pytestmark = pytest.mark.gpu

ROWS = [0, 1, 4097, 2_000_003, 3_931_111, 5_555_555, 7_864_319]   # of N_p = 7,864,320
BINS = [0, 977, 1999]


@pytest.fixture(scope="module")
def full_scan(hsn):
    sc = synth.config_scan("full", counts=False)
    show("full scan: counts drawn on the GPU", n_p=sc.n_p, n_k=sc.n_bins)
    y, yo = synth.device_counts(sc, seed=5)
    p, _, pooled, _, _ = hsn.hsn_normalize_pooled(y, yo, hsn.PREC_BF16)
    torch.cuda.synchronize()
    yield sc, y, yo, p, pooled
    del y, yo, p, pooled
    torch.cuda.empty_cache()


def _oracle_rows(sc, y, yo, rows):
    """The oracle's p for single rows of the counts (row r is pixel r mod N_r N_c of view r // (N_r N_c))."""
    out = []
    for r in rows:
        pix = r % (sc.n_rows * sc.n_cols)
        yr = y.view(sc.n_p, sc.n_bins)[r].cpu().numpy().view(np.uint16).reshape(1, 1, 1, -1)
        yor = yo.view(-1, sc.n_bins)[pix].cpu().numpy().view(np.uint16).reshape(1, 1, -1)
        pr, _, _ = onorm(yr, yor)
        out.append(pr[0])
    return np.stack(out)


def _bits_to_f32(bits):
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32)


def test_full_normalize_sampled_rows(hsn, full_scan):
    sc, y, yo, p, pooled = full_scan
    ref = _oracle_rows(sc, y, yo, ROWS)
    got = p[ROWS, :sc.n_bins].cpu().numpy().astype(np.float64)
    rms = np.sqrt(np.mean(ref * ref))
    show("full normalize rows", max_abs=float(np.abs(got - ref).max()), rms=rms)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(np.abs(ref), rms))
    # pooled input: bin means of the bfloat16-rounded p, rounded to bfloat16;
    # within one bfloat16 unit of the oracle's pooling of those values
    ref_pool = omlp.pool(_bits_to_f32(bf16_rne(got.astype(np.float32))).astype(np.float64))
    gp = _bits_to_f32(pooled[ROWS].cpu().numpy().view(np.uint16)).astype(np.float64)
    assert np.all(np.abs(gp - ref_pool) <= 2.0 ** -8 * np.abs(ref_pool) + 1e-30)


def test_full_anls_round(hsn, full_scan):
    # One ANLS round (the polish step) from a seeded start.  V rows against the
    # oracle's exact row NNLS on the oracle's own p rows; D rows must meet the
    # NNLS optimality conditions for the returned V and the kernel's p.
    sc, y, yo, p, _ = full_scan
    K, n_k = 5, sc.n_bins
    V0, D0 = synth.random_factors(sc.n_p, n_k, K, 31)
    V = torch.from_numpy(V0.astype(np.float32)).cuda()
    D = torch.from_numpy(D0.astype(np.float32)).cuda()
    show("full anls round", n_p=sc.n_p, n_k=n_k, k=K)
    hsn.hsn_subspace_nmf(p, None, n_k, V, D, algo=hsn.ALGO_ANLS, max_iter=1, check_every=1)
    d0 = D0.astype(np.float32).astype(np.float64)
    G = d0.T @ d0
    lam_max = np.linalg.eigvalsh(G)[-1]
    P = _oracle_rows(sc, y, yo, ROWS)
    Vr = V[ROWS].cpu().numpy().astype(np.float64)
    for i, r in enumerate(ROWS):
        h = P[i] @ d0
        ref = onnls.nnls_gram(G, h)
        scale = max(np.linalg.norm(ref), np.linalg.norm(h) / lam_max, 1e-30)
        assert np.linalg.norm(Vr[i] - ref) <= 1e-4 * scale, (r, Vr[i], ref)
    V1 = V.cpu().numpy().astype(np.float64)
    GV = V1.T @ V1
    D1 = D.cpu().numpy().astype(np.float64)
    for b in BINS:
        h = V1.T @ p[:, b].cpu().numpy().astype(np.float64)
        grad = GV @ D1[b] - h
        scale = np.abs(h).max()
        show("full anls bin", b=b, d=D1[b], grad=grad / scale)
        assert np.all(D1[b] >= 0.0)
        assert np.all(grad >= -1e-4 * scale), b                 # no descent direction into d >= 0
        on = D1[b] > 1e-6 * max(D1[b].max(), 1e-30)
        assert np.all(np.abs(grad[on]) <= 1e-4 * scale), b       # stationary on the support


def test_full_projector_sampled_slices(hsn):
    n_v, n_r, n, k = 120, 256, 256, 5
    shape = hsn.hsn_projector_launch_info(n_v, n_r, n, k)
    show("full projector", shape=shape)
    assert shape[0] > 0 and shape[2] > 0   # the LDS-staged kernels
    x = synth.random_volume(n_r, n, k, 41).astype(np.float32)
    s = hsn.hsn_project(to_dev(x), n_v)
    for r in (3, 200):
        ref = oprj.project(x[r:r + 1].astype(np.float64), n_v)
        assert rel_fro(s[:, r:r + 1].cpu().numpy(), ref) <= 1e-5, r
    del s
    g = np.random.Generator(np.random.PCG64(42))
    sino = g.standard_normal((n_v, n_r, n, k)).astype(np.float32)
    show("full backprojector")
    xb = hsn.hsn_backproject(to_dev(sino))
    for r in (17, 255):
        ref = oprj.backproject(sino[:, r:r + 1].astype(np.float64), n)
        assert rel_fro(xb[r:r + 1].cpu().numpy(), ref) <= 1e-5, r
