"""GPU parity of the bfloat16 MFMA pass (eq. 4 bulk iterations).

The bfloat16 pass reads the bfloat16 copy of p (round-to-nearest-even of the
float32 p) and keeps D and V as float32 split into bfloat16 hi + lo halves,
accumulating in float32.  Its reference is the FP64 oracle applied to the
same bfloat16-rounded p: the split products carry ~2^-17 relative error and
the float32 accumulation over <= 2048 bins stays below that, so one step is
held to 2e-5 relative (Frobenius).  After the float32 polish the canonical
coefficients are held to the 1e-2 bound against the oracle running the same
schedule in FP64."""
import numpy as np
import pytest
import torch

import synth
from oracle import nmf as onmf
from oracle.metrics import canonical
from oracle.normalize import normalize as onorm
from tests.gpu_util import bf16_rne, rel_fro, show, to_dev

pytestmark = pytest.mark.gpu


def _bf16_dev(p32, n_k, ldb=None):
    n_p = p32.shape[0]
    ldb = ldb or (n_k + 31) // 32 * 32
    bits = np.zeros((n_p, ldb), np.uint16)
    bits[:, :n_k] = bf16_rne(p32)
    return torch.from_numpy(bits.view(np.int16)).cuda(), bits[:, :n_k]


def _bits_to_f64(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _problem(shape, k, seed):
    n_p, n_k = shape
    if shape == (5760, 256):
        sc = synth.config_scan("tiny")
        p, _, _ = onorm(sc.y, sc.yo)
    else:
        g = np.random.Generator(np.random.PCG64(seed))
        p = np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k)) + 0.1 * g.standard_normal((n_p, n_k)), 0)
    return p.astype(np.float32)


@pytest.mark.parametrize("shape,k,algo", [((5760, 256), 3, "mu"), ((1001, 2000), 5, "mu"), ((777, 1024), 8, "hals"),
                                          ((5760, 256), 3, "hals"), ((100, 64), 1, "mu"), ((2053, 512), 4, "mu"),
                                          ])
def test_bf16_one_step(hsn, shape, k, algo):
    n_p, n_k = shape
    p32 = _problem(shape, k, n_k + k)
    pb, bits = _bf16_dev(p32, n_k)
    pq = _bits_to_f64(bits)
    V0, D0 = synth.random_factors(n_p, n_k, k, 31)
    V0 = V0.astype(np.float32).astype(np.float64)
    D0 = D0.astype(np.float32).astype(np.float64)
    show("bf16 one step", n_p=n_p, n_k=n_k, k=k, algo=algo)
    step = {"mu": onmf.mu_step, "hals": onmf.hals_step, "anls": onmf.anls_round}[algo]
    V1, D1, fh, _ = step(pq, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    code = {"mu": hsn.ALGO_MU, "hals": hsn.ALGO_HALS, "anls": hsn.ALGO_ANLS}[algo]
    st = hsn.hsn_subspace_nmf(None, pb, n_k, V, D, algo=code, precision=hsn.PREC_BF16, max_iter=1, check_every=1)
    ev, ed = rel_fro(V.cpu().numpy(), V1), rel_fro(D.cpu().numpy(), D1)
    # The exact D solve (ANLS) maps the ~2^-17 relative error of the split
    # products in N_D = P^T V through G_V = V^T V: its bound is cond(G_V) 2^-16.
    tol_d = 2e-5 if algo != "anls" else max(2e-5, np.linalg.cond(V1.T @ V1) * 2.0 ** -16)
    show("  err", V=ev, D=ed, tol_d=tol_d, f=abs(st["history"][0] - fh) / fh)
    assert ev <= 2e-5 and ed <= tol_d
    assert abs(st["history"][0] - fh) <= 2e-5 * fh


def test_bf16_bulk_then_fp32_polish_canonical(hsn):
    # 100 bf16 MU iterations + 15 float32 ANLS rounds against the oracle's
    # float64 run of the same schedule (MU on the bf16-rounded p, ANLS on p).
    sc = synth.config_scan("tiny")
    p, _, _ = onorm(sc.y, sc.yo)
    p32 = p.astype(np.float32)
    n_p, n_k = p.shape
    pb, bits = _bf16_dev(p32, n_k)
    pq = _bits_to_f64(bits)
    V0, D0 = synth.random_factors(n_p, n_k, 3, 32)
    V0 = V0.astype(np.float32).astype(np.float64)
    D0 = D0.astype(np.float32).astype(np.float64)
    Vr, Dr, _, _ = onmf.mu_run(pq, V0, D0, 100)
    for _ in range(15):
        Vr, Dr, _, _ = onmf.anls_round(p32.astype(np.float64), Vr, Dr)
    pf = torch.from_numpy(np.ascontiguousarray(np.pad(p32, ((0, 0), (0, (-n_k) % 4))))).cuda()
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    show("bf16 bulk + polish")
    hsn.hsn_subspace_nmf(pf, pb, n_k, V, D, algo=hsn.ALGO_MU, precision=hsn.PREC_BF16, max_iter=100,
                         check_every=100, polish_rounds=15, polish_algo=hsn.ALGO_ANLS)
    Vg, Dg = canonical(V.cpu().numpy(), D.cpu().numpy(), library=sc.mu)
    Vc, Dc = canonical(Vr, Dr, library=sc.mu)
    show("  err", V=rel_fro(Vg, Vc), D=rel_fro(Dg, Dc))
    assert rel_fro(Vg, Vc) <= 1e-2
    assert rel_fro(Dg, Dc) <= 1e-2


def test_bf16_mid_config_one_step(hsn):
    # Full mid-size workload in the benchmark's launch shape (bfloat16 copy
    # written by the library's own normalisation).
    sc = synth.config_scan("mid")
    y = torch.from_numpy(sc.y.view(np.int16)).cuda()
    yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
    p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
    n_p, n_k = sc.n_p, sc.n_bins
    bits = pb.cpu().numpy().view(np.uint16)[:, :n_k]
    pq = _bits_to_f64(bits)
    V0, D0 = synth.random_factors(n_p, n_k, 4, 33)
    V0 = V0.astype(np.float32).astype(np.float64)
    D0 = D0.astype(np.float32).astype(np.float64)
    show("bf16 mid one step")
    V1, D1, fh, _ = onmf.mu_step(pq, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(None, pb, n_k, V, D, precision=hsn.PREC_BF16, max_iter=1, check_every=1)
    assert rel_fro(V.cpu().numpy(), V1) <= 2e-5
    assert rel_fro(D.cpu().numpy(), D1) <= 2e-5
    assert abs(st["history"][0] - fh) <= 2e-5 * fh


def test_bf16_rejects_wide_rows(hsn):
    V = torch.ones((10, 3), device="cuda")
    D = torch.ones((2100, 3), device="cuda")
    pb = torch.zeros((10, 2112), dtype=torch.int16, device="cuda")
    with pytest.raises(hsn.HsnError) as e:
        hsn.hsn_subspace_nmf(None, pb, 2100, V, D, precision=hsn.PREC_BF16, max_iter=1)
    assert e.value.status == hsn.ERR_SHAPE
