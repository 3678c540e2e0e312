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


def _split(A):
    """D' = hi + lo of a float32-valued array: hi = bf16(A), lo = bf16(A - hi),
    the split the MFMA pass multiplies with (exact in float32)."""
    a = np.asarray(A, np.float32)
    hi = _bits_to_f64(bf16_rne(a)).astype(np.float32)
    lo = _bits_to_f64(bf16_rne((a - hi).astype(np.float32))).astype(np.float32)
    return (hi + lo).astype(np.float64)


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
                                          ((5760, 256), 3, "anls"), ((1001, 2000), 5, "anls"),
                                          ((777, 1024), 8, "anls"), ((2053, 512), 4, "anls"), ((100, 64), 1, "anls"),
                                          ((301, 1500), 6, "anls"), ((64, 96), 7, "anls")])
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
    # The bfloat16 ANLS pass solves the V rows exactly for D' = D_hi + D_lo,
    # the split its products use (and reports that solution's objective):
    # the oracle takes the same D'.
    V1, D1, fh, _ = step(pq, V0, _split(D0) if algo == "anls" else D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    code = {"mu": hsn.ALGO_MU, "hals": hsn.ALGO_HALS, "anls": hsn.ALGO_ANLS}[algo]
    st = hsn.hsn_subspace_nmf(None, pb, n_k, V, D, algo=code, precision=hsn.PREC_BF16, max_iter=1, check_every=1)
    ev, ed = rel_fro(V.cpu().numpy(), V1), rel_fro(D.cpu().numpy(), D1)
    # The exact solves (ANLS) map the ~2^-17 relative error of the split
    # products in N_V = P D and N_D = P^T V through G_D = D^T D and
    # G_V = V^T V: their bounds are cond(G) 2^-16.
    tol_v = 2e-5 if algo != "anls" else max(2e-5, np.linalg.cond(D0.T @ D0) * 2.0 ** -16)
    tol_d = 2e-5 if algo != "anls" else max(2e-5, np.linalg.cond(V1.T @ V1) * 2.0 ** -16)
    show("  err", V=ev, D=ed, tol_v=tol_v, tol_d=tol_d, f=abs(st["history"][0] - fh) / fh)
    assert ev <= tol_v and ed <= tol_d
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


def test_normalize_bf16_bias(hsn):
    # -||p - p_bf16||^2 from the normalisation pass equals minus the sum over
    # the returned p and p_bf16 (float64, another order: 1e-9 relative)
    sc = synth.config_scan("tiny")
    y = torch.from_numpy(sc.y.view(np.int16)).cuda()
    yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
    p, pb, _, ss, bias = hsn.hsn_normalize(y, yo, want_bf16=True, want_bias=True)
    n_k = sc.n_bins
    p64 = p[:, :n_k].cpu().numpy().astype(np.float64)
    q64 = _bits_to_f64(pb.cpu().numpy().view(np.uint16)[:, :n_k])
    ref = -float(np.sum((p64 - q64) ** 2))
    show("bf16 bias", gpu=float(bias), ref=ref, sumsq=float(ss))
    assert ref < 0 and abs(float(bias) - ref) <= -1e-9 * ref
    assert abs(float(ss) - float(np.sum(p64 * p64))) <= 1e-12 * float(ss)


def test_bf16_anls_polish_then_fp32_decides_the_stop(hsn):
    # MU bulk on the float32 p, then ANLS polish rounds on p_bf16 until the
    # bias-corrected objective meets the tolerance, then float32 ANLS rounds
    # that confirm (or calibrate the estimate and resume the bfloat16 rounds)
    # and decide the stop on the float32 objective.  The estimate's error,
    # 2 <p - p_bf16, p - V D^T>, spreads by about 2 sqrt(N) 2^-9 |p|
    # sigma_noise: 3e-4 of f* on this 1.5 M-entry scan (relatively less on
    # larger ones), so the tolerance here is 1e-3.
    import json
    import os
    sc = synth.config_scan("tiny")
    p, _, _ = onorm(sc.y, sc.yo)
    p32 = p.astype(np.float32)
    n_p, n_k = p.shape
    pb, bits = _bf16_dev(p32, n_k)
    pq = _bits_to_f64(bits)
    bias = torch.tensor(-float(np.sum((p32.astype(np.float64) - pq) ** 2)), dtype=torch.float64, device="cuda")
    V0, D0 = synth.random_factors(n_p, n_k, 3, 10)
    V0 = V0.astype(np.float32).astype(np.float64)
    D0 = D0.astype(np.float32).astype(np.float64)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nmf_tiny_stationary.json")) as fh:
        f_star = json.load(fh)["f_star"]
    pf = torch.from_numpy(np.ascontiguousarray(np.pad(p32, ((0, 0), (0, (-n_k) % 4))))).cuda()
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    show("bf16 polish + fp32 stop")
    st = hsn.hsn_subspace_nmf(pf, pb, n_k, V, D, max_iter=20, check_every=20, polish_rounds=200,
                              polish_bf16_rounds=150, polish_algo=hsn.ALGO_ANLS, rel_obj_tol=1e-3, f_ref=f_star,
                              bf16_bias=bias)
    show("  done", bf16=st["polish_bf16_done"], total=st["polish_done"], rel=st["rel_obj"])
    assert st["rel_obj"] <= 1e-3
    assert 0 < st["polish_bf16_done"] < 150            # the bfloat16 rounds ended on their own test
    assert st["polish_done"] > st["polish_bf16_done"]  # and float32 rounds made the stop decision
    # the reported objective is the float32 one: f(V, D_prev) >= f(V, D) on the float32 p
    f_end = onmf.objective(p32.astype(np.float64), V.cpu().numpy().astype(np.float64),
                           D.cpu().numpy().astype(np.float64))
    assert f_end <= st["objective"] * (1 + 1e-6)
    assert st["objective"] == st["history"][-1]


def test_bf16_anls_polish_without_stop_runs_every_round(hsn):
    # No stop test: all polish_bf16_rounds bfloat16 rounds run, then the
    # float32 ones; the counts add up.
    p32 = _problem((400, 96), 3, 5)
    n_p, n_k = p32.shape
    pb, _ = _bf16_dev(p32, n_k)
    pf = torch.from_numpy(np.ascontiguousarray(p32)).cuda()
    V0, D0 = synth.random_factors(n_p, n_k, 3, 6)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(pf, pb, n_k, V, D, max_iter=0, polish_rounds=7, polish_bf16_rounds=4,
                              polish_algo=hsn.ALGO_ANLS)
    # ANLS rounds evaluate the objective on every round (on p_bf16 it comes
    # from the row solves at no cost)
    assert st["polish_done"] == 7 and st["polish_bf16_done"] == 4 and len(st["history"]) == 7
    h = st["history"]
    assert np.all(np.diff(h[:4]) <= 1e-6 * h[0]) and np.all(np.diff(h[4:]) <= 1e-6 * h[4])


@pytest.mark.parametrize("algo", ["anls", "hals"])
def test_bf16_polish_rounds_then_fp32_against_oracle(hsn, algo):
    # polish_bf16_rounds honoured for both polish algorithms: 2 rounds on the
    # bfloat16 p, then 1 on the float32 p, against the oracle's same three
    # rounds (on the bfloat16-rounded p, then on p).  Each round adds at most
    # its one-round bound (2e-5, or cond(G) 2^-16 for the exact solves).
    p32 = _problem((400, 96), 3, 5)
    n_p, n_k = p32.shape
    pb, bits = _bf16_dev(p32, n_k)
    pq = _bits_to_f64(bits)
    pf = torch.from_numpy(np.ascontiguousarray(p32)).cuda()
    V0, D0 = synth.random_factors(n_p, n_k, 3, 8)
    V0 = V0.astype(np.float32).astype(np.float64)
    D0 = D0.astype(np.float32).astype(np.float64)
    step = {"anls": onmf.anls_round, "hals": onmf.hals_step}[algo]
    Vr, Dr = V0, D0
    conds = []
    for P in (pq, pq, p32.astype(np.float64)):
        conds.append(max(np.linalg.cond(Dr.T @ Dr), np.linalg.cond(Vr.T @ Vr)))
        Vr, Dr, _, _ = step(P, Vr, Dr)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    code = {"anls": hsn.ALGO_ANLS, "hals": hsn.ALGO_HALS}[algo]
    st = hsn.hsn_subspace_nmf(pf, pb, n_k, V, D, max_iter=0, polish_rounds=3, polish_bf16_rounds=2,
                              polish_algo=code)
    assert st["polish_done"] == 3 and st["polish_bf16_done"] == 2
    ev, ed = rel_fro(V.cpu().numpy(), Vr), rel_fro(D.cpu().numpy(), Dr)
    per = [2e-5 if algo == "hals" else max(2e-5, c * 2.0 ** -16) for c in conds]
    tol = 3 * sum(per)
    show("bf16 polish rounds then fp32", algo=algo, V=ev, D=ed, tol=tol)
    assert ev <= tol and ed <= tol


def test_mid_bf16_bulk_then_fp32_polish_against_oracle(hsn):
    # The mid workload's BF16 schedule (100 MU iterations on the bfloat16 p
    # on MFMA, then 15 float32 ANLS rounds) against the float64 oracle's run
    # of the same schedule, stored by tests/golden/make_mid_bf16_polish.py:
    # canonical D, canonical V on every 240th row within 1e-2, and the final
    # objective within 1e-3.
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mid_bf16_polish.json")) as fh:
        gold = json.load(fh)
    sc = synth.config_scan("mid")
    p, _, _ = onorm(sc.y, sc.yo)
    p32 = p.astype(np.float32)
    n_p, n_k = p.shape
    pb, _ = _bf16_dev(p32, n_k)
    V0, D0 = synth.random_factors(n_p, n_k, sc.n_mat, 52)
    V = to_dev(V0.astype(np.float32), torch.float32)
    D = to_dev(D0.astype(np.float32), torch.float32)
    pf = torch.from_numpy(np.ascontiguousarray(p32)).cuda()
    show("mid bf16 bulk + polish vs oracle", n_p=n_p, n_k=n_k)
    st = hsn.hsn_subspace_nmf(pf, pb, n_k, V, D, algo=hsn.ALGO_MU, precision=hsn.PREC_BF16, max_iter=100,
                              check_every=100, polish_rounds=15, polish_algo=hsn.ALGO_ANLS)
    Vg, Dg = canonical(V.cpu().numpy(), D.cpu().numpy(), library=sc.mu)
    f_end = onmf.objective(p32.astype(np.float64), V.cpu().numpy().astype(np.float64),
                           D.cpu().numpy().astype(np.float64))
    ev = rel_fro(Vg[::gold["row_step"]], np.array(gold["V_canonical_rows"]))
    ed = rel_fro(Dg, np.array(gold["D_canonical"]))
    show("  err", V=ev, D=ed, f=(f_end - gold["f_end"]) / gold["f_end"], rounds=st["polish_done"])
    assert ev <= 1e-2 and ed <= 1e-2
    assert abs(f_end - gold["f_end"]) <= 1e-3 * gold["f_end"]
