"""GPU parity of the NMF (eq. 4) against the FP64 oracle.

Float32 path: one multiplicative-update step from a shared state, V and D
within 1e-5 relative (Frobenius); 200 steps on the tiny workload, the
product V D^T and every evaluated objective within 1e-5 (the factors
themselves may drift along the flat directions of the factorisation, so
they are compared per step only).  ANLS rounds: exact row-wise NNLS, unique
minimisers, so V and D are compared directly."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import nmf as onmf
from oracle.normalize import normalize as onorm
from tests.gpu_util import rel_fro, show, to_dev

pytestmark = pytest.mark.gpu


def _tiny_p():
    sc = synth.config_scan("tiny")
    p, _, _ = onorm(sc.y, sc.yo)
    return p


def _p_dev(p, ldp=None):
    n_p, n_k = p.shape
    ldp = ldp or (n_k + 3) // 4 * 4
    buf = torch.zeros((n_p, ldp), dtype=torch.float32, device="cuda")
    buf[:, :n_k] = torch.from_numpy(p.astype(np.float32)).cuda()
    return buf


def _as32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("shape,k", [((5760, 256), 3), ((1001, 37), 1), ((777, 1500), 8), ((2048, 1024), 4),
                                     ((95, 2048), 5)])
def test_mu_one_step(hsn, shape, k):
    n_p, n_k = shape
    g = np.random.Generator(np.random.PCG64(n_p + n_k + k))
    if shape == (5760, 256):
        p = _tiny_p()
    else:
        p = np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k)) + 0.1 * g.standard_normal((n_p, n_k)), 0)
    V0, D0 = synth.random_factors(n_p, n_k, k, 7)
    V0, D0, p = _as32(V0), _as32(D0), _as32(p)
    show("mu one step", n_p=n_p, n_k=n_k, k=k)
    V1, D1, fh, ff = onmf.mu_step(p, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=1, check_every=1)
    assert rel_fro(V.cpu().numpy(), V1) <= 1e-5
    assert rel_fro(D.cpu().numpy(), D1) <= 1e-5
    assert abs(st["history"][0] - fh) <= 1e-5 * fh


def test_mu_200_steps_tiny(hsn):
    p = _as32(_tiny_p())
    n_p, n_k = p.shape
    V0, D0 = synth.random_factors(n_p, n_k, 3, 8)
    V0, D0 = _as32(V0), _as32(D0)
    show("mu 200 tiny")
    Vr, Dr, fh, _ = onmf.mu_run(p, V0, D0, 200)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=200, check_every=1)
    h = np.array(st["history"])
    assert len(h) == 200
    np.testing.assert_allclose(h, fh, rtol=1e-5)
    assert rel_fro(V.cpu().numpy() @ D.cpu().numpy().T, Vr @ Dr.T) <= 1e-5
    assert np.all(np.diff(h) <= 1e-6 * h[0])


@pytest.mark.parametrize("passes", [1, 2])
@pytest.mark.parametrize("shape,k", [((5760, 256), 3), ((503, 1100), 6), ((95, 2048), 5), ((1001, 37), 7),
                                     ((333, 64), 8), ((17, 8), 1)])
def test_anls_round(hsn, shape, k, passes):
    # One fused pass (the V rows solved inside the pass by support
    # enumeration) and the two-pass form (N_V pass, Lawson-Hanson row
    # solves, N_D pass) against the oracle's exact block minimisation.
    n_p, n_k = shape
    g = np.random.Generator(np.random.PCG64(k))
    if shape == (5760, 256):
        p = _tiny_p()
    else:
        p = np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k)) + 0.1 * g.standard_normal((n_p, n_k)), 0)
    p = _as32(p)
    V0, D0 = synth.random_factors(n_p, n_k, k, 9)
    V0, D0 = _as32(V0), _as32(D0)
    show("anls round", n_p=n_p, n_k=n_k, k=k, passes=passes)
    V1, D1, fh, ff = onmf.anls_round(p, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    hsn.hsn_nmf_set_launch(passes)
    try:
        st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, algo=hsn.ALGO_ANLS, max_iter=1, check_every=1)
    finally:
        hsn.hsn_nmf_set_launch(0)
    # The exact solves map float32 rounding of N_V = P D and N_D = P^T V
    # (2^-24 relative) through G_D = D^T D and G_V = V^T V: bounds cond(G) 2^-24.
    tol_v = max(1e-5, np.linalg.cond(D0.T @ D0) * 2.0 ** -24)
    tol_d = max(1e-5, np.linalg.cond(V1.T @ V1) * 2.0 ** -24)
    show("  err", V=rel_fro(V.cpu().numpy(), V1), D=rel_fro(D.cpu().numpy(), D1), tol_v=tol_v, tol_d=tol_d)
    assert rel_fro(V.cpu().numpy(), V1) <= tol_v
    assert rel_fro(D.cpu().numpy(), D1) <= tol_d
    assert abs(st["history"][0] - fh) <= 1e-5 * fh


def test_anls_rounds_with_active_constraints(hsn):
    # Rows whose NNLS solutions sit on faces of the orthant (many zeros):
    # p built from sparse non-negative coefficients plus noise, three fused
    # rounds against the oracle, and the fused and two-pass forms agree.
    g = np.random.Generator(np.random.PCG64(77))
    n_p, n_k, k = 2000, 300, 5
    C = g.uniform(0, 1, (n_p, k)) * (g.uniform(0, 1, (n_p, k)) < 0.4)
    p = _as32(np.maximum(C @ g.uniform(0, 1, (k, n_k)) + 0.05 * g.standard_normal((n_p, n_k)), 0))
    V0, D0 = synth.random_factors(n_p, n_k, k, 78)
    V0, D0 = _as32(V0), _as32(D0)
    Vr, Dr = V0, D0
    fhs = []
    for _ in range(3):
        Vr, Dr, fh, _ = onmf.anls_round(p, Vr, Dr)
        fhs.append(fh)
    assert np.mean(Vr == 0) > 0.01  # the case exercises active constraints
    outs = []
    for passes in (1, 2):
        V = to_dev(V0, torch.float32)
        D = to_dev(D0, torch.float32)
        hsn.hsn_nmf_set_launch(passes)
        try:
            st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, algo=hsn.ALGO_ANLS, max_iter=3, check_every=1)
        finally:
            hsn.hsn_nmf_set_launch(0)
        show("anls active", passes=passes, V=rel_fro(V.cpu().numpy(), Vr), D=rel_fro(D.cpu().numpy(), Dr))
        np.testing.assert_allclose(st["history"], fhs, rtol=1e-5)
        assert rel_fro(V.cpu().numpy(), Vr) <= 1e-5 and rel_fro(D.cpu().numpy(), Dr) <= 1e-5
        outs.append(V.cpu().numpy())
    assert rel_fro(outs[0], outs[1]) <= 1e-6


def test_nmf_launch_knob_rejects_bad_values(hsn):
    for bad in (-1, 3):
        with pytest.raises(hsn.HsnError):
            hsn.hsn_nmf_set_launch(bad)


@pytest.mark.parametrize("shape,k", [((5760, 256), 3), ((1001, 1500), 5), ((333, 64), 8)])
def test_hals_sweeps(hsn, shape, k):
    # HALS (the paper's Fast HALS) as the fused pass's row rule: one sweep and
    # five sweeps from a shared start against the oracle's column sweeps.
    n_p, n_k = shape
    g = np.random.Generator(np.random.PCG64(k + 40))
    if shape == (5760, 256):
        p = _tiny_p()
    else:
        p = np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k)) + 0.1 * g.standard_normal((n_p, n_k)), 0)
    p = _as32(p)
    V0, D0 = synth.random_factors(n_p, n_k, k, 12)
    V0, D0 = _as32(V0), _as32(D0)
    show("hals", n_p=n_p, n_k=n_k, k=k)
    V1, D1, fh1, _ = onmf.hals_step(p, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, algo=hsn.ALGO_HALS, max_iter=1, check_every=1)
    assert rel_fro(V.cpu().numpy(), V1) <= 1e-5
    assert rel_fro(D.cpu().numpy(), D1) <= 1e-5
    assert abs(st["history"][0] - fh1) <= 1e-5 * fh1
    Vr, Dr = V0, D0
    fhs = []
    for _ in range(5):
        Vr, Dr, fh, _ = onmf.hals_step(p, Vr, Dr)
        fhs.append(fh)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, algo=hsn.ALGO_HALS, max_iter=5, check_every=1)
    np.testing.assert_allclose(st["history"], fhs, rtol=1e-5)
    assert rel_fro(V.cpu().numpy() @ D.cpu().numpy().T, Vr @ Dr.T) <= 1e-5


def test_polish_after_mu_reaches_reference(hsn):
    # MU bulk then ANLS polish on the float32 p: the objective decreases
    # monotonically and reaches the oracle's stationary value.
    # f* from tests/golden/nmf_tiny_stationary.json, written by
    # tests/golden/make_nmf_stationary.py (the oracle's ANLS to a relative
    # change of 1e-12 from this start, about 8 minutes of CPU).
    p = _as32(_tiny_p())
    n_p, n_k = p.shape
    V0, D0 = synth.random_factors(n_p, n_k, 3, 10)
    V0, D0 = _as32(V0), _as32(D0)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nmf_tiny_stationary.json")) as fh:
        f_star = json.load(fh)["f_star"]
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    show("mu+polish tiny")
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=50, check_every=10, polish_rounds=40,
                              rel_obj_tol=1e-4, f_ref=f_star)
    assert st["rel_obj"] <= 1e-4
    h = np.array(st["history"])
    assert np.all(np.diff(h) <= 1e-6 * h[0])


def test_mu_mid_config_one_step(hsn):
    # Full mid-size workload (122880 x 1024, K = 4) in the benchmark's launch shape.
    sc = synth.config_scan("mid")
    p, _, _ = onorm(sc.y, sc.yo)
    p = _as32(p)
    n_p, n_k = p.shape
    V0, D0 = synth.random_factors(n_p, n_k, 4, 11)
    V0, D0 = _as32(V0), _as32(D0)
    show("mu one step mid")
    V1, D1, fh, _ = onmf.mu_step(p, V0, D0)
    V = to_dev(V0, torch.float32)
    D = to_dev(D0, torch.float32)
    st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=1, check_every=1)
    assert rel_fro(V.cpu().numpy(), V1) <= 1e-5
    assert rel_fro(D.cpu().numpy(), D1) <= 1e-5
    assert abs(st["history"][0] - fh) <= 1e-5 * fh


def test_bad_arguments_raise(hsn):
    V = torch.ones((10, 3), device="cuda")
    D = torch.ones((20, 3), device="cuda")
    p = torch.ones((10, 22), device="cuda")       # pitch 22 is not a multiple of 4
    with pytest.raises(hsn.HsnError) as e:
        hsn.hsn_subspace_nmf(p, None, 20, V, D, max_iter=1)
    assert e.value.status == hsn.ERR_INVALID_ARG
    V9 = torch.ones((10, 9), device="cuda")
    D9 = torch.ones((20, 9), device="cuda")
    with pytest.raises(hsn.HsnError) as e:
        hsn.hsn_subspace_nmf(torch.ones((10, 20), device="cuda"), None, 20, V9, D9, max_iter=1)
    assert e.value.status == hsn.ERR_SHAPE


@pytest.mark.parametrize("algo", ["mu", "anls"])
def test_nan_in_p_stops_with_numeric_error(hsn, algo):
    # A NaN planted in p (host side, ordinary data): the first objective is
    # NaN, the run stops there and the call reports HSN_ERR_NUMERIC.
    g = np.random.Generator(np.random.PCG64(90))
    p = _as32(g.uniform(0, 1, (300, 40)))
    p[123, 7] = np.nan
    V0, D0 = synth.random_factors(300, 40, 3, 91)
    V = to_dev(_as32(V0), torch.float32)
    D = to_dev(_as32(D0), torch.float32)
    code = {"mu": hsn.ALGO_MU, "anls": hsn.ALGO_ANLS}[algo]
    with pytest.raises(hsn.HsnError) as e:
        hsn.hsn_subspace_nmf(_p_dev(p), None, 40, V, D, algo=code, max_iter=50, check_every=1)
    assert e.value.status == hsn.ERR_NUMERIC
    assert "step 0" in str(e.value)


def test_zero_column_in_d_stays_finite(hsn):
    # A zero column of D (a material absent from the start): its Gram is
    # singular; MU keeps the column at zero, ANLS never enters a support with
    # a singular principal submatrix.  Results stay finite and match the oracle.
    g = np.random.Generator(np.random.PCG64(92))
    n_p, n_k, k = 400, 64, 4
    p = _as32(np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k)) + 0.05 * g.standard_normal((n_p, n_k)), 0))
    V0, D0 = synth.random_factors(n_p, n_k, k, 93)
    V0, D0 = _as32(V0), _as32(D0)
    D0[:, 2] = 0.0
    for algo, step in ((hsn.ALGO_MU, onmf.mu_step), (hsn.ALGO_ANLS, onmf.anls_round)):
        V1, D1, fh, _ = step(p, V0, D0)
        V = to_dev(V0, torch.float32)
        D = to_dev(D0, torch.float32)
        st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, algo=algo, max_iter=1, check_every=1)
        Vg, Dg = V.cpu().numpy(), D.cpu().numpy()
        show("zero column", algo=algo, V=rel_fro(Vg, V1), D=rel_fro(Dg, D1))
        assert np.all(np.isfinite(Vg)) and np.all(np.isfinite(Dg))
        assert rel_fro(Vg, V1) <= 1e-5 and rel_fro(Dg, D1) <= 1e-5
        assert abs(st["history"][0] - fh) <= 1e-5 * fh


@pytest.mark.parametrize("passes", [1, 2])
def test_extrapolated_anls_rounds_against_oracle(hsn, passes):
    # Eight extrapolated ANLS rounds (fused pass or two-pass form) from a
    # seeded start against the oracle's run of the same rule: the objective
    # of every round within 1e-5, V and D within 1e-4 (float32 factors
    # between exact float64 solves, carried through the extrapolation).
    g = np.random.Generator(np.random.PCG64(95))
    n_p, n_k, k = 1500, 300, 4
    p = _as32(np.maximum(g.uniform(0, 1, (n_p, k)) @ g.uniform(0, 1, (k, n_k))
                         + 0.05 * g.standard_normal((n_p, n_k)), 0))
    V0, D0 = synth.random_factors(n_p, n_k, k, 96)
    V0, D0 = _as32(V0), _as32(D0)
    Vr, Dr, hr = onmf.anls_extrapolated_run(p, V0, D0, 8)
    hsn.hsn_nmf_set_launch(passes)
    try:
        V = to_dev(V0, torch.float32)
        D = to_dev(D0, torch.float32)
        st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=0, polish_rounds=8,
                                  polish_algo=hsn.ALGO_ANLS, anls_extrapolate=True)
    finally:
        hsn.hsn_nmf_set_launch(0)
    h = np.array(st["history"])
    ev, ed = rel_fro(V.cpu().numpy(), Vr), rel_fro(D.cpu().numpy(), Dr)
    show("extrapolated anls", passes=passes, V=ev, D=ed, h=float(np.max(np.abs(h - hr) / hr)))
    assert h.shape == hr.shape and np.all(np.abs(h - hr) <= 1e-5 * hr)
    assert ev <= 1e-4 and ed <= 1e-4


def test_extrapolated_anls_reaches_reference_in_fewer_rounds(hsn):
    # The tiny scan's stationary reference f*: with the stop test at 1e-4 the
    # extrapolated rounds stop within the tolerance in fewer rounds than the
    # plain ones, and the returned factors are at least as good as the last
    # reported objective.
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nmf_tiny_stationary.json")) as fh:
        f_star = json.load(fh)["f_star"]
    p = _tiny_p()
    n_p, n_k = p.shape
    V0, D0 = synth.random_factors(n_p, n_k, 3, 10)
    rounds = {}
    for ex in (False, True):
        V = to_dev(_as32(V0), torch.float32)
        D = to_dev(_as32(D0), torch.float32)
        st = hsn.hsn_subspace_nmf(_p_dev(p), None, n_k, V, D, max_iter=0, polish_rounds=3000,
                                  polish_algo=hsn.ALGO_ANLS, rel_obj_tol=1e-4, f_ref=f_star, anls_extrapolate=ex)
        f_end = onmf.objective(p.astype(np.float64), V.cpu().numpy().astype(np.float64),
                               D.cpu().numpy().astype(np.float64))
        show("  stop", extrapolate=ex, rounds=st["polish_done"], rel=st["rel_obj"])
        assert st["rel_obj"] <= 1e-4 and f_end <= st["objective"] * (1 + 1e-6)
        rounds[ex] = st["polish_done"]
    assert rounds[True] < rounds[False]
