"""Pins for the NMF oracle (eq. 4): multiplicative updates, ANLS, HALS, NNDSVD."""
import numpy as np
import pytest

from oracle import nmf
from oracle.metrics import canonical
import synth


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _noisy_lowrank(seed, n_p=80, n_k=40, k=3, noise=0.05):
    g = _rng(seed)
    V = g.uniform(0, 1, (n_p, k))
    D = g.uniform(0, 1, (n_k, k))
    P = np.maximum(V @ D.T + noise * g.standard_normal((n_p, n_k)), 0)
    return P


@pytest.mark.parametrize("seed", range(5))
def test_mu_monotone_and_nonnegative(seed):
    # Lee-Seung: neither half-step increases f; iterates stay >= 0.
    P = _noisy_lowrank(seed)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, seed + 100)
    f_prev = nmf.objective(P, V, D)
    for _ in range(60):
        V, D, fh, ff = nmf.mu_step(P, V, D)
        assert fh <= f_prev * (1 + 1e-14)
        assert ff <= fh * (1 + 1e-14)
        assert np.all(V >= 0) and np.all(D >= 0)
        f_prev = ff


def test_mu_fixed_point():
    # P = V* D*^T exactly: one MU step leaves (V*, D*) unchanged.
    g = _rng(3)
    V = g.uniform(0.2, 1, (30, 4))
    D = g.uniform(0.2, 1, (20, 4))
    P = V @ D.T
    V1, D1, fh, ff = nmf.mu_step(P, V, D)
    np.testing.assert_allclose(V1, V, rtol=1e-13)
    np.testing.assert_allclose(D1, D, rtol=1e-13)
    assert ff <= 1e-24 * np.sum(P * P)


def test_mu_scale_and_permutation_equivariance():
    P = _noisy_lowrank(4)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, 5)
    V1, D1, _, _ = nmf.mu_step(P, V, D)
    c = 3.7
    V2, D2, _, _ = nmf.mu_step(P, c * V, D / c)
    np.testing.assert_allclose(V2, c * V1, rtol=1e-13)
    np.testing.assert_allclose(D2, D1 / c, rtol=1e-13)
    perm = [2, 0, 1]
    V3, D3, _, _ = nmf.mu_step(P, V[:, perm], D[:, perm])
    np.testing.assert_allclose(V3, V1[:, perm], rtol=1e-13)
    np.testing.assert_allclose(D3, D1[:, perm], rtol=1e-13)


def test_mu_one_step_by_hand_tiny():
    # 2x2 case worked through scalar algebra (no matrix products), K = 1.
    P = np.array([[1.0, 2.0], [3.0, 4.0]])
    V = np.array([[1.0], [1.0]])
    D = np.array([[1.0], [0.5]])
    # G_D = 1 + 0.25 = 1.25; N_V = [1+1, 3+2] = [2, 5]; V G_D = [1.25, 1.25]
    v_new = np.array([2 / 1.25, 5 / 1.25])                 # [1.6, 4.0]
    # G_V = 1.6^2 + 4^2 = 18.56; N_D = [1*1.6+3*4, 2*1.6+4*4] = [13.6, 19.2]
    d_new = np.array([1.0 * 13.6 / (1.0 * 18.56), 0.5 * 19.2 / (0.5 * 18.56)])
    V1, D1, _, _ = nmf.mu_step(P, V, D)
    np.testing.assert_allclose(V1[:, 0], v_new, rtol=1e-15)
    np.testing.assert_allclose(D1[:, 0], d_new, rtol=1e-15)


def test_mu_rank1_converges_to_perron_pair():
    P = _noisy_lowrank(6, k=1, noise=0.0) + 0.01
    V, D = synth.random_factors(P.shape[0], P.shape[1], 1, 7)
    V, D, _, ff = nmf.mu_run(P, V, D, 3000)
    U, S, Vt = np.linalg.svd(P)
    best = S[0] ** 2 * 0 + np.sum(P * P) - S[0] ** 2     # Eckart-Young for rank 1
    assert abs(ff[-1] - best) <= 1e-8 * np.sum(P * P)
    np.testing.assert_allclose(V @ D.T, S[0] * np.outer(U[:, 0], Vt[0]), rtol=1e-6, atol=1e-8)


def test_expansion_objective_matches_direct():
    P = _noisy_lowrank(8)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, 9)
    V1, D1, _, ff = nmf.mu_step(P, V, D)
    N_D = P.T @ V1
    G_V = V1.T @ V1
    fe = nmf.mu_expansion_objective(np.sum(P * P), N_D, D1, G_V)
    assert abs(fe - ff) <= 1e-10 * np.sum(P * P)


def test_anls_monotone_and_exact_rank_k_recovery():
    # Noiseless p = L (D^m)^T (eq. 3 with w = 0) has rank K = N_m: ANLS
    # reaches f ~ 0 and the recovered basis spans exactly the columns of D^m.
    # (With strictly positive spectra the factors themselves are unique only
    # up to a non-negative mixing, so the span is what is fixed.)
    sc = synth.make_scan(n_views=20, n_rows=1, n_cols=32, n_bins=48, n_mat=3, flux=1e4,
                         seed=11, counts=False)
    P = sc.p_clean()
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, 12)
    f_prev = nmf.objective(P, V, D)
    for _ in range(300):
        V, D, fh, ff = nmf.anls_round(P, V, D)
        assert fh <= f_prev * (1 + 1e-12) + 1e-300
        assert ff <= fh * (1 + 1e-12) + 1e-300
        f_prev = ff
        if ff <= 1e-22 * np.sum(P * P):
            break
    assert f_prev <= 1e-20 * np.sum(P * P)
    Q, _ = np.linalg.qr(D)
    resid = sc.mu - Q @ (Q.T @ sc.mu)
    assert np.linalg.norm(resid) <= 1e-9 * np.linalg.norm(sc.mu)
    np.testing.assert_allclose(V @ D.T, P, atol=1e-9 * P.max())


@pytest.mark.parametrize("seed", range(3))
def test_hals_monotone(seed):
    P = _noisy_lowrank(seed + 20)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, seed + 30)
    f_prev = nmf.objective(P, V, D)
    for _ in range(40):
        V, D, fh, ff = nmf.hals_step(P, V, D)
        assert fh <= f_prev * (1 + 1e-13)
        assert ff <= fh * (1 + 1e-13)
        f_prev = ff


def test_hals_matches_scikit_learn_coordinate_descent():
    # scikit-learn's NMF 'cd' solver is the paper's Fast HALS implementation;
    # one iteration from the same start updates W (= V) column by column and
    # then H (= D^T), which is the same sweep.
    from sklearn.decomposition import non_negative_factorization
    P = _noisy_lowrank(40)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, 41)
    W, H, _ = non_negative_factorization(P, W=V.copy(), H=D.T.copy(), n_components=3, init="custom",
                                         solver="cd", max_iter=1, tol=0.0, shuffle=False)
    V1, D1, _, _ = nmf.hals_step(P, V, D)
    np.testing.assert_allclose(W, V1, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(H.T, D1, rtol=1e-10, atol=1e-12)


def test_nndsvd_rank1_and_k1():
    # K = 1: NNDSVD is sqrt(s1)|u1| sqrt(s1)|v1|^T, the best rank-1 fit for a
    # non-negative P (Perron vectors have one sign).
    g = _rng(50)
    a, b = g.uniform(0.1, 1, 25), g.uniform(0.1, 1, 15)
    P = np.outer(a, b)
    W, H = nmf.nndsvd(P, 1, variant="plain")
    np.testing.assert_allclose(W @ H.T, P, rtol=1e-12)
    P2 = _noisy_lowrank(51)
    U, S, Vt = np.linalg.svd(P2)
    W2, H2 = nmf.nndsvd(P2, 1, variant="plain")
    np.testing.assert_allclose(W2 @ H2.T, S[0] * np.outer(np.abs(U[:, 0]), np.abs(Vt[0])), rtol=1e-12)


def test_nndsvd_a_strictly_positive_and_sign_invariant():
    P = _noisy_lowrank(52, k=4)
    W, H = nmf.nndsvd(P, 4, variant="a")
    assert np.all(W > 0) and np.all(H > 0)
    # An SVD fixes each pair (u_j, v_j) only up to a joint sign flip; the
    # construction must give the same factors for either sign.
    U, S, Vt = np.linalg.svd(P, full_matrices=False)
    for j in range(4):
        U2, Vt2 = U.copy(), Vt.copy()
        U2[:, j] *= -1
        Vt2[j] *= -1
        W2, H2 = nmf.nndsvd_from_svd(U2, S, Vt2, 4, "a", P.mean())
        np.testing.assert_allclose(W2, W, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(H2, H, rtol=1e-13, atol=1e-15)


def test_nndsvd_hand_example():
    # Two-term SVD built by hand: u2 = (1, -1)/sqrt2, v2 = (1, 1)/sqrt2 has
    # positive parts (1,0)/sqrt2 and (1,1)/sqrt2 (norms 1/sqrt2, 1) and
    # negative parts (0,1)/sqrt2 and 0; m+ = 1/sqrt2 > m- = 0, so the second
    # pair is sqrt(s2/sqrt2) * (1, 0), sqrt(s2/sqrt2) * (1, 1)/sqrt2.
    r = 1 / np.sqrt(2)
    U = np.array([[r, r], [r, -r]])
    Vt = np.array([[r, -r], [r, r]])
    S = np.array([3.0, 1.0])
    W, H = nmf.nndsvd_from_svd(U, S, Vt, 2, "plain", 0.0)
    np.testing.assert_allclose(W[:, 0], np.sqrt(3) * np.array([r, r]), rtol=1e-15)
    np.testing.assert_allclose(H[:, 0], np.sqrt(3) * np.array([r, r]), rtol=1e-15)
    c = np.sqrt(1.0 * r)
    np.testing.assert_allclose(W[:, 1], c * np.array([1.0, 0.0]), rtol=1e-15)
    np.testing.assert_allclose(H[:, 1], c * np.array([r, r]), rtol=1e-15)


def test_stationary_reference_is_lower_than_mu():
    P = _noisy_lowrank(60)
    V, D = synth.random_factors(P.shape[0], P.shape[1], 3, 61)
    _, _, _, ff = nmf.mu_run(P, V, D, 200)
    fs, _, _ = nmf.stationary_reference(P, V, D)
    assert fs <= ff[-1] * (1 + 1e-12)


def test_kkt_residual_hand_cases():
    # 1 x 1 problem p = 1, D = 1: g_V = 2 (v - 1).
    P, D = np.array([[1.0]]), np.array([[1.0]])
    # v = 0 with a negative gradient (-2) violates g >= 0: residual |g| / |2 p d| = 1
    assert nmf.kkt_residual(P, np.array([[0.0]]), D)[0] == pytest.approx(1.0, rel=1e-15)
    # v = 2 > 0 with g = 2 violates x g = 0: residual min(2, 2) / 2 = 1
    assert nmf.kkt_residual(P, np.array([[2.0]]), D)[0] == pytest.approx(1.0, rel=1e-15)
    # v = 1: g = 0, stationary
    assert nmf.kkt_residual(P, np.array([[1.0]]), D)[0] == 0.0
    # p = -1: v = 0 is the constrained minimiser (g = 2 >= 0 at x = 0)
    assert nmf.kkt_residual(-P, np.array([[0.0]]), D)[0] == 0.0
    # an exact positive factorisation is stationary in both blocks
    g = _rng(70)
    V = g.uniform(0.2, 1, (40, 3))
    D = g.uniform(0.2, 1, (25, 3))
    rv, rd = nmf.kkt_residual(V @ D.T, V, D)
    assert rv <= 1e-14 and rd <= 1e-14


def test_kkt_residual_gradient_is_the_objective_gradient():
    # the interior residual is the gradient itself: check it against central
    # differences of f = ||P - V D^T||^2 at a strictly positive point
    P = _noisy_lowrank(71, n_p=12, n_k=9, k=2)
    g = _rng(72)
    V = g.uniform(0.5, 1, (12, 2))
    D = g.uniform(0.5, 1, (9, 2))
    gV = 2.0 * (V @ (D.T @ D) - P @ D)
    h = 1e-6
    for (i, j) in [(0, 0), (5, 1), (11, 0)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[i, j] += h
        Vm[i, j] -= h
        fd = (nmf.objective(P, Vp, D) - nmf.objective(P, Vm, D)) / (2 * h)
        assert fd == pytest.approx(gV[i, j], rel=1e-7)
    # where every gradient entry is below its x, the residual is ||g|| / ||2 P D||
    if np.all(np.abs(gV) < V):
        assert nmf.kkt_residual(P, V, D)[0] == pytest.approx(np.linalg.norm(gV) / np.linalg.norm(2 * P @ D))


def test_stationary_reference_is_a_kkt_point():
    # A small noisy scan, where plain ANLS is still 2e-4 above the minimum
    # after 300 rounds: the reference must end at a first-order stationary
    # point (both KKT residuals <= 1e-9 relative) and below every ANLS iterate.
    sc = synth.make_scan(n_views=12, n_rows=1, n_cols=24, n_bins=48, n_mat=3, flux=1e4, seed=5)
    from oracle.normalize import normalize
    P, _, _ = normalize(sc.y, sc.yo)
    V0, D0 = synth.random_factors(P.shape[0], P.shape[1], 3, 7)
    fs, Vs, Ds = nmf.stationary_reference(P, V0, D0, max_rounds=50)
    rv, rd = nmf.kkt_residual(P, Vs, Ds)
    assert rv <= 1e-9 and rd <= 1e-9, (rv, rd)
    assert np.all(Vs >= 0) and np.all(Ds >= 0)
    assert fs == pytest.approx(nmf.objective(P, Vs, Ds), rel=1e-15)
    f_anls, Va, Da = nmf.stationary_reference(P, V0, D0, max_rounds=50, refine=False)
    assert fs <= f_anls
    # the pin bites: an early-stopped reference (one ANLS round, or the
    # 50 rounds alone) is far from stationary
    assert max(nmf.kkt_residual(P, Va, Da)) > 1e-6
    _, V1, D1 = nmf.stationary_reference(P, V0, D0, max_rounds=1, refine=False)
    assert max(nmf.kkt_residual(P, V1, D1)) > 1e-4


def test_extrapolated_anls_without_weight_is_plain_anls():
    # beta0 = 0 keeps the weight at 0: every round is a plain ANLS round.
    P = _noisy_lowrank(11, 60, 30, 3)
    V0, D0 = synth.random_factors(60, 30, 3, 12)
    V, D = V0.copy(), D0.copy()
    hist = []
    for _ in range(6):
        V, D, fh, _ = nmf.anls_round(P, V, D)
        hist.append(fh)
    Ve, De, he = nmf.anls_extrapolated_run(P, V0, D0, 6, beta0=0.0)
    assert np.array_equal(Ve, V) and np.array_equal(De, D)
    assert np.array_equal(he, np.array(hist))


def test_extrapolated_anls_accelerates_to_the_stationary_point():
    # The small noisy scan where plain ANLS is still 1.6e-3 above the
    # KKT-pinned stationary reference after 400 rounds: the extrapolated
    # rounds get within 1e-4 of it in about 110 rounds, while plain ANLS after
    # 150 rounds is still more than ten times as far, and they end near a
    # KKT point.
    sc = synth.make_scan(n_views=12, n_rows=1, n_cols=24, n_bins=48, n_mat=3, flux=1e4, seed=5)
    from oracle.normalize import normalize
    P, _, _ = normalize(sc.y, sc.yo)
    V0, D0 = synth.random_factors(P.shape[0], P.shape[1], 3, 7)
    fs, _, _ = nmf.stationary_reference(P, V0, D0, max_rounds=50)
    Ve, De, he = nmf.anls_extrapolated_run(P, V0, D0, 220)
    hit = np.nonzero((he - fs) / fs <= 1e-4)[0]
    assert hit.size and hit[0] < 150, hit[:1]
    V, D = V0.copy(), D0.copy()
    hp = []
    for _ in range(150):
        V, D, fh, _ = nmf.anls_round(P, V, D)
        hp.append(fh)
    assert (min(hp) - fs) / fs > 1e-3
    assert max(nmf.kkt_residual(P, Ve, De)) <= 1e-3


def test_extrapolated_anls_stop_keeps_the_exact_d():
    # With a stop test the run ends at the first objective within the
    # tolerance and returns that round's exact D, no worse than the recorded
    # objective.
    P = _noisy_lowrank(13, 70, 35, 3)
    V0, D0 = synth.random_factors(70, 35, 3, 14)
    _, _, h = nmf.anls_extrapolated_run(P, V0, D0, 60)
    f_ref = h.min() * (1 - 1e-9)
    V, D, hs = nmf.anls_extrapolated_run(P, V0, D0, 60, f_ref=f_ref, tol=1e-3)
    assert (hs[-1] - f_ref) / f_ref <= 1e-3 and np.all((hs[:-1] - f_ref) / f_ref > 1e-3)
    assert nmf.objective(P, V, D) <= hs[-1] * (1 + 1e-12)
    assert np.array_equal(D, nmf.nnls_rows(V.T @ V, P.T @ V))
