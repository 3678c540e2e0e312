"""Pins for the MLP oracle (warm start), eq. (6) expansion and the eq. (7)-(9) tail."""
import math

import numpy as np
import pytest

import synth
from oracle import expand, mlp


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_activation_special_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.softplus(np.array([0.0]))[0] - math.log(2.0)) < 1e-16
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    np.testing.assert_allclose((mlp.softplus(z + h) - mlp.softplus(z - h)) / (2 * h), mlp.sigmoid(z), rtol=1e-8)
    np.testing.assert_allclose((mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), mlp.gelu_grad(z), rtol=1e-7, atol=1e-9)
    # GELU(z) -> z for large z, -> 0 for very negative z; softplus -> z
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-15
    assert abs(mlp.softplus(np.array([40.0]))[0] - 40.0) < 1e-15


def test_pool_bounds_identity_and_mean():
    P = _rng(1).uniform(0, 2, (5, 256))
    np.testing.assert_array_equal(mlp.pool(P), P)
    lo, hi = mlp.pool_bounds(1000)
    assert lo[0] == 0 and hi[-1] == 1000
    assert all(h > l for l, h in zip(lo, hi))
    Q = _rng(2).uniform(0, 2, (3, 1000))
    pooled = mlp.pool(Q)
    np.testing.assert_allclose(pooled[:, 7], Q[:, lo[7]:hi[7]].mean(axis=1), rtol=1e-15)


def test_gradient_finite_differences():
    k = 3
    theta = synth.mlp_init(k, 4)
    theta = theta + 0.05 * _rng(5).standard_normal(theta.shape)     # non-zero biases too
    x = _rng(6).uniform(0, 2, (7, 256))
    t = _rng(7).uniform(0, 1, (7, k))
    loss, grads = mlp.loss_and_grad(mlp.unflatten(theta, k), x, t)
    g = mlp.flatten(grads)
    idx = _rng(8).choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(mlp.unflatten(tp, k), x, t)[0] - mlp.loss_and_grad(mlp.unflatten(tm, k), x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-9


def test_gradient_matches_torch_autograd_fp64():
    torch = pytest.importorskip("torch")
    k = 4
    theta = synth.mlp_init(k, 9) + 0.01
    x = _rng(10).uniform(0, 2, (11, 256))
    t = _rng(11).uniform(0, 1, (11, k))
    loss, grads = mlp.loss_and_grad(mlp.unflatten(theta, k), x, t)
    ps = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in mlp.unflatten(theta, k)]
    X = torch.tensor(x)
    h1 = torch.nn.functional.gelu(X @ ps[0] + ps[1])
    h2 = torch.nn.functional.gelu(h1 @ ps[2] + ps[3])
    y = torch.nn.functional.softplus(h2 @ ps[4] + ps[5])
    L = ((y - torch.tensor(t)) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) <= 1e-14 * loss
    for a, b in zip(grads, ps):
        np.testing.assert_allclose(a, b.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_adam_on_quadratic_closed_form():
    # First Adam step moves every coordinate by exactly lr * sign(g)
    # (m_hat = g, v_hat = g^2), up to eps.
    theta = np.array([1.0, -2.0, 0.5])
    g = 2 * theta                   # gradient of sum(theta^2)
    new, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(new, theta - 1e-3 * np.sign(g), rtol=1e-15)
    # Second step from the closed-form moments.
    g2 = 2 * new
    new2, _, _ = mlp.adam_step(new, g2, m, v, 2, lr=1e-3, eps=0.0)
    m2 = 0.9 * m + 0.1 * g2
    v2 = 0.999 * v + 0.001 * g2 * g2
    ref = new - 1e-3 * (m2 / (1 - 0.81)) / np.sqrt(v2 / (1 - 0.999 ** 2))
    np.testing.assert_allclose(new2, ref, rtol=1e-15)


def test_rehydrate_ranges():
    xs = _rng(12).standard_normal((20, 3))
    D = _rng(13).uniform(0, 1, (15, 3))
    full = expand.rehydrate(xs, D)
    assert full.shape == (20, 15)
    np.testing.assert_allclose(full[3, 4], xs[3] @ D[4], rtol=1e-15)
    np.testing.assert_array_equal(expand.rehydrate(xs, D, vox=(2, 9), bins=(5, 11)), full[2:9, 5:11])


def test_fmd_tail_appendix_b_identity():
    # Appendix B: if x^s = x^m T then D^m = D^s T^T reproduces the same
    # spectra: (A x^m)(D^m)^T = (A x^s)(D^s)^T.  With pure-material masks,
    # eq. (7) recovers T, eq. (8) recovers x^m, eq. (9) recovers D^m.
    g = _rng(14)
    n_x, n_m, n_s, n_k = 60, 3, 5, 12
    lab = g.integers(0, n_m, n_x)
    xm = np.zeros((n_x, n_m))
    xm[np.arange(n_x), lab] = 1.0
    T = g.uniform(0.1, 1, (n_m, n_s))
    xs = xm @ T
    Ds = g.uniform(0, 1, (n_k, n_s))
    masks = [np.flatnonzero(lab == i) for i in range(n_m)]
    T_est = expand.transform_matrix(xs, masks)
    np.testing.assert_allclose(T_est, T, rtol=1e-14)
    np.testing.assert_allclose(expand.material_volumes(xs, T_est), xm, atol=1e-12)
    Dm = expand.material_spectra(Ds, T_est)
    np.testing.assert_allclose(xm @ Dm.T, xs @ Ds.T, rtol=1e-13)


def test_canonical_form_pins():
    """Canonical form of an NMF pair: a planted permutation and positive column
    scaling of a known (V, D) is undone exactly, the product is unchanged, and
    without a library the columns are ordered by the norm of the scaled V."""
    import itertools
    from oracle.metrics import canonical
    g = np.random.Generator(np.random.PCG64(5))
    k, n_p, n_k = 4, 50, 30
    L = g.uniform(0.1, 1.0, (n_k, k))
    Ln = L / np.linalg.norm(L, axis=0)
    V = g.uniform(0.0, 2.0, (n_p, k))
    perm = [2, 0, 3, 1]
    scale = np.array([0.5, 3.0, 1.7, 0.2])
    Dp = (Ln * scale)[:, perm]
    Vp = (V / scale)[:, perm]
    Vc, Dc = canonical(Vp, Dp, library=L)
    assert np.allclose(Dc, Ln, rtol=1e-14, atol=0)
    assert np.allclose(Vc, V, rtol=1e-13, atol=1e-15)
    assert np.allclose(Vc @ Dc.T, Vp @ Dp.T, rtol=1e-13)
    # the chosen permutation maximises the summed cosine (brute force)
    cos = (Dp / np.linalg.norm(Dp, axis=0)).T @ Ln
    best = max(itertools.permutations(range(k)), key=lambda p: sum(cos[p[m], m] for m in range(k)))
    assert list(best) == [perm.index(m) for m in range(k)]
    # without a library: descending norm of the scaled V columns
    Vn, Dn = canonical(Vp, Dp)
    norms = np.linalg.norm(Vn, axis=0)
    assert np.all(np.diff(norms) <= 0)
    assert np.allclose(np.linalg.norm(Dn, axis=0), 1.0, rtol=1e-14)
