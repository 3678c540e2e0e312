"""Subspace extraction by NMF (eq. 4): (V, D) = argmin_{V,D >= 0} ||p - V D^T||_F^2.

p is N_p x N_k, V is N_p x K (subspace views), D is N_k x K (basis).

Readings where the paper is silent (each is listed in the design notes):
  * multiplicative updates follow Lee & Seung (the paper's NMF citation):
    V first, then D with the *new* V (Gauss-Seidel order);
  * no epsilon in the numerator; the denominator is guarded only against
    an exact zero (1e-300), so the monotonicity theorem holds exactly;
  * the objective is eq. (4) verbatim, with no factor 1/2;
  * NNDSVD follows Boutsidis & Gallopoulos (the paper's initialisation);
    the 'a' variant fills exact zeros with mean(p); on a tie between the
    positive and negative parts the positive part is taken;
  * HALS is the column-wise exact update of Cichocki & Phan (the paper's
    "Fast HALS" solver), with each column clipped at zero.
"""
from __future__ import annotations

import numpy as np

from .nnls import nnls_rows

TINY = 1e-300


def objective(P, V, D) -> float:
    """f = ||P - V D^T||_F^2, computed directly from the residual."""
    R = P - V @ D.T
    return float(np.sum(R * R))


def mu_step(P, V, D):
    """One Lee-Seung multiplicative-update iteration.

    Returns (V_new, D_new, f_half, f_full) where f_half = f(V_new, D_old)
    (the objective after the V half-step) and f_full = f(V_new, D_new).
    """
    P = np.asarray(P, np.float64)
    G_D = D.T @ D
    N_V = P @ D
    V_new = V * N_V / np.maximum(V @ G_D, TINY)
    f_half = objective(P, V_new, D)
    G_V = V_new.T @ V_new
    N_D = P.T @ V_new
    D_new = D * N_D / np.maximum(D @ G_V, TINY)
    f_full = objective(P, V_new, D_new)
    return V_new, D_new, f_half, f_full


def mu_expansion_objective(P_sumsq, N_D, D_new, G_V):
    """The same f(V_new, D_new) from the pass's accumulated terms:
    ||P||^2 - 2 <P^T V, D> + <V^T V, D^T D>."""
    return float(P_sumsq - 2.0 * np.sum(N_D * D_new) + np.sum(G_V * (D_new.T @ D_new)))


def mu_run(P, V, D, n_iter: int):
    """n_iter MU iterations; returns V, D and the per-iteration f_half / f_full."""
    fh, ff = [], []
    for _ in range(n_iter):
        V, D, a, b = mu_step(P, V, D)
        fh.append(a)
        ff.append(b)
    return V, D, np.array(fh), np.array(ff)


def anls_round(P, V, D):
    """One alternating exact block minimisation: every row of V is the exact
    NNLS solution for the current D, then every row of D for the new V.
    Returns (V_new, D_new, f_half, f_full)."""
    P = np.asarray(P, np.float64)
    V_new = nnls_rows(D.T @ D, P @ D)
    f_half = objective(P, V_new, D)
    D_new = nnls_rows(V_new.T @ V_new, P.T @ V_new)
    return V_new, D_new, f_half, objective(P, V_new, D_new)


def anls_extrapolated_run(P, V, D, rounds: int, f_ref: float = 0.0, tol: float = 0.0, beta0: float = 0.5,
                          grow: float = 1.05, cap_grow: float = 1.01, shrink: float = 1.5):
    """ANLS rounds with extrapolation of D between rounds (Ang & Gillis,
    Neural Computation 31(2), 2019), in the form the library runs.

    Round k solves every row of V exactly for D_hat (the start D at k = 0),
    records e_k = f(V, D_hat), then solves every row of D exactly for V
    (D_new).  The weight beta (start beta0, cap 1) is adapted from the
    recorded objectives: if e_k <= e_{k-1}, beta <- min(cap, grow beta),
    cap <- min(1, cap_grow cap) and D_hat <- max(0, D_new + beta (D_new -
    D_prev)); otherwise cap <- beta, beta <- beta / shrink and D_hat <- D_new.
    D_prev <- D_new.  With f_ref > 0 the run stops at the first e_k with
    (e_k - f_ref)/f_ref <= tol, keeping that round's D_new.
    Returns (V, D_hat, history of e_k)."""
    P = np.asarray(P, np.float64)
    D_hat = np.array(D, np.float64)
    D_prev = D_hat.copy()
    beta, cap, e_prev = beta0, 1.0, np.inf
    hist = []
    for _ in range(rounds):
        V = nnls_rows(D_hat.T @ D_hat, P @ D_hat)
        e = objective(P, V, D_hat)
        hist.append(e)
        D_new = nnls_rows(V.T @ V, P.T @ V)
        stop = f_ref > 0.0 and (e - f_ref) / f_ref <= tol
        use = 0.0
        if not stop:
            if e <= e_prev:
                beta = min(cap, grow * beta)
                cap = min(1.0, cap_grow * cap)
                use = beta
            else:
                cap = beta
                beta = beta / shrink
        e_prev = e
        D_hat = np.maximum(0.0, D_new + use * (D_new - D_prev)) if use > 0.0 else D_new
        D_prev = D_new
        if stop:
            break
    return V, D_hat, np.array(hist)


def hals_step(P, V, D):
    """One HALS sweep: columns of V in order, then columns of D, each set to
    its exact non-negative minimiser with the other columns fixed."""
    P = np.asarray(P, np.float64)
    V = V.copy()
    D = D.copy()
    G_D = D.T @ D
    N_V = P @ D
    for j in range(V.shape[1]):
        if G_D[j, j] > 0:
            V[:, j] = np.maximum(0.0, V[:, j] + (N_V[:, j] - V @ G_D[:, j]) / G_D[j, j])
    f_half = objective(P, V, D)
    G_V = V.T @ V
    N_D = P.T @ V
    for j in range(D.shape[1]):
        if G_V[j, j] > 0:
            D[:, j] = np.maximum(0.0, D[:, j] + (N_D[:, j] - D @ G_V[:, j]) / G_V[j, j])
    return V, D, f_half, objective(P, V, D)


def nndsvd(P, k: int, variant: str = "a"):
    """NNDSVD initialisation (Boutsidis & Gallopoulos 2008) of P.

    Returns (V0 [N_p][K], D0 [N_k][K]); see nndsvd_from_svd.
    """
    P = np.asarray(P, np.float64)
    U, S, Vt = np.linalg.svd(P, full_matrices=False)
    return nndsvd_from_svd(U, S, Vt, k, variant, P.mean())


def nndsvd_from_svd(U, S, Vt, k: int, variant: str, p_mean: float):
    """NNDSVD from given leading singular triplets (s_j, u_j, v_j).

    The first pair is sqrt(s_1)|u_1|, sqrt(s_1)|v_1|; for j >= 2 the
    positive or negative parts of (u_j, v_j) with the larger product of
    norms m are kept and scaled by sqrt(s_j m) (a tie keeps the positive
    parts).  variant 'a' replaces exact zeros by the mean of P.
    """
    n_p, n_k = U.shape[0], Vt.shape[1]
    W = np.zeros((n_p, k))
    H = np.zeros((n_k, k))
    W[:, 0] = np.sqrt(S[0]) * np.abs(U[:, 0])
    H[:, 0] = np.sqrt(S[0]) * np.abs(Vt[0])
    for j in range(1, k):
        x, y = U[:, j], Vt[j]
        xp, xn = np.maximum(x, 0), np.maximum(-x, 0)
        yp, yn = np.maximum(y, 0), np.maximum(-y, 0)
        xpn, xnn = np.linalg.norm(xp), np.linalg.norm(xn)
        ypn, ynn = np.linalg.norm(yp), np.linalg.norm(yn)
        mp, mn = xpn * ypn, xnn * ynn
        if mp >= mn:
            u, v, m = (xp / xpn if xpn > 0 else xp), (yp / ypn if ypn > 0 else yp), mp
        else:
            u, v, m = xn / xnn, yn / ynn, mn
        W[:, j] = np.sqrt(S[j] * m) * u
        H[:, j] = np.sqrt(S[j] * m) * v
    if variant == "a":
        W[W == 0] = p_mean
        H[H == 0] = p_mean
    return W, H


def kkt_residual(P, V, D):
    """Distance of (V, D) from a first-order stationary point of eq. (4)
    under V, D >= 0: with the gradients g_V = 2 (V D^T D - P D) and
    g_D = 2 (D V^T V - P^T V), the KKT conditions are x >= 0, g >= 0 and
    x g = 0 entrywise, all of which hold exactly where min(x, g) = 0.
    Returns (||min(V, g_V)|| / ||2 P D||, ||min(D, g_D)|| / ||2 P^T V||)."""
    P = np.asarray(P, np.float64)
    gV = 2.0 * (V @ (D.T @ D) - P @ D)
    gD = 2.0 * (D @ (V.T @ V) - P.T @ V)
    sV = max(np.linalg.norm(2.0 * P @ D), TINY)
    sD = max(np.linalg.norm(2.0 * P.T @ V), TINY)
    return float(np.linalg.norm(np.minimum(V, gV)) / sV), float(np.linalg.norm(np.minimum(D, gD)) / sD)


def stationary_reference(P, V, D, max_rounds: int = 500, rtol: float = 1e-12, refine: bool = True,
                         refine_iters: int = 50000):
    """f* for the relative objective: a stationary point of eq. (4) reached
    from (V, D).  Three stages:
      1. ANLS rounds until the relative change of f drops below rtol (or
         max_rounds);
      2. (refine) a projected quasi-Newton minimisation of f over (V, D) >= 0
         (scipy's L-BFGS-B, the library routine as one step, restarted while
         it still lowers f).  Alternating
         exact block minimisation crawls along the shallow valleys that the
         mixing freedom of nearly collinear spectra leaves in f; the
         quasi-Newton curvature model does not;
      3. (refine) five ANLS rounds, which make D exactly optimal for V.
    The result's stationarity is checked by kkt_residual.  Returns (f*, V, D)."""
    P = np.asarray(P, np.float64)
    f_prev = objective(P, V, D)
    for _ in range(max_rounds):
        V, D, _, f = anls_round(P, V, D)
        if f_prev - f <= rtol * f:
            f_prev = min(f, f_prev)
            break
        f_prev = f
    if not refine:
        return f_prev, V, D
    from scipy.optimize import minimize

    n_p, k = V.shape
    n_k = D.shape[0]

    def f_and_grad(z):
        Vz = z[:n_p * k].reshape(n_p, k)
        Dz = z[n_p * k:].reshape(n_k, k)
        R = Vz @ Dz.T - P
        return float(np.sum(R * R)), np.concatenate([(2.0 * R @ Dz).ravel(), (2.0 * R.T @ Vz).ravel()])

    # The routine can stop early when its line search stalls; it is restarted
    # (fresh curvature memory) until a restart no longer lowers f.
    z = np.concatenate([np.asarray(V, np.float64).ravel(), np.asarray(D, np.float64).ravel()])
    f_z = f_and_grad(z)[0]
    for _ in range(10):
        r = minimize(f_and_grad, z, jac=True, method="L-BFGS-B", bounds=[(0.0, None)] * z.size,
                     options=dict(maxiter=refine_iters, maxfun=2 * refine_iters, ftol=1e-16, gtol=1e-14,
                                  maxcor=30))
        done = r.fun >= f_z * (1.0 - 1e-15)
        if r.fun <= f_z:
            z, f_z = r.x, r.fun
        if done:
            break
    Vr = z[:n_p * k].reshape(n_p, k).copy()
    Dr = z[n_p * k:].reshape(n_k, k).copy()
    f = objective(P, Vr, Dr)
    for _ in range(5):
        Vr, Dr, _, f = anls_round(P, Vr, Dr)
    if f <= f_prev:
        return f, Vr, Dr
    return f_prev, V, D
