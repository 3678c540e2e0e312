"""Training data and training of the learned NMF start.

The network learns from decompositions that the plain method itself
produces (eq. 4): synthetic scans that share one fixed material library are
decomposed (NNDSVDa start, MU bulk, ANLS polish), each pair is put in
canonical form against the library, and the pooled spectra of the rays with
their canonical coefficients form the training set.  All computation runs in
the library's kernels; this module only sequences the calls.

    python -m paper_2410_22500_amd.warmstart --phantoms 348 --epochs 20 --out net.bin
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

import synth
from paper_2410_22500_amd import hsn

# The learned start serves scans made of the mid workload's four materials
# (their spectra come from this library seed); geometry and noise vary.
LIBRARY_SEED = 2
N_MAT = 4
# Training scans: the tiny workload's geometry (90 views over 180 degrees,
# one 64-column slice, 256 bins, flux 1e4).
TRAIN_GEOMETRY = dict(n_views=90, n_rows=1, n_cols=64, n_bins=256, flux=1e4)
HELD_OUT_SEED0 = 10041
MID_GEOMETRY = dict(n_views=60, n_rows=16, n_cols=128, n_bins=1024, flux=2e3)
MID_SEED = 2


def scans(seed0: int, count: int, k: int = N_MAT, library_seed: int = LIBRARY_SEED, geometry=None,
          counts: bool = True):
    """The first `count` scans from seeds seed0, seed0+1, ...  A seed whose
    objects cannot be placed without overlap is skipped (deterministically).
    counts=False leaves the counts to be drawn on the GPU (scan_to_device)."""
    geometry = dict(geometry or TRAIN_GEOMETRY)
    s, got = seed0, 0
    while got < count:
        try:
            scan = synth.make_scan(n_mat=k, seed=s, library_seed=library_seed, counts=counts, **geometry)
        except RuntimeError:
            s += 1
            continue
        yield s, scan
        s += 1
        got += 1


def scan_to_device(scan, seed: int = 0):
    """Normalised p (float32) and its bfloat16 copy on the GPU; a scan made
    without counts gets them drawn on the GPU from `seed`."""
    if scan.y is None:
        y, yo = synth.device_counts(scan, seed=seed)
    else:
        y = torch.from_numpy(scan.y.view(np.int16)).cuda()
        yo = torch.from_numpy(scan.yo.view(np.int16)).cuda()
    p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
    return p, pb


def workload_geometry(n_bins: int, flux: float):
    """Training geometry for a workload: the tiny workload's phantoms and
    views (90 views, one 64-column slice) at the workload's own spectral
    sampling and flux, so that the pooled spectra carry its noise level."""
    return dict(TRAIN_GEOMETRY, n_bins=int(n_bins), flux=float(flux))


def plain_decomposition(p, pb, n_k: int, k: int, mu_iters: int = 200, polish: int = 60,
                        precision: int = hsn.PREC_FP32, f_ref: float = 0.0, tol: float = 0.0):
    """NNDSVDa start, MU bulk, ANLS polish; returns (V, D, stats)."""
    n_p = p.shape[0]
    V = torch.empty((n_p, k), dtype=torch.float32, device=p.device)
    D = torch.empty((n_k, k), dtype=torch.float32, device=p.device)
    st = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, algo=hsn.ALGO_MU, precision=precision, max_iter=mu_iters,
                              check_every=max(mu_iters, 1), polish_rounds=polish, polish_algo=hsn.ALGO_ANLS,
                              init=hsn.INIT_NNDSVDA, f_ref=f_ref, rel_obj_tol=tol)
    return V, D, st


def make_training_set(n_scans: int, seed0: int = 40, k: int = N_MAT, library_seed: int = LIBRARY_SEED,
                      geometry=None, mu_iters: int = 200, polish: int = 60, joint: bool = True, log=None):
    """Pooled spectra X [N][256] (bfloat16 bits) and canonical coefficient
    targets T [N][K] float32 over the rays of n_scans scans from seed0 on.

    joint=True decomposes the rows of all scans as one NMF, so every target
    is expressed in one basis D; joint=False decomposes scan by scan (the NMF
    is unique only up to a mixing of its columns that the canonical form does
    not remove, so those targets differ from scan to scan by that mixing)."""
    geometry = dict(geometry or TRAIN_GEOMETRY)
    n_p = geometry["n_views"] * geometry["n_rows"] * geometry["n_cols"]
    n_k = geometry["n_bins"]
    N = n_scans * n_p
    X = torch.empty((N, hsn.MLP_IN), dtype=torch.int16, device="cuda")
    T = torch.empty((N, k), dtype=torch.float32, device="cuda")
    P_all = Pb_all = None
    t_gen = t_dec = 0.0
    # counts of wide spectra are drawn on the GPU (seeded), narrow ones on the host
    host_counts = n_k <= 256
    it = scans(seed0, n_scans, k, library_seed, geometry, counts=host_counts)
    lib = None
    for i in range(n_scans):
        t0 = time.perf_counter()
        s, scan = next(it)
        t1 = time.perf_counter()
        p, pb = scan_to_device(scan, seed=7919 * s + 1)
        if lib is None:
            lib = torch.from_numpy(scan.mu.astype(np.float32)).cuda()
        rows = slice(i * n_p, (i + 1) * n_p)
        if joint:
            if P_all is None:
                P_all = torch.empty((N, p.shape[1]), dtype=torch.float32, device="cuda")
                Pb_all = torch.empty((N, pb.shape[1]), dtype=torch.int16, device="cuda")
            P_all[rows] = p
            Pb_all[rows] = pb
        else:
            V, D, _ = plain_decomposition(p, pb, n_k, k, mu_iters, polish)
            hsn.hsn_canonicalize(V, D, torch.from_numpy(scan.mu.astype(np.float32)).cuda())
            T[rows] = V
        X[rows] = hsn.hsn_mlp_pool(pb, n_k, hsn.PREC_BF16)
        torch.cuda.synchronize()
        t_gen += t1 - t0
        t_dec += time.perf_counter() - t1
        if log and (i + 1) % 50 == 0:
            log(f"training set: {i + 1}/{n_scans} scans")
    if joint:
        t1 = time.perf_counter()
        V, D, _ = plain_decomposition(P_all, Pb_all, n_k, k, mu_iters, polish)
        hsn.hsn_canonicalize(V, D, lib)
        T.copy_(V)
        torch.cuda.synchronize()
        t_dec += time.perf_counter() - t1
        del P_all, Pb_all
    return X, T, dict(scan_s=t_gen, decompose_s=t_dec)


def train(X, T, k: int = N_MAT, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 40,
          init_seed: int = 40, precision: int = hsn.PREC_BF16):
    m = hsn.hsn_mlp_create(k, precision, synth.mlp_init(k, init_seed).astype(np.float32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = hsn.hsn_mlp_train(m, X, T, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    return m, hist, time.perf_counter() - t0


def reference_objective(p, pb, n_k: int, k: int, mlp=None, rounds: int = 1500):
    """f*: the lowest objective reached by long runs (cold NNDSVDa start and,
    when given, the learned start), each polished by ANLS to stationarity."""
    best = np.inf
    V, D, st = plain_decomposition(p, pb, n_k, k, 200, rounds)
    best = min(best, st["objective"])
    if mlp is not None:
        V2 = torch.empty_like(V)
        D2 = torch.empty_like(D)
        st2 = hsn.hsn_subspace_nmf(p, pb, n_k, V2, D2, max_iter=0, polish_rounds=rounds,
                                   polish_algo=hsn.ALGO_ANLS, init=hsn.INIT_MLP, mlp=mlp)
        best = min(best, st2["objective"])
    return best


def time_to_tol(p, pb, n_k: int, k: int, f_ref: float, tol: float = 1e-4, mlp=None, precision=hsn.PREC_FP32,
                bulk: int = None, polish_cap: int = 1500):
    """One run to rel obj <= tol: MU bulk (`bulk` iterations in `precision`)
    then ANLS polish, from NNDSVDa (cold) or from the learned start (mlp).
    Default bulk: 200 cold, 0 warm.  Returns the stats dict."""
    n_p = p.shape[0]
    V = torch.empty((n_p, k), dtype=torch.float32, device=p.device)
    D = torch.empty((n_k, k), dtype=torch.float32, device=p.device)
    if bulk is None:
        bulk = 200 if mlp is None else 0
    return hsn.hsn_subspace_nmf(p, pb, n_k, V, D, algo=hsn.ALGO_MU, precision=precision, max_iter=bulk,
                                check_every=max(bulk, 1), polish_rounds=polish_cap, polish_algo=hsn.ALGO_ANLS,
                                init=hsn.INIT_NNDSVDA if mlp is None else hsn.INIT_MLP, mlp=mlp, f_ref=f_ref,
                                rel_obj_tol=tol)


def compare_held_out(mlp, n_scans: int, seed0: int = HELD_OUT_SEED0, k: int = N_MAT, geometry=None,
                     tol: float = 1e-4, library_seed: int = LIBRARY_SEED):
    """Warm versus cold on held-out scans: passes over p and device ms to
    rel obj <= tol (f* from reference_objective).  library_seed other than
    the training library's gives scans of materials the network never saw."""
    geometry = dict(geometry or TRAIN_GEOMETRY)
    n_k = geometry["n_bins"]
    rows = []
    for s, scan in scans(seed0, n_scans, k, library_seed, geometry, counts=n_k <= 256):
        p, pb = scan_to_device(scan, seed=7919 * s + 1)
        f_ref = reference_objective(p, pb, n_k, k, mlp)
        cold = time_to_tol(p, pb, n_k, k, f_ref, tol)
        warm = time_to_tol(p, pb, n_k, k, f_ref, tol, mlp=mlp)
        rows.append(dict(seed=int(s), f_ref=f_ref,
                         cold_iters=cold["iters"] + cold["polish_done"], cold_rel=cold["rel_obj"], cold_ms=cold["ms"],
                         warm_iters=warm["iters"] + warm["polish_done"], warm_rel=warm["rel_obj"], warm_ms=warm["ms"]))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--phantoms", type=int, default=348)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--held-out", type=int, default=32)
    ap.add_argument("--per-scan", action="store_true", help="targets from per-scan decompositions")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--mid", action="store_true", help="also compare on the mid workload (1024 bins pooled)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--json", default=None)
    ap.add_argument("--unseen-library", type=int, default=None,
                    help="also compare on held-out scans of this material library (not seen in training)")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    X, T, t = make_training_set(a.phantoms, joint=not a.per_scan, log=log)
    log(f"training set: {X.shape[0]} spectra, scans {t['scan_s']:.1f} s, decompositions {t['decompose_s']:.1f} s")
    m, hist, t_train = train(X, T, epochs=a.epochs, batch=a.batch, lr=a.lr)
    log(f"training: {a.epochs} epochs in {t_train:.2f} s, loss {hist[0]:.4g} -> {hist[-1]:.4g}")
    if a.out:
        hsn.hsn_mlp_save(m, a.out)
    def summarise(rows):
        cw = np.array([[r["cold_iters"], r["warm_iters"], r["cold_ms"], r["warm_ms"]] for r in rows], float)
        return dict(cold_iters_mean=cw[:, 0].mean(), warm_iters_mean=cw[:, 1].mean(),
                    cold_ms_mean=cw[:, 2].mean(), warm_ms_mean=cw[:, 3].mean(),
                    cold_ms_median=float(np.median(cw[:, 2])), warm_ms_median=float(np.median(cw[:, 3])),
                    warm_reached=int(sum(r["warm_rel"] <= 1e-4 for r in rows)),
                    cold_reached=int(sum(r["cold_rel"] <= 1e-4 for r in rows)), held_out=len(rows))

    rows = compare_held_out(m, a.held_out)
    for r in rows:
        log(json.dumps(r))
    summary = dict(spectra=int(X.shape[0]), epochs=a.epochs, train_s=t_train, loss_first=hist[0],
                   loss_last=hist[-1], library_seed=LIBRARY_SEED, **summarise(rows), **t)
    rows_unseen = None
    if a.unseen_library is not None:
        rows_unseen = compare_held_out(m, a.held_out, library_seed=a.unseen_library)
        for r in rows_unseen:
            log("unseen library: " + json.dumps(r))
        summary["unseen_library"] = dict(library_seed=a.unseen_library, **summarise(rows_unseen))
    if a.mid:
        scan = synth.make_scan(n_mat=N_MAT, seed=MID_SEED, library_seed=LIBRARY_SEED, **MID_GEOMETRY)
        p, pb = scan_to_device(scan)
        n_k = MID_GEOMETRY["n_bins"]
        f_ref = reference_objective(p, pb, n_k, N_MAT, m)
        mid = dict(f_ref=f_ref)
        for name, kw in [("cold_fp32", {}), ("cold_bf16", dict(precision=hsn.PREC_BF16)),
                         ("warm", dict(mlp=m)), ("warm_bf16_mu20", dict(mlp=m, precision=hsn.PREC_BF16, bulk=20))]:
            st = time_to_tol(p, pb, n_k, N_MAT, f_ref, **kw)
            mid[name] = dict(iters=st["iters"] + st["polish_done"], rel=st["rel_obj"], ms=st["ms"])
            log(f"mid {name}: {mid[name]}")
        summary["mid"] = mid
    log(json.dumps(summary))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(dict(summary=summary, rows=rows, rows_unseen_library=rows_unseen, loss=hist), f, indent=1)


if __name__ == "__main__":
    main()
