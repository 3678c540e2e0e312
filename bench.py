#!/usr/bin/env python
"""Benchmark of the fast-hyperspectral-reconstruction hot path on one GPU.

One step = the whole path over one synthetic scan already resident in HBM:
  -log normalisation of the counts (eq. 2)
  -> NMF subspace decomposition until the relative objective (f - f*)/f*
     reaches 1e-4 (eq. 4): multiplicative-update bulk, then exact ANLS
     polish on the float32 p
  -> 20 CGLS iterations (20 A / A^T pairs) on all K channels (eq. 5, h = 0)
  -> expansion of one slice to every bin (eq. 6).

value = view*pixel*bins of the scan / step time.  The NMF-only rate, the
projector voxel-rays/s and each kernel's share are reported beside it.
f* (the stationary objective of the instance) is computed before timing by
running the same float32 path to stationarity.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mid|tiny]
                [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
REL_OBJ = 1e-4
CGLS_ITERS = 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mid", choices=["mid", "tiny"])
    ap.add_argument("--bulk-iters", type=int, default=200)
    ap.add_argument("--polish-rounds", type=int, default=600)
    ap.add_argument("--check-every", type=int, default=200)
    ap.add_argument("--polish-bf16", type=int, default=0,
                    help="the first polish rounds run on the bfloat16 copy of p")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"],
                    help="bulk iterations on the bfloat16 copy of p (MFMA) or on the float32 p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "the hot path's multi-GPU sharding is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2410_22500_amd import hsn

    dev = torch.device("cuda:0")
    t0 = time.time()
    sc = synth.config_scan(args.workload)
    K = sc.n_mat
    n_p, n_k = sc.n_p, sc.n_bins
    vpb = n_p * n_k
    log(f"workload {args.workload}: N_v={sc.n_views} N_r={sc.n_rows} N_c={sc.n_cols} N_k={n_k} K={K} "
        f"({vpb:.3e} vpb), generated in {time.time() - t0:.1f}s")
    y = torch.from_numpy(sc.y.view(np.int16)).to(dev)
    yo = torch.from_numpy(sc.yo.view(np.int16)).to(dev)
    V0n, D0n = synth.random_factors(n_p, n_k, K, 1000 + sc.n_views)
    V0 = torch.from_numpy(V0n.astype(np.float32)).to(dev)
    D0 = torch.from_numpy(D0n.astype(np.float32)).to(dev)
    V = torch.empty_like(V0)
    D = torch.empty_like(D0)

    # f*: the lowest objective reached by long float32 runs of two schedules
    # (MU then ANLS to stationarity; MU then HALS), not timed.
    p, _, _, _ = hsn.hsn_normalize(y, yo)
    refs = []
    for algo_p, rounds in ((hsn.ALGO_ANLS, 800), (hsn.ALGO_HALS, 3000)):
        V.copy_(V0)
        D.copy_(D0)
        st = hsn.hsn_subspace_nmf(p, None, n_k, V, D, max_iter=args.bulk_iters, check_every=args.bulk_iters,
                                  polish_rounds=rounds, polish_algo=algo_p)
        hist = np.array(st["history"])
        refs.append(float(hist.min()))
        log(f"reference run polish={algo_p}: min f {hist.min():.9e}, last rel change "
            f"{abs(hist[-2] - hist[-1]) / hist[-1]:.2e}")
    f_star = min(refs)

    bf16 = args.precision == "bf16"

    def step(record=None):
        p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=bf16)
        V.copy_(V0)
        D.copy_(D0)
        s = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, max_iter=args.bulk_iters, check_every=args.check_every,
                                 precision=hsn.PREC_BF16 if bf16 else hsn.PREC_FP32,
                                 polish_rounds=args.polish_rounds, polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ,
                                 polish_bf16_rounds=args.polish_bf16 if bf16 else 0, f_ref=f_star)
        sino = V.view(sc.n_views, sc.n_rows, sc.n_cols, K)
        x = hsn.hsn_cgls(sino, CGLS_ITERS)
        hsn.hsn_rehydrate(x.view(-1, K), D, vox=(0, sc.n_cols * sc.n_cols), bins=(0, n_k))
        if record is not None:
            record.append(s)
        return s

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    hsn.hsn_profile_enable(True)
    for kk in (hsn.KERN_NMF_PASS, hsn.KERN_NMF_PASS_BF16, hsn.KERN_PROJECT, hsn.KERN_BACKPROJECT, hsn.KERN_NORMALIZE):
        hsn.hsn_profile_read(kk, reset=True)
    recs = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step(recs)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    hsn.hsn_profile_enable(False)
    ms_step = ms_total / args.steps
    nmf_ms = float(np.mean([r["ms"] for r in recs]))
    reached = all(r["rel_obj"] <= REL_OBJ for r in recs)
    pass_ms, pass_n = hsn.hsn_profile_read(hsn.KERN_NMF_PASS)
    bpass_ms, bpass_n = hsn.hsn_profile_read(hsn.KERN_NMF_PASS_BF16)
    prj_ms, prj_n = hsn.hsn_profile_read(hsn.KERN_PROJECT)
    bpj_ms, bpj_n = hsn.hsn_profile_read(hsn.KERN_BACKPROJECT)
    nrm_ms, nrm_n = hsn.hsn_profile_read(hsn.KERN_NORMALIZE)

    # Algorithmic bytes of the streaming passes over p, per kind:
    #   bfloat16 MU bulk pass: 2 B per element of p + V read and written (8K B per row);
    #   float32 ANLS round = N_V pass (4 B per element + N_V written) and
    #   N_D pass (4 B per element + V read).
    # Launches queued after the stop test fired return at once; they are
    # counted in the measured time (a few us each), so the rates are conservative.
    it, pol = recs[-1]["iters"], recs[-1]["polish_done"]
    elems = float(n_p) * n_k
    vbytes = 4.0 * n_p * K
    kinds = {}
    b_bytes = sum(r["iters"] for r in recs) * ((2.0 if bf16 else 4.0) * elems + 2 * vbytes)
    f_bytes = sum(r["polish_done"] for r in recs) * 2 * (4.0 * elems + vbytes)
    b_launch = sum(r["iters"] for r in recs)
    f_launch = sum(2 * r["polish_done"] for r in recs)
    if not bf16:
        f_bytes, f_launch = f_bytes + b_bytes, f_launch + b_launch
        b_bytes, b_launch = 0.0, 0
    if b_launch:
        kinds["nmf pass bfloat16 MFMA (pass_bf16_kernel, MU bulk)"] = (b_bytes, b_launch, bpass_ms)
    if f_launch:
        kinds["nmf pass float32 (pass_f32_kernel, ANLS N_V/N_D)" if bf16 else
              "nmf pass float32 (pass_f32_kernel)"] = (f_bytes, f_launch, pass_ms)
    dom = max(kinds, key=lambda k: kinds[k][2])
    roof = {}
    for name, (by, nl, ms) in kinds.items():
        ach = by / (ms * 1e-3) / 1e9
        roof[name] = {"achieved": ach, "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": ms / nl, "launches": nl,
                      "alg_bytes_per_launch": by / nl}
    vox_rays = sc.n_views * sc.n_rows * sc.n_cols * sc.n_cols * K

    out = {
        "metric": "view*pixel*bins decomposed/s at rel obj 1e-4 (whole hot-path step)",
        "value": vpb / (ms_step * 1e-3),
        "unit": "vpb/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32" if bf16 else "f32",
        "data": "synthetic (seeded phantom, Bragg-edge-like spectra, Poisson counts)",
        "config": {"workload": f"{args.workload}: {sc.n_rows} slices x {sc.n_cols}^2, {sc.n_views} views, "
                               f"{n_k} bins, K={K}, flux {sc.flux:g}",
                   "nmf": f"{args.precision} bulk: {args.bulk_iters} MU, then ANLS polish ({args.polish_bf16 if bf16 else 0} rounds bf16, rest float32) until rel obj {REL_OBJ:g}",
                   "recon": f"CGLS {CGLS_ITERS} pairs", "parallelism": "single GPU"},
        "nmf": {"vpb_per_s": vpb / (nmf_ms * 1e-3), "ms": nmf_ms, "mu_iters": it, "polish_rounds": pol,
                "rel_obj": recs[-1]["rel_obj"], "reached": reached, "f_star": f_star},
        "projector": {"voxel_rays_per_s_A": vox_rays / (prj_ms / prj_n * 1e-3),
                      "voxel_rays_per_s_AT": vox_rays / (bpj_ms / bpj_n * 1e-3),
                      "ms_A": prj_ms / prj_n, "ms_AT": bpj_ms / bpj_n},
        "normalize_ms": nrm_ms / max(nrm_n, 1),
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": roof[dom]["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": roof[dom]["frac"], "traffic": None,
                     "avg_launch_ms": roof[dom]["avg_launch_ms"], "launches": roof[dom]["launches"],
                     "alg_bytes_per_launch": roof[dom]["alg_bytes_per_launch"], "all_passes": roof},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, V0n, D0n, it, pol)
    print(json.dumps(out), flush=True)


def cpu_baseline(sc, V0n, D0n, mu_iters, polish_rounds):
    """The FP64 oracle as it stands, on a bounded sample of the same workload:
    detector row 0 (1 of N_r slices).  Normalisation, CGLS and the expansion
    run in full on that slice.  The NMF is timed on the first quarter of the
    slice's rays (10 MU iterations, 1 ANLS round) and extrapolated linearly
    in rows and per iteration to the slice and the counts the GPU needed.
    Rate in vpb/s of the slice."""
    from threadpoolctl import threadpool_info
    from oracle import cgls as ocgls
    from oracle import expand as oexp
    from oracle import nmf as onmf
    from oracle.normalize import normalize as onorm

    K = sc.n_mat
    ysub = sc.y[:, :1]
    yosub = sc.yo[:1]
    rows = np.arange(sc.n_p).reshape(sc.n_views, sc.n_rows, sc.n_cols)[:, 0].ravel()
    t0 = time.perf_counter()
    p, _, _ = onorm(ysub, yosub)
    t_norm = time.perf_counter() - t0
    q = max(1, p.shape[0] // 4)
    V, D = V0n[rows].astype(np.float32).astype(np.float64), D0n.astype(np.float32).astype(np.float64)
    n_mu = min(mu_iters, 10)
    t0 = time.perf_counter()
    Vq, Dq, _, _ = onmf.mu_run(p[:q], V[:q], D, n_mu)
    t_mu = (time.perf_counter() - t0) / max(n_mu, 1) * (p.shape[0] / q)
    t0 = time.perf_counter()
    onmf.anls_round(p[:q], Vq, Dq)
    t_an = (time.perf_counter() - t0) * (p.shape[0] / q)
    t0 = time.perf_counter()
    sino = V.reshape(sc.n_views, 1, sc.n_cols, K)
    x = ocgls.cgls(sino, sc.n_cols, CGLS_ITERS)
    oexp.rehydrate(x.reshape(-1, K), D)
    t_rec = time.perf_counter() - t0
    t = t_norm + t_mu * mu_iters + t_an * polish_rounds + t_rec
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    vpb = p.shape[0] * p.shape[1]
    return {"value": vpb / t, "unit": "vpb/s", "cores": threads, "kind": "oracle",
            "sample": f"detector row 0 of {sc.n_rows} ({p.shape[0]} x {p.shape[1]}): normalise, CGLS {CGLS_ITERS}, "
                      f"expansion in full; NMF timed on {q} rays ({n_mu} MU, 1 ANLS) and extrapolated to "
                      f"{mu_iters} MU + {polish_rounds} ANLS on the slice; {t:.1f}s total (estimate) on "
                      f"{os.cpu_count()} host cpus ({platform.processor() or platform.machine()})",
            "seconds": t}


if __name__ == "__main__":
    main()
