#!/usr/bin/env python
"""Benchmark of the fast-hyperspectral-reconstruction hot path on one GPU.

One step = the whole path over one synthetic scan already resident in HBM:
  -log normalisation of the counts (eq. 2), float32 p and its bfloat16 copy
  -> NMF subspace decomposition until the relative objective (f - f*)/f*
     reaches 1e-4 (eq. 4): learned start (the warm-start network on MFMA over
     the pooled bfloat16 p, then D0 by exact NNLS), then exact ANLS rounds on
     the float32 p with FP64 K x K Cholesky solves
  -> 20 CGLS iterations (20 A / A^T pairs) on all K channels (eq. 5, h = 0)
  -> expansion of one slice to every bin (eq. 6).

value = view*pixel*bins of the scan / step time.  Before timing (not timed):
the warm-start network is trained on the GPU on decompositions of 348
tiny-geometry scans made of the workload's materials (2.0 M spectra), and
f* is the lowest objective of long reference runs.  Beside the flagship
path, the plain FP32 path (NNDSVDa start, float32 MU bulk, ANLS polish) and
the cold BF16 path (NNDSVDa, bfloat16 MFMA MU bulk, ANLS polish) are timed
to the same relative objective.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mid|tiny]
                [--mlp-scans N] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (packed)
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
REL_OBJ = 1e-4
CGLS_ITERS = 20
BULK = 200
POLISH_CAP = 1500


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="full", choices=["full", "mid", "tiny", "batched", "ksweep"],
                    help="full / mid / tiny: the whole path on one scan; batched: 32 uneven decompositions; "
                         "ksweep: the subspace size study on the mid scan (K = N_m .. 2 N_m)")
    ap.add_argument("--mlp-scans", type=int, default=None, help="training scans (default 348; 40 with --quick)")
    ap.add_argument("--quick", action="store_true",
                    help="short set-up and no comparison paths or CPU baseline (for profiler runs)")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="steps of each comparison path (plain FP32, cold BF16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain device copy of 1 GiB (reference for HBM counters) and exit")
    ap.add_argument("--counters", action="store_true",
                    help="for rocprofv3 --pmc runs: only the full-size kernels of one step (normalisation with "
                         "the pooled input, 4 bfloat16 and 2 float32 ANLS rounds from a seeded start, 3 CGLS "
                         "iterations), no network training, no references, and exit")
    ap.add_argument("--traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="turn two rocprofv3 --pmc runs of this benchmark on --workload (FETCH_SIZE, WRITE_SIZE; "
                         "csv) into HBM bytes per launch of its kernels, scaled by the copy probe, and exit")
    return ap.parse_args()


# Kernels whose every launch in a workload's benchmark has that workload's
# shape: name -> (template instance prefix as rocprofv3 prints it, source).
_PRJ = "paper_2410_22500_amd/csrc/projector.hip"
TRAFFIC_KERNELS = {
    "mid": {
        "project_lds_kernel": ("project_lds_kernel<4, true>", _PRJ),
        "backproject_lds_kernel": ("backproject_lds_kernel<4, 1, true>", _PRJ),
        "xpby_transpose_kernel": ("xpby_transpose_kernel<4>", _PRJ),
        "cgls_rstep_kernel": ("cgls_rstep_kernel(", _PRJ),
        "prior_apply_kernel": ("prior_apply_kernel<4>", _PRJ),
        "mbir_step_kernel": ("mbir_step_kernel<4>", _PRJ),
    },
    "full": {
        "pass_bf16_kernel": ("pass_bf16_kernel<5, 4, ", "paper_2410_22500_amd/csrc/nmf_bf16.hip"),
        "pass_f32_kernel": ("pass_f32_kernel<5, 2, 4, true>", "paper_2410_22500_amd/csrc/nmf_f32.hip"),
        "normalize": ("normalize_", "paper_2410_22500_amd/csrc/normalize.hip"),
        "project_lds_kernel": ("project_lds_kernel<5,", _PRJ),
        "backproject_lds_kernel": ("backproject_lds_kernel<5,", _PRJ),
    },
}
WORKLOAD_TEXT = {"mid": "mid (60 views, 16 slices, 128 columns, 1024 bins, K=4)",
                 "full": "full (120 views, 256 slices, 256 columns, 2000 bins, K=5)"}


def traffic_from_counters(fetch_dir, write_dir, out_json, workload="mid"):
    """Average FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel from the
    rocprofv3 csv output, times the copy probe's bytes-per-KiB factors (kept in
    the existing record or in profiles/pmc_traffic_mid.json), with the SHA-256
    of each kernel's source file."""
    import csv
    import glob
    import hashlib

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        acc = {}
        for fn in files:
            for row in csv.DictReader(open(fn)):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                for key, (inst, _) in TRAFFIC_KERNELS[workload].items():
                    if inst in name and not (key == "project_lds_kernel" and "backproject" in name):
                        acc.setdefault(key, []).append(float(row["Counter_Value"]))
        return acc

    old = json.load(open(out_json)) if os.path.exists(out_json) else {}
    probe = old.get("copy_probe")
    if not probe:
        mid_rec = os.path.join(ROOT, "profiles", "pmc_traffic_mid.json")
        probe = json.load(open(mid_rec)).get("copy_probe") if os.path.exists(mid_rec) else None
    if not probe:
        sys.exit("--traffic: the copy probe factors are missing from " + out_json)
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    kernels = {}
    for key, (inst, src) in TRAFFIC_KERNELS[workload].items():
        if key not in fetch or key not in write:
            continue
        fk = sum(fetch[key]) / len(fetch[key])
        wk = sum(write[key]) / len(write[key])
        fb, wb = fk * 1024 * probe["fetch_factor"], wk * 1024 * probe["write_factor"]
        kernels[key] = {"instance": inst.rstrip("("), "workload": WORKLOAD_TEXT[workload],
                        "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
                        "dispatches": [len(fetch[key]), len(write[key])], "fetch_bytes": fb, "write_bytes": wb,
                        "hbm_bytes_per_launch": fb + wb, "source": src,
                        "source_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()}
    rec = {"note": old.get("note", ""), "copy_probe": probe, "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: round(v["hbm_bytes_per_launch"] / 1e6, 3) for k, v in kernels.items()}), flush=True)


def copy_probe():
    """A plain device-to-device copy of 1 GiB (float32), 10 times: the
    reference kernel whose FETCH_SIZE / WRITE_SIZE per dispatch scale the
    HBM counters of the path's kernels, and the achievable copy bandwidth."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": ms,
                      "gbs_read_plus_write": 8.0 * n / (ms * 1e-3) / 1e9}), flush=True)


def counter_run(args):
    """The hot path's kernels at the workload's shape, each launched as in a
    timed step, and nothing else at another shape: the run that rocprofv3
    --pmc counts (FETCH_SIZE, WRITE_SIZE, SQ counters).  The bfloat16 ANLS
    rounds keep the timed path's mix (the objective on every 4th round)."""
    import torch
    import synth
    from paper_2410_22500_amd import hsn

    dev = torch.device("cuda:0")
    cfg = synth.CONFIGS[args.workload]
    full = args.workload == "full"
    sc = synth.config_scan(args.workload, counts=not full)
    K, n_p, n_k = sc.n_mat, sc.n_p, sc.n_bins
    if full:
        y, yo = synth.device_counts(sc, seed=cfg["seed"] * 7919 + 1, device=dev)
    else:
        y = torch.from_numpy(sc.y.view(np.int16)).to(dev)
        yo = torch.from_numpy(sc.yo.view(np.int16)).to(dev)
    p, pb, _, _, _, bias = hsn.hsn_normalize_pooled(y, yo, hsn.PREC_BF16, want_bf16=True, want_bias=True)
    del y, yo
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    V = torch.rand((n_p, K), device=dev, generator=g) + 0.05
    D = torch.rand((n_k, K), device=dev, generator=g) + 0.05
    st = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, max_iter=0, polish_rounds=6, polish_bf16_rounds=4,
                              polish_algo=hsn.ALGO_ANLS, bf16_bias=bias)
    del p, pb
    x = hsn.hsn_cgls(V.view(sc.n_views, sc.n_rows, sc.n_cols, K), 3)
    torch.cuda.synchronize()
    log(f"counter run {args.workload}: {st['polish_bf16_done']} bf16 + "
        f"{st['polish_done'] - st['polish_bf16_done']} f32 ANLS rounds, CGLS 3, |x| {float(x.norm()):.4g}")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.traffic:
        traffic_from_counters(*args.traffic, workload=args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (got --gpus {args.gpus}); "
              "sharding across GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "ksweep":
        run_ksweep(args)
        return
    if args.counters:
        counter_run(args)
        return

    import torch
    import synth
    from paper_2410_22500_amd import hsn, warmstart

    dev = torch.device("cuda:0")
    t0 = time.time()
    cfg = synth.CONFIGS[args.workload]
    full = args.workload == "full"
    # The full workload's 15.7 G counts are drawn on the GPU (seeded Philox).
    sc = synth.config_scan(args.workload, counts=not full)
    K = sc.n_mat
    n_p, n_k = sc.n_p, sc.n_bins
    vpb = n_p * n_k
    if full:
        y, yo = synth.device_counts(sc, seed=cfg["seed"] * 7919 + 1, device=dev)
    else:
        y = torch.from_numpy(sc.y.view(np.int16)).to(dev)
        yo = torch.from_numpy(sc.yo.view(np.int16)).to(dev)
    torch.cuda.synchronize()
    log(f"workload {args.workload}: N_v={sc.n_views} N_r={sc.n_rows} N_c={sc.n_cols} N_k={n_k} K={K} "
        f"({vpb:.3e} vpb), generated in {time.time() - t0:.1f}s")
    V = torch.empty((n_p, K), dtype=torch.float32, device=dev)
    D = torch.empty((n_k, K), dtype=torch.float32, device=dev)

    # Warm-start network (not timed): trained on decompositions of tiny-geometry
    # scans made of the workload's materials (256 bins, flux 1e4: the pooled
    # input has 256 bins for any bin count).  Training at the workload's own bin
    # count and flux was measured too: the same full-size step (230.0 against
    # 231.5 ms) and a worse mid-size start (3.41 against 2.07 ms per step).
    t0 = time.time()
    n_scans = args.mlp_scans if args.mlp_scans is not None else (40 if args.quick else 348)
    geo = dict(warmstart.TRAIN_GEOMETRY)
    X, T, tt = warmstart.make_training_set(n_scans, k=K, library_seed=cfg["seed"], geometry=geo,
                                           log=lambda s: log(s))
    mlp, loss_hist, t_train = warmstart.train(X, T, k=K, epochs=args.mlp_epochs)
    n_train = int(X.shape[0])
    del X, T
    torch.cuda.empty_cache()
    log(f"network: {n_train} spectra ({n_scans} scans, {geo['n_bins']} bins, flux {geo['flux']:g}), training "
        f"{t_train:.2f}s, loss {loss_hist[0]:.3g} -> {loss_hist[-1]:.3g} (set-up {time.time() - t0:.1f}s)")

    # f*: the lowest objective of long float32 ANLS reference runs from two
    # starts (not timed); the last 100 rounds' relative decrease says how close
    # to stationary each run ended.
    p, pb, _, _, bias = hsn.hsn_normalize(y, yo, want_bf16=True, want_bias=True)
    refs = {}
    r_rounds = 100 if args.quick else (600 if full else 2000)
    for name, kw in (("nndsvda+mu+anls", dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, polish_rounds=r_rounds,
                                              precision=hsn.PREC_BF16 if full else hsn.PREC_FP32)),
                     ("learned+anls", dict(init=hsn.INIT_MLP, mlp=mlp, max_iter=0, polish_rounds=r_rounds))):
        t1 = time.time()
        st = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, check_every=BULK, polish_algo=hsn.ALGO_ANLS,
                                  anls_extrapolate=True, **kw)
        h = np.array(st["history"])
        tail = float((h[-101] - h[-1]) / h[-1]) if len(h) > 101 else None
        refs[name] = {"f": float(h.min()), "rounds": st["polish_done"], "last_100_rounds_rel_decrease": tail}
        log(f"reference {name}: min f {h.min():.9e}, last-100-round rel decrease {tail}, {time.time() - t1:.1f}s")
    f_star = min(r["f"] for r in refs.values())
    del p, pb, bias
    torch.cuda.empty_cache()

    bf16_rounds = POLISH_CAP - 100
    paths = {
        # learned start, ANLS rounds on the bfloat16 p until the bias-corrected
        # objective meets the tolerance, then float32 ANLS rounds decide the stop
        # (a learned start whose first objective is more than 50 % above f* is
        # replaced by NNDSVDa: a guard against a network that does not fit the scan)
        "learned": dict(init=hsn.INIT_MLP, mlp=mlp, max_iter=0, polish_bf16_rounds=bf16_rounds,
                        mlp_fallback_rel=0.5, anls_extrapolate=True),
        "learned_fp32": dict(init=hsn.INIT_MLP, mlp=mlp, max_iter=0, mlp_fallback_rel=0.5),
        "plain_fp32": dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, precision=hsn.PREC_FP32),
        # the paper's solver: plain NNDSVD start and Fast HALS (float32), then
        # the same ANLS rounds; with the MU bulk from the same start beside it,
        # both checking the objective every 10 bulk iterations
        "nndsvd_hals_fp32": dict(init=hsn.INIT_NNDSVD, algo=hsn.ALGO_HALS, max_iter=BULK,
                                 precision=hsn.PREC_FP32, check_every=10),
        "nndsvd_mu_fp32": dict(init=hsn.INIT_NNDSVD, max_iter=BULK, precision=hsn.PREC_FP32, check_every=10),
        "cold_bf16": dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, precision=hsn.PREC_BF16,
                          polish_bf16_rounds=bf16_rounds),
    }
    last_x = {}
    learned_bufs = {}

    def step(path, record=None):
        if path == "learned":
            # The whole path in one C call (hsn_fhr_step): one normalisation pass writes p,
            # its bfloat16 copy (with -||p - p_bf16||^2) and the network's pooled input,
            # the learned start, ANLS rounds to rel obj 1e-4, CGLS, and x^h of one slice.
            x, _, s = hsn.hsn_fhr_step(y, yo, V, D, CGLS_ITERS, vox=(0, sc.n_cols * sc.n_cols), bins=(0, n_k),
                                       bufs=learned_bufs, check_every=BULK, polish_rounds=POLISH_CAP,
                                       polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star, **paths[path])
            last_x["x"] = x
        else:
            want_b = paths[path].get("polish_bf16_rounds", 0) > 0 or paths[path].get("precision") == hsn.PREC_BF16
            p, pb, _, _, bias = hsn.hsn_normalize(y, yo, want_bf16=True, want_bias=True)
            kw = dict(paths[path])
            kw.setdefault("check_every", BULK)
            s = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, polish_rounds=POLISH_CAP,
                                     polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star,
                                     bf16_bias=bias if want_b else None, **kw)
            del p, pb
            sino = V.view(sc.n_views, sc.n_rows, sc.n_cols, K)
            x = hsn.hsn_cgls(sino, CGLS_ITERS)
            last_x["x"] = x
            hsn.hsn_rehydrate(x.view(-1, K), D, vox=(0, sc.n_cols * sc.n_cols), bins=(0, n_k))
        if record is not None:
            record.append(s)
        return s

    def timed(path, steps, profile):
        if profile:
            hsn.hsn_profile_enable(True)
            for kk in range(hsn.KERN_COUNT):
                hsn.hsn_profile_read(kk, reset=True)
        recs = []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            step(path, recs)
        e1.record()
        torch.cuda.synchronize()
        prof = {}
        if profile:
            hsn.hsn_profile_enable(False)
            prof = {kk: hsn.hsn_profile_read(kk) for kk in range(hsn.KERN_COUNT)}
        return e0.elapsed_time(e1) / steps, recs, prof

    for _ in range(args.warmup):
        step("learned")
    # The headline time comes from unprofiled steps; the same steps are then
    # repeated with the library's per-launch HIP events on, which give each
    # kernel's launch duration for the roofline (the events add host calls
    # between launches, so that repeat's step time is reported separately).
    ms_step, recs, _ = timed("learned", args.steps, False)
    ms_step_prof, recs_prof, prof = timed("learned", args.steps, True)
    nmf_ms = float(np.mean([r["ms"] for r in recs]))
    reached = all(r["rel_obj"] <= REL_OBJ for r in recs)
    if any(r["fell_back"] for r in recs):
        log("learned path: the learned start fell back to NNDSVDa")
    log(f"learned path: {ms_step:.3f} ms/step, NMF {nmf_ms:.3f} ms, rounds {recs[-1]['polish_done']} "
        f"({recs[-1]['polish_bf16_done']} on p_bf16), rel obj {recs[-1]['rel_obj']:.3e}")
    x_flag = last_x["x"].clone()
    V_flag, D_flag = V.clone(), D.clone()

    # Material decomposition tail (Alg. 2, eq. 7-9) and "FHR with FBP" against
    # DHR (Section V, Table II): the mid workload only (not part of the step).
    fmd = fbp_cmp = None
    if not full and not args.quick:
        frac = synth.volume_fractions(sc.objs, sc.n_cols, sc.n_rows, sc.n_mat)
        lab = np.where(frac.max(axis=-1) >= 0.999, frac.argmax(axis=-1), -1).astype(np.int32).ravel()
        lab_d = torch.from_numpy(lab).to(dev)
        xs = last_x["x"].reshape(-1, K)
        hsn.hsn_fmd(xs, lab_d, sc.n_mat, D)
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            hsn.hsn_fmd(xs, lab_d, sc.n_mat, D)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        fmd = {"ms": float(np.median(ts)), "voxels_per_s": xs.shape[0] / (float(np.median(ts)) * 1e-3),
               "voxels": int(xs.shape[0]), "materials": sc.n_mat, "labelled_voxels": int((lab >= 0).sum())}
        log(f"fmd tail: {fmd['ms']:.3f} ms for {xs.shape[0]} voxels")
        fbp_cmp = fbp_comparison(sc, y, yo, mlp, V, D, paths["learned_fp32"], f_star, last_x["x"])
        log(f"fbp comparison: FHR with FBP {fbp_cmp['fhr_fbp_ms']:.2f} ms, DHR {fbp_cmp['dhr_fbp_ms']:.2f} ms "
            f"({fbp_cmp['speedup']:.1f}x); SNR FHR-FBP {fbp_cmp['snr_db']['fhr_fbp']:.2f} dB, "
            f"DHR {fbp_cmp['snr_db']['dhr_fbp']:.2f} dB, FHR-CGLS {fbp_cmp['snr_db']['fhr_cgls']:.2f} dB")

    compare = {}
    compare_prof = {}
    for path in () if args.quick else ("plain_fp32", "nndsvd_hals_fp32", "nndsvd_mu_fp32", "cold_bf16",
                                       "learned_fp32"):
        step(path)
        ms_p, rp, _ = timed(path, args.compare_steps, False)
        _, rpp, pp = timed(path, args.compare_steps, True)
        compare_prof[path] = (pp, rpp)
        nm = float(np.mean([r["ms"] for r in rp]))
        compare[path] = {"ms_per_step": ms_p, "nmf_ms": nm, "nmf_vpb_per_s": vpb / (nm * 1e-3),
                         "bulk": "HALS" if paths[path].get("algo") == hsn.ALGO_HALS else "MU",
                         "mu_iters": rp[-1]["iters"], "anls_rounds": rp[-1]["polish_done"],
                         "anls_rounds_bf16": rp[-1]["polish_bf16_done"],
                         "rel_obj": rp[-1]["rel_obj"], "reached": all(r["rel_obj"] <= REL_OBJ for r in rp)}
        log(f"{path}: {ms_p:.3f} ms/step, NMF {nm:.3f} ms, {rp[-1]['iters']} {compare[path]['bulk']} + "
            f"{rp[-1]['polish_done']} ANLS "
            f"({rp[-1]['polish_bf16_done']} on p_bf16), rel obj {rp[-1]['rel_obj']:.3e}")

    # Roofline of each profiled kernel kind over the timed region: algorithmic
    # bytes (or flops) per launch / average launch time.
    elems = float(n_p) * n_k
    vb = 4.0 * n_p * K
    rounds = sum(r["polish_done"] for r in recs_prof)
    rounds_bf = sum(r["polish_bf16_done"] for r in recs_prof)
    taps = 2.0 * float(np.mean([max(abs(math.cos(v * math.pi / sc.n_views)), abs(math.sin(v * math.pi / sc.n_views)))
                                for v in range(sc.n_views)]))
    triples = float(sc.n_views) * sc.n_rows * sc.n_cols * sc.n_cols * K
    mlp_flops_row = 2.0 * (256 * 128 + 128 * 128 + 128 * 16)
    pool_b = 512.0 if mlp.precision == hsn.PREC_BF16 else 1024.0
    work = {  # kind -> (name, total algorithmic units over the timed region, bound)
        hsn.KERN_NORMALIZE: ("normalize (u16 counts -> f32 p + bf16 p + pooled network input)",
                             args.steps * (8.0 * elems + 2.0 * sc.n_rows * sc.n_cols * n_k + pool_b * n_p), "hbm"),
        hsn.KERN_NMF_PASS_BF16: ("pass_bf16_kernel (D0 solve and fused ANLS rounds over bf16 p, MFMA)",
                                 (args.steps + rounds_bf) * (2.0 * elems + vb), "hbm"),
        hsn.KERN_NMF_PASS: ("pass_f32_kernel (fused ANLS rounds over f32 p)",
                            (rounds - rounds_bf) * (4.0 * elems + vb), "hbm"),
        hsn.KERN_MLP_ROWS: ("mlp_infer2_kernel (network inference, bf16 MFMA)",
                            args.steps * mlp_flops_row * n_p, "mfma"),
        hsn.KERN_PROJECT: ("project_lds_kernel (A, Joseph footprint, K channels, LDS-staged)", None, "alu"),
        hsn.KERN_BACKPROJECT: ("backproject_lds_kernel (A^T, LDS-staged)", None, "alu"),
    }
    # Passes that did work: the learned start's D0 pass (on p_bf16, since the
    # first round is) and every round run; passes queued after the stop test
    # fired return at once (their time stays in the total).
    real = {hsn.KERN_NMF_PASS: rounds - rounds_bf, hsn.KERN_NMF_PASS_BF16: args.steps + rounds_bf}
    roof = {}
    for kk, (name, units, bound) in work.items():
        ms, n = prof.get(kk, (0.0, 0))
        if n == 0:
            continue
        queued = n
        n = real.get(kk, n)
        if n <= 0:
            continue
        if bound == "alu":
            units = n * 2.0 * taps * triples
        peak, unit = {"hbm": (HBM_PEAK_GBS, "GB/s"), "alu": (VALU_PEAK_TFLOPS, "TFLOP/s"),
                      "mfma": (MFMA_BF16_PEAK_TFLOPS, "TFLOP/s")}[bound]
        ach = units / (ms * 1e-3) / (1e9 if unit == "GB/s" else 1e12)
        roof[name] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                      "avg_launch_ms": ms / n, "launches": n, "queued": queued, "total_ms": ms,
                      "alg_per_launch": units / n}
    # HBM bytes per launch from the committed counter runs, valid only while
    # the kernel's source is the one the counters were taken on.
    traffic = load_traffic(args.workload)
    for name, r in roof.items():
        r["traffic"] = traffic.get(name.split(" ")[0])
    for path, (pp, rp) in compare_prof.items():
        it_ = sum(r["iters"] for r in rp)
        rd_ = sum(r["polish_done"] for r in rp)
        rb_ = sum(r["polish_bf16_done"] for r in rp)
        bf_bulk = paths[path].get("precision") == hsn.PREC_BF16
        ent = {}
        ms, nq = pp.get(hsn.KERN_NMF_PASS_BF16, (0.0, 0))
        nl = (it_ if bf_bulk else 0) + rb_
        if nl and ms > 0:
            by = (it_ if bf_bulk else 0) * (2.0 * elems + 2 * vb) + rb_ * (2.0 * elems + vb)
            ach = by / (ms * 1e-3) / 1e9
            ent["bf16 passes"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": ms / nl, "launches": nl, "queued": nq}
        ms, nq = pp.get(hsn.KERN_NMF_PASS, (0.0, 0))
        nl = (0 if bf_bulk else it_) + (rd_ - rb_) + (1 if path == "learned_fp32" else 0) * len(rp)
        if nl and ms > 0:
            by = (0 if bf_bulk else it_) * (4.0 * elems + 2 * vb) + (nl - (0 if bf_bulk else it_)) * (4.0 * elems + vb)
            ach = by / (ms * 1e-3) / 1e9
            ent["f32 passes"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": ms / nl, "launches": nl, "queued": nq}
        gms, gn = pp.get(hsn.KERN_NNDSVD_GRAM, (0.0, 0))
        if gn:
            fl = 2.0 * n_p * n_k * n_k
            ent["NNDSVD Gram (MFMA)"] = {"bound": "mfma", "achieved": fl / (gms / gn * 1e-3) / 1e12,
                                         "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                         "frac": fl / (gms / gn * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS,
                                         "avg_launch_ms": gms / gn, "launches": gn}
        compare[path]["roofline"] = ent
    dom = max(roof, key=lambda k: roof[k]["total_ms"])
    d = roof[dom]
    prj = roof.get(work[hsn.KERN_PROJECT][0])
    bpj = roof.get(work[hsn.KERN_BACKPROJECT][0])

    out = {
        "metric": "view*pixel*bins decomposed/s at rel obj 1e-4 (whole hot-path step)",
        "value": vpb / (ms_step * 1e-3),
        "unit": "vpb/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_profiled": ms_step_prof,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32",
        "data": "synthetic (seeded phantom, Bragg-edge-like spectra, Poisson counts)",
        "config": {"workload": f"{args.workload}: {sc.n_rows} slices x {sc.n_cols}^2, {sc.n_views} views, "
                               f"{n_k} bins, K={K}, flux {sc.flux:g}",
                   "nmf": f"learned start (bf16 MFMA network, {n_train} training spectra) + extrapolated fused ANLS "
                          f"rounds on the bf16 p (bias-corrected stop) then on the f32 p until rel obj {REL_OBJ:g}",
                   "recon": f"CGLS {CGLS_ITERS} pairs", "parallelism": "single GPU"},
        "nmf": {"vpb_per_s": vpb / (nmf_ms * 1e-3), "ms": nmf_ms, "anls_rounds": recs[-1]["polish_done"],
                "anls_rounds_bf16": recs[-1]["polish_bf16_done"], "rel_obj": recs[-1]["rel_obj"],
                "reached": reached, "fell_back": any(r["fell_back"] for r in recs), "f_star": f_star,
                "history_last_step": recs[-1]["history"],
                "references": refs,
                "f_star_note": "lowest objective of the float32 extrapolated-ANLS reference runs; their "
                               "last-100-round relative decrease bounds how far from stationary they ended"},
        "compare": compare,
        "speedup_vs_plain_fp32": ({"nmf": compare["plain_fp32"]["nmf_ms"] / nmf_ms,
                                   "step": compare["plain_fp32"]["ms_per_step"] / ms_step}
                                  if "plain_fp32" in compare else None),
        "fmd_tail": fmd,
        "fbp_comparison": fbp_cmp,
        "network": {"train_spectra": n_train, "train_scans": n_scans, "train_geometry": geo,
                    "library": f"the workload's material library (spectra seed {cfg['seed']})",
                    "epochs": args.mlp_epochs, "train_s": t_train, "loss_first": loss_hist[0],
                    "loss_last": loss_hist[-1]},
        "projector": {"voxel_rays_per_s_A": triples / (prj["avg_launch_ms"] * 1e-3) if prj else None,
                      "voxel_rays_per_s_AT": triples / (bpj["avg_launch_ms"] * 1e-3) if bpj else None,
                      "ms_A": prj["avg_launch_ms"] if prj else None, "ms_AT": bpj["avg_launch_ms"] if bpj else None},
        "roofline": {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                     "unit": d["unit"], "frac": d["frac"], "traffic": d["traffic"],
                     "avg_launch_ms": d["avg_launch_ms"], "launches": d["launches"],
                     "alg_per_launch": d["alg_per_launch"], "all_kernels": roof},
    }
    if not args.no_cpu_baseline and not args.quick:
        plain = compare.get("plain_fp32", {"mu_iters": BULK, "anls_rounds": 15})
        cb, err = cpu_baseline(sc, y, yo, learned_bufs["p"], x_flag, V_flag, D_flag, plain["mu_iters"],
                               plain["anls_rounds"])
        out["cpu_baseline"] = cb
        out["error_vs_fp64"] = err
    print(json.dumps(out), flush=True)


def load_traffic(workload):
    """kernel -> HBM bytes per launch of the workload's kernels from
    profiles/pmc_traffic_<workload>.json (rocprofv3 FETCH_SIZE / WRITE_SIZE
    scaled by the copy probe), for kernels whose source file still hashes to
    the value recorded with the counters."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    out = {}
    for name, k in rec.get("kernels", {}).items():
        src = os.path.join(ROOT, k["source"])
        if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == k["source_sha256"]:
            out[name] = k["hbm_bytes_per_launch"]
    return out


def fbp_comparison(sc, y, yo, mlp, V, D, learned_kw, f_star, x_cgls):
    """FHR with FBP vs DHR (one FBP per bin) on the same counts: times and SNR_FHR."""
    import torch
    import synth
    from paper_2410_22500_amd import hsn

    n_k, K = sc.n_bins, V.shape[1]
    n_x = sc.n_rows * sc.n_cols * sc.n_cols
    dev = V.device
    # regions from the phantom: pure-material voxels, and empty voxels in the field of view
    frac = synth.volume_fractions(sc.objs, sc.n_cols, sc.n_rows, sc.n_mat).reshape(n_x, sc.n_mat)
    g = np.arange(sc.n_cols) - (sc.n_cols - 1) / 2.0
    rr = np.sqrt(g[None, :] ** 2 + g[:, None] ** 2)
    fov = np.broadcast_to(rr < sc.n_cols / 2.0 - 2.0, (sc.n_rows, sc.n_cols, sc.n_cols)).reshape(n_x)
    regions = [torch.from_numpy(np.nonzero(frac[:, m] >= 0.999)[0]).to(dev) for m in range(sc.n_mat)]
    regions = [r for r in regions if r.numel() >= 20]
    bg = torch.from_numpy(np.nonzero((frac.sum(axis=1) == 0) & fov)[0]).to(dev)

    def snr(values_at):  # values_at(idx) -> [len(idx)][n_k]
        sig = torch.stack([values_at(r).double().mean(dim=0) for r in regions])  # [N_m][N_k]
        sd = values_at(bg).double().std(dim=0)
        return float(10.0 * torch.log10(((sig / sd) ** 2).mean()))

    def fhr():
        p, _, pooled, _, _ = hsn.hsn_normalize_pooled(y, yo, mlp.precision)
        hsn.hsn_subspace_nmf(p, None, n_k, V, D, check_every=BULK, polish_rounds=POLISH_CAP,
                             polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star, mlp_pooled=pooled,
                             **learned_kw)
        xs = hsn.hsn_fbp(V, sc.n_views, sc.n_rows, sc.n_cols, K)
        return xs, hsn.hsn_rehydrate(xs.view(-1, K), D)

    # FHR with MBIR (eq. (5) with the qGGMRF prior): started from the K-channel
    # FBP; sigma_v per channel from the subspace sinogram's RMS at 30 dB, sigma_x
    # per channel 0.2 x the FBP image's RMS (stated readings, no paper values).
    mbir_cfg = dict(p=1.2, T=1.0, n_outer=10, n_inner=4, snr_db=30.0, sigma_x_frac=0.2)

    def fhr_mbir():
        p, _, pooled, _, _ = hsn.hsn_normalize_pooled(y, yo, mlp.precision)
        hsn.hsn_subspace_nmf(p, None, n_k, V, D, check_every=BULK, polish_rounds=POLISH_CAP,
                             polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star, mlp_pooled=pooled,
                             **learned_kw)
        x0 = hsn.hsn_fbp(V, sc.n_views, sc.n_rows, sc.n_cols, K)
        sv = (V.double().pow(2).mean(dim=0).sqrt() * 10.0 ** (-mbir_cfg["snr_db"] / 20.0)).tolist()
        sx = (x0.view(-1, K).double().pow(2).mean(dim=0).sqrt() * mbir_cfg["sigma_x_frac"]).tolist()
        xs = hsn.hsn_mbir(V.view(sc.n_views, sc.n_rows, sc.n_cols, K), sv, sx, p=mbir_cfg["p"], T=mbir_cfg["T"],
                          n_outer=mbir_cfg["n_outer"], n_inner=mbir_cfg["n_inner"], x0=x0)
        return xs, hsn.hsn_rehydrate(xs.view(-1, K), D)

    n_ch = (n_k + 7) // 8
    xd = [torch.empty((sc.n_rows, sc.n_cols, sc.n_cols, min(8, n_k - 8 * c)), device=dev) for c in range(n_ch)]

    def dhr():
        p, _, _, _ = hsn.hsn_normalize(y, yo)
        for c in range(n_ch):
            hsn.hsn_fbp(p[:, 8 * c:], sc.n_views, sc.n_rows, sc.n_cols, xd[c].shape[-1], ld=p.stride(0), out=xd[c])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    t_fhr, (xs, xh) = timed(fhr)
    snr_fhr = snr(lambda idx: xh[idx])
    del xs, xh
    t_mbir, (xs, xh) = timed(fhr_mbir)
    snr_mbir = snr(lambda idx: xh[idx])
    del xs, xh
    t_dhr, _ = timed(dhr)
    snr_dhr = snr(lambda idx: torch.cat([x.view(n_x, -1)[idx] for x in xd], dim=1))
    Dd = D.double()
    snr_cgls = snr(lambda idx: x_cgls.reshape(n_x, K)[idx].double() @ Dd.T)
    del xd
    return {"fhr_fbp_ms": t_fhr, "fhr_mbir_ms": t_mbir, "dhr_fbp_ms": t_dhr, "speedup": t_dhr / t_fhr,
            "snr_db": {"fhr_fbp": snr_fhr, "fhr_mbir": snr_mbir, "dhr_fbp": snr_dhr, "fhr_cgls": snr_cgls},
            "mbir": mbir_cfg,
            "regions": {"materials": len(regions), "voxels_per_material": [int(r.numel()) for r in regions],
                        "background_voxels": int(bg.numel())},
            "what": "FHR-FBP = normalise + learned NMF (to rel obj 1e-4) + K-channel FBP + x^h = x^s D^T for all "
                    "voxels and bins; FHR-MBIR = the same with qGGMRF-MBIR started from the FBP; "
                    "DHR = normalise + one FBP per bin (8 bins per launch)",
            "paper_table_ii": {"dhr_min": 817.44, "fhr_fbp_min": 23.62, "fhr_mbir_min": 62.96, "snr_dhr_db": -2.33,
                               "snr_fhr_fbp_db": 26.34, "snr_fhr_mbir_db": 42.13,
                               "note": "simulated data, whole pipelines on the paper's hardware: context only"}}


KSWEEP_ROUNDS = 60


def run_ksweep(args):
    """Subspace size study (Section V-D: N_s = beta N_m; the paper finds beta = 1 enough on simulated
    data, 2 on measured data): on the mid scan (N_m = 4 materials), for K = N_m .. min(2 N_m, 8),
    the plain method (NNDSVDa, 200 MU, 60 extrapolated ANLS rounds: a fixed schedule, since each K has
    its own optimum), 20 CGLS iterations on the K channels, and the semi-supervised material tail
    (Alg. 2 with the phantom's pure-material voxels as masks).  Reports, per K, the relative NMF
    residual f / ||p||^2, the times, SNR_FMD (eq. 12) of the material images, SNR_FHR (eq. 11) of the
    rehydrated reconstruction and the error of the estimated material spectra D^m against the
    generator's (relative Frobenius)."""
    import torch
    import synth
    from paper_2410_22500_amd import hsn

    dev = torch.device("cuda:0")
    sc = synth.config_scan("mid")
    n_m, n_k = sc.n_mat, sc.n_bins
    n_v, n_r, n_c = sc.n_views, sc.n_rows, sc.n_cols
    n_p, n_x = sc.n_p, sc.n_rows * sc.n_cols * sc.n_cols
    y = torch.from_numpy(sc.y.view(np.int16)).to(dev)
    yo = torch.from_numpy(sc.yo.view(np.int16)).to(dev)
    p, _, _, psq = hsn.hsn_normalize(y, yo)
    psq = float(psq)
    frac = synth.volume_fractions(sc.objs, n_c, n_r, n_m).reshape(n_x, n_m)
    lab = np.where(frac.max(axis=-1) >= 0.999, frac.argmax(axis=-1), -1).astype(np.int32)
    lab_d = torch.from_numpy(lab).to(dev)
    g = np.arange(n_c) - (n_c - 1) / 2.0
    fov = np.broadcast_to(np.sqrt(g[None, :] ** 2 + g[:, None] ** 2) < n_c / 2.0 - 2.0, (n_r, n_c, n_c)).reshape(n_x)
    regions = [torch.from_numpy(np.nonzero(lab == m)[0]).to(dev) for m in range(n_m)]
    bg = torch.from_numpy(np.nonzero((frac.sum(axis=1) == 0) & fov)[0]).to(dev)
    mu = torch.from_numpy(np.asarray(sc.mu, np.float64)).to(dev)  # [n_k][n_m], the generator's spectra
    log(f"ksweep: mid scan N_v={n_v} N_r={n_r} N_c={n_c} N_k={n_k} N_m={n_m}; "
        f"pure voxels per material {[int(r.numel()) for r in regions]}, background {int(bg.numel())}")

    def timed(fn):  # the second of two runs (the first allocates workspaces)
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    rows = []
    for K in range(n_m, min(2 * n_m, 8) + 1):
        V = torch.empty((n_p, K), dtype=torch.float32, device=dev)
        D = torch.empty((n_k, K), dtype=torch.float32, device=dev)
        st, nmf_ms = timed(lambda: hsn.hsn_subspace_nmf(
            p, None, n_k, V, D, algo=hsn.ALGO_MU, max_iter=BULK, check_every=BULK, polish_rounds=KSWEEP_ROUNDS,
            polish_algo=hsn.ALGO_ANLS, init=hsn.INIT_NNDSVDA, anls_extrapolate=True))
        xs, cgls_ms = timed(lambda: hsn.hsn_cgls(V.view(n_v, n_r, n_c, K), CGLS_ITERS))
        (T, xm, Dm), fmd_ms = timed(lambda: hsn.hsn_fmd(xs.view(n_x, K), lab_d, n_m, D))
        xmd = xm.double()
        snr_fmd = float(10.0 * torch.log10(torch.stack(
            [(xmd[r, m].mean() / xmd[bg, m].std(unbiased=False)) ** 2 for m, r in enumerate(regions)]).mean()))
        Dd, xsd = D.double(), xs.view(n_x, K).double()
        sig = torch.stack([(xsd[r] @ Dd.T).mean(dim=0) for r in regions])  # [n_m][n_k]
        sd = (xsd[bg] @ Dd.T).std(dim=0, unbiased=False)
        snr_fhr = float(10.0 * torch.log10(((sig / sd) ** 2).mean()))
        mu_err = float(torch.linalg.norm(Dm.double() - mu) / torch.linalg.norm(mu))
        row = {"K": K, "beta": K / n_m, "rel_resid": st["objective"] / psq, "anls_rounds": st["polish_done"],
               "nmf_ms": nmf_ms, "cgls_ms": cgls_ms, "fmd_ms": fmd_ms, "snr_fmd_db": snr_fmd, "snr_fhr_db": snr_fhr,
               "mu_rel_err": mu_err}
        rows.append(row)
        log(f"ksweep K={K}: f/|p|^2 {row['rel_resid']:.4e}, NMF {nmf_ms:.1f} ms, CGLS {cgls_ms:.1f} ms, "
            f"SNR_FMD {snr_fmd:.2f} dB, SNR_FHR {snr_fhr:.2f} dB, spectra error {mu_err:.3e}")
    print(json.dumps({"metric": "k_sweep", "unit": "per K", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                      "config": {"workload": f"ksweep: mid scan, {n_r} slices x {n_c}^2, {n_v} views, {n_k} bins, "
                                             f"{n_m} materials; K = {n_m} .. {rows[-1]['K']}",
                                 "schedule": f"NNDSVDa, {BULK} MU, {KSWEEP_ROUNDS} extrapolated ANLS rounds, "
                                             f"CGLS {CGLS_ITERS}, FMD with pure-voxel masks"},
                      "rows": rows}), flush=True)


def run_batched(args):
    """32 uneven decompositions (views 30-180, columns 64-256, bins 512-2048,
    K 2-6, one slice each): MU bulk (200 iterations, float32 or bfloat16 on
    the matrix cores) then float32 ANLS rounds until each instance's relative
    objective reaches 1e-4, from seeded random starts.  Timed: 32
    per-instance calls one after the other, and the batched call (one launch
    per phase and kernel shape) without graphs, with graphs, and with graphs
    and the autotuned partition, for both bulk precisions."""
    import torch
    import synth
    from paper_2410_22500_amd import hsn

    t0 = time.time()
    scans = synth.batched_scans(32, 3)
    insts = []
    for i, sc in enumerate(scans):
        y = torch.from_numpy(sc.y.view(np.int16)).cuda()
        yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
        p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
        V0, D0 = synth.random_factors(sc.n_p, sc.n_bins, sc.n_mat, 500 + i)
        insts.append(dict(p=p, pb=pb, n_k=sc.n_bins, V0=torch.from_numpy(V0.astype(np.float32)).cuda(),
                          D0=torch.from_numpy(D0.astype(np.float32)).cuda()))
    elems = float(sum(sc.n_p * sc.n_bins for sc in scans))
    log(f"batched: {len(scans)} instances, {elems:.3e} elements, generated in {time.time() - t0:.1f}s")
    for x in insts:
        x["V"] = torch.empty_like(x["V0"])
        x["D"] = torch.empty_like(x["D0"])

    def reset():
        for x in insts:
            x["V"].copy_(x["V0"])
            x["D"].copy_(x["D0"])

    # f* per instance: a long batched run (not timed).
    reset()
    st = hsn.hsn_subspace_nmf_batched([(x["p"], x["n_k"], x["V"], x["D"], 0.0) for x in insts], max_iter=BULK,
                                      check_every=BULK, polish_rounds=1000, flags=hsn.BATCH_GRAPH)
    f_ref = [min(s["history"]) for s in st]
    kw = dict(max_iter=BULK, check_every=BULK, polish_rounds=POLISH_CAP, rel_obj_tol=REL_OBJ)

    def per_instance(prec=hsn.PREC_FP32):
        out = []
        for x, f in zip(insts, f_ref):
            out.append(hsn.hsn_subspace_nmf(x["p"], x["pb"] if prec == hsn.PREC_BF16 else None, x["n_k"], x["V"],
                                            x["D"], polish_algo=hsn.ALGO_ANLS, f_ref=f, precision=prec, **kw))
        return out

    def batched(flags, prec=hsn.PREC_FP32):
        return hsn.hsn_subspace_nmf_batched([(x["p"], x["n_k"], x["V"], x["D"], f, x["pb"])
                                             for x, f in zip(insts, f_ref)], flags=flags, precision=prec, **kw)

    bf = hsn.PREC_BF16
    runs = {"per_instance": per_instance, "batched": lambda: batched(0),
            "batched_graph": lambda: batched(hsn.BATCH_GRAPH),
            "batched_graph_autotuned": lambda: batched(hsn.BATCH_GRAPH | hsn.BATCH_AUTOTUNE),
            "per_instance_bf16": lambda: per_instance(bf),
            "batched_bf16_graph": lambda: batched(hsn.BATCH_GRAPH, bf),
            "batched_bf16_graph_autotuned": lambda: batched(hsn.BATCH_GRAPH | hsn.BATCH_AUTOTUNE, bf)}
    res = {}
    for name, fn in runs.items():
        reset()
        fn()  # warm-up (plan, graphs, tuning)
        times, last = [], None
        for _ in range(args.steps):
            reset()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            last = fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        reached = sum(s["rel_obj"] <= REL_OBJ for s in last)
        steps = sum(s["iters"] + s["polish_done"] for s in last)
        res[name] = {"ms": ms, "vpb_per_s": elems / (ms * 1e-3), "reached": reached, "steps": steps}
        if name.startswith("batched"):
            res[name]["plan"] = hsn.hsn_batched_plan_info()
        log(f"{name}: {ms:.2f} ms, {reached}/{len(last)} reached rel obj {REL_OBJ:g}, {steps} steps in total")
    best_name = "batched_bf16_graph_autotuned"
    best = res[best_name]
    out = {
        "metric": "view*pixel*bins decomposed/s at rel obj 1e-4 (32 uneven decompositions)",
        "value": best["vpb_per_s"], "unit": "vpb/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32", "data": "synthetic (seeded phantoms, Bragg-edge-like spectra, Poisson counts)",
        "config": {"workload": "batched: 32 instances, views 30-180, columns 64-256, bins 512-2048, K 2-6, "
                               "one slice each, flux 1e4",
                   "nmf": f"MU {BULK} on the bf16 p (MFMA) + f32 ANLS until rel obj {REL_OBJ:g}",
                   "parallelism": "single GPU"},
        "runs": res,
        "speedup_vs_per_instance": {"bf16": res["per_instance_bf16"]["ms"] / best["ms"],
                                    "f32": res["per_instance"]["ms"] / res["batched_graph_autotuned"]["ms"]},
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(sc, y, yo, p_gpu, x_gpu, V_gpu, D_gpu, mu_iters, polish_rounds):
    """The FP64 oracle as it stands, on a bounded sample of the same workload
    (detector row 0, one slice of N_r), running the plain method: the
    normalisation, NNDSVDa, `mu_iters` MU iterations and `polish_rounds` ANLS
    rounds (the counts the plain FP32 GPU path needed), CGLS and the
    expansion.  Timed parts: normalisation and the expansion in full, two MU
    iterations on the slice, NNDSVDa and one ANLS round on a quarter of its
    rays, two CGLS iterations on the slice; each is extrapolated linearly (in
    rays and iterations) to the slice's run, and the rate (vpb/s of the slice)
    holds for the whole scan under linear extrapolation in N_r.  A second run
    of the sampled parts on one thread gives the single-core rate.

    The same leg measures each GPU result against the oracle on that sample
    (error_vs_fp64): p, one exact ANLS round from the flagship's final (V, D)
    (sampled V rows; the NNLS optimality of sampled D rows), A and A^T, three
    CGLS iterations and the expansion, on slice 0."""
    import platform
    import torch
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import cgls as ocgls
    from oracle import expand as oexp
    from oracle import nmf as onmf
    from oracle import nnls as onnls
    from oracle import projector as oprj
    from oracle.normalize import normalize as onorm
    import synth
    from paper_2410_22500_amd import hsn

    K, n_k = sc.n_mat, sc.n_bins
    n_v, n_r, n_c = sc.n_views, sc.n_rows, sc.n_cols
    y0 = y[:, 0:1].cpu().numpy().view(np.uint16)
    yo0 = yo[0:1].cpu().numpy().view(np.uint16)

    def sample_times():
        t = {}
        t0 = time.perf_counter()
        p0, _, _ = onorm(y0, yo0)
        t["normalize"] = time.perf_counter() - t0
        n0 = p0.shape[0]
        q = n0 // 4
        t0 = time.perf_counter()
        Vq, Dq = onmf.nndsvd(p0[:q], K, variant="a")
        t["nndsvda"] = (time.perf_counter() - t0) * n0 / q
        V0, D0 = synth.random_factors(n0, n_k, K, 3)
        t0 = time.perf_counter()
        onmf.mu_run(p0, V0, D0, 2)
        t["mu_iter"] = (time.perf_counter() - t0) / 2
        t0 = time.perf_counter()
        onmf.anls_round(p0[:q], Vq, Dq)
        t["anls_round"] = (time.perf_counter() - t0) * n0 / q
        sino = V0.reshape(n_v, 1, n_c, K)
        t0 = time.perf_counter()
        xs = ocgls.cgls(sino, n_c, 2)
        t["cgls_iter"] = (time.perf_counter() - t0) / 2
        t0 = time.perf_counter()
        oexp.rehydrate(xs.reshape(-1, K), D0)
        t["rehydrate"] = time.perf_counter() - t0
        total = (t["normalize"] + t["nndsvda"] + mu_iters * t["mu_iter"] + polish_rounds * t["anls_round"]
                 + CGLS_ITERS * t["cgls_iter"] + t["rehydrate"])
        return p0, t, total

    t_all = time.perf_counter()
    p0, parts, total = sample_times()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        _, parts1, total1 = sample_times()
    vpb0 = p0.shape[0] * n_k
    cpu_model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cb = {"value": vpb0 / total, "unit": "vpb/s", "cores": threads, "kind": "oracle",
          "sample": f"detector row 0 of {n_r} ({p0.shape[0]} x {n_k}): the plain method (normalise, NNDSVDa, "
                    f"{mu_iters} MU, {polish_rounds} ANLS, CGLS {CGLS_ITERS}, expansion) extrapolated from timed "
                    f"parts (2 MU on the slice, NNDSVDa and 1 ANLS round on a quarter of its rays, 2 CGLS "
                    f"iterations); extrapolated: {total:.1f} s for the slice, x {n_r} slices for the scan",
          "extrapolated": True, "seconds_slice_estimate": total, "parts_s": parts,
          "single_thread": {"value": vpb0 / total1, "seconds_slice_estimate": total1, "parts_s": parts1},
          "host_cpus": os.cpu_count(), "cpu_model": cpu_model}

    # --- error of the GPU results against the oracle on slice 0 ---------------
    def rel(a, b):
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    err = {"sample": "detector row 0 (slice 0)"}
    ldp = p_gpu.shape[1]
    pg0 = p_gpu.view(n_v, n_r, n_c, ldp)[:, 0, :, :n_k].reshape(-1, n_k).cpu().numpy().astype(np.float64)
    rms = float(np.sqrt(np.mean(p0 * p0)))
    err["p"] = {"rel_fro": rel(pg0, p0), "max_abs_over_rms": float(np.abs(pg0 - p0).max() / rms)}
    # one exact ANLS round (the fused float32 pass) from the flagship's result
    Vt, Dt = V_gpu.clone(), D_gpu.clone()
    hsn.hsn_subspace_nmf(p_gpu, None, n_k, Vt, Dt, algo=hsn.ALGO_ANLS, max_iter=1, check_every=1)
    d0 = D_gpu.cpu().numpy().astype(np.float64)
    G = d0.T @ d0
    rows = np.random.Generator(np.random.PCG64(11)).choice(p0.shape[0], size=min(2048, p0.shape[0]), replace=False)
    rows.sort()
    ref_v = np.stack([onnls.nnls_gram(G, p0[i] @ d0) for i in rows])
    gpu_rows = (rows // n_c) * (n_r * n_c) + (rows % n_c)
    got_v = Vt[torch.from_numpy(gpu_rows).to(Vt.device)].cpu().numpy().astype(np.float64)
    err["anls_round_V_rows"] = {"rel_fro": rel(got_v, ref_v), "rows": int(len(rows))}
    V1 = Vt.cpu().numpy().astype(np.float64)
    GV = V1.T @ V1
    D1 = Dt.cpu().numpy().astype(np.float64)
    kkt = []
    for b in np.linspace(0, n_k - 1, 8).astype(int):
        h = V1.T @ p_gpu[:, b].cpu().numpy().astype(np.float64)
        grad = GV @ D1[b] - h
        kkt.append(float(np.linalg.norm(np.minimum(D1[b], grad)) / max(np.abs(h).max(), 1e-300)))
    err["anls_round_D_rows_kkt"] = {"max_rel": max(kkt), "bins": 8,
                                    "what": "||min(d, G_V d - V^T p_k)|| / max|V^T p_k| per sampled bin k"}
    # projector, CGLS and expansion on slice 0
    x0 = x_gpu[0:1].contiguous()
    s_gpu = hsn.hsn_project(x0, n_v)
    err["A"] = {"rel_fro": rel(s_gpu.cpu().numpy(), oprj.project(x0.cpu().numpy().astype(np.float64), n_v))}
    s0 = V_gpu.view(n_v, n_r, n_c, K)[:, 0:1].contiguous()
    xb = hsn.hsn_backproject(s0)
    err["AT"] = {"rel_fro": rel(xb.cpu().numpy(), oprj.backproject(s0.cpu().numpy().astype(np.float64), n_c))}
    xc = hsn.hsn_cgls(s0, 3)
    err["cgls_3_iters"] = {"rel_fro": rel(xc.cpu().numpy(), ocgls.cgls(s0.cpu().numpy().astype(np.float64), n_c, 3))}
    xs_flat = x_gpu.view(-1, K)
    xh = hsn.hsn_rehydrate(xs_flat, D_gpu, vox=(0, 1024), bins=(0, n_k))
    err["rehydrate"] = {"rel_fro": rel(xh.cpu().numpy(), oexp.rehydrate(
        xs_flat[:1024].cpu().numpy().astype(np.float64), d0))}
    cb["seconds_total"] = time.perf_counter() - t_all
    return cb, err


if __name__ == "__main__":
    main()
