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
    ap.add_argument("--workload", default="mid", choices=["mid", "tiny", "full", "batched"],
                    help="mid / tiny / full: the whole path on one scan; batched: 32 uneven decompositions")
    ap.add_argument("--mlp-scans", type=int, default=348)
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="steps of each comparison path (plain FP32, cold BF16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain device copy of 1 GiB (reference for HBM counters) and exit")
    ap.add_argument("--traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="turn two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, WRITE_SIZE; csv) into "
                         "HBM bytes per launch of the mid-shape kernels, scaled by the copy probe, and exit")
    return ap.parse_args()


# Kernels whose every launch in the mid benchmark has the mid shape (the CGLS
# and MBIR loops of the measured steps), their template instance and source.
TRAFFIC_KERNELS = {
    "project_lds_kernel": ("project_lds_kernel<4, true>", "paper_2410_22500_amd/csrc/projector.hip"),
    "backproject_lds_kernel": ("backproject_lds_kernel<4, 1, true>", "paper_2410_22500_amd/csrc/projector.hip"),
    "xpby_transpose_kernel": ("xpby_transpose_kernel<4>", "paper_2410_22500_amd/csrc/projector.hip"),
    "cgls_rstep_kernel": ("cgls_rstep_kernel(", "paper_2410_22500_amd/csrc/projector.hip"),
    "prior_apply_kernel": ("prior_apply_kernel<4>", "paper_2410_22500_amd/csrc/projector.hip"),
    "mbir_step_kernel": ("mbir_step_kernel<4>", "paper_2410_22500_amd/csrc/projector.hip"),
}


def traffic_from_counters(fetch_dir, write_dir, out_json):
    """Average FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel from the
    rocprofv3 csv output, times the copy probe's bytes-per-KiB factors (kept in
    the existing record), with the SHA-256 of each kernel's source file."""
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
                for key, (inst, _) in TRAFFIC_KERNELS.items():
                    if inst in name and not (key == "project_lds_kernel" and "backproject" in name):
                        acc.setdefault(key, []).append(float(row["Counter_Value"]))
        return acc

    old = json.load(open(out_json)) if os.path.exists(out_json) else {}
    probe = old.get("copy_probe")
    if not probe:
        sys.exit("--traffic: the copy probe factors are missing from " + out_json)
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    kernels = {}
    for key, (inst, src) in TRAFFIC_KERNELS.items():
        if key not in fetch or key not in write:
            continue
        fk = sum(fetch[key]) / len(fetch[key])
        wk = sum(write[key]) / len(write[key])
        fb, wb = fk * 1024 * probe["fetch_factor"], wk * 1024 * probe["write_factor"]
        kernels[key] = {"instance": inst.rstrip("("), "workload": "mid (60 views, 16 slices, 128 columns, K=4)",
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.traffic:
        traffic_from_counters(*args.traffic)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (got --gpus {args.gpus}); "
              "sharding across GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        run_batched(args)
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

    # Warm-start network: trained on the workload's material library (not timed).
    t0 = time.time()
    X, T, tt = warmstart.make_training_set(args.mlp_scans, k=K, library_seed=cfg["seed"],
                                           log=lambda s: log(s))
    mlp, loss_hist, t_train = warmstart.train(X, T, k=K, epochs=args.mlp_epochs)
    n_train = int(X.shape[0])
    del X, T
    log(f"network: {n_train} spectra, training {t_train:.2f}s, loss {loss_hist[0]:.3g} -> {loss_hist[-1]:.3g} "
        f"(set-up {time.time() - t0:.1f}s)")

    # f*: lowest objective of long float32 reference runs (not timed).
    p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
    refs = {}
    # (the full workload's reference runs are shorter: an ANLS round streams 126 GB there)
    r_anls, r_hals = (400, 600) if full else (2000, 3000)
    for name, kw in (("nndsvda+mu+anls", dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, polish_algo=hsn.ALGO_ANLS,
                                              polish_rounds=r_anls, precision=hsn.PREC_BF16 if full else
                                              hsn.PREC_FP32)),
                     ("nndsvda+mu+hals", dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, polish_algo=hsn.ALGO_HALS,
                                              polish_rounds=r_hals, precision=hsn.PREC_BF16 if full else
                                              hsn.PREC_FP32)),
                     ("learned+anls", dict(init=hsn.INIT_MLP, mlp=mlp, max_iter=0, polish_algo=hsn.ALGO_ANLS,
                                           polish_rounds=r_anls))):
        st = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, check_every=BULK, **kw)
        h = np.array(st["history"])
        refs[name] = float(h.min())
        log(f"reference {name}: min f {h.min():.9e}, last rel change {abs(h[-2] - h[-1]) / h[-1]:.2e}")
    f_star = min(refs.values())
    del p, pb

    paths = {
        "learned": dict(init=hsn.INIT_MLP, mlp=mlp, max_iter=0),
        "plain_fp32": dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, precision=hsn.PREC_FP32),
        "cold_bf16": dict(init=hsn.INIT_NNDSVDA, max_iter=BULK, precision=hsn.PREC_BF16),
    }

    last_x = {}

    learned_bufs = {}

    def step(path, record=None):
        if path == "learned":
            # The whole path in one C call (hsn_fhr_step): one normalisation pass writes p
            # and the network's pooled input (no bfloat16 copy of p), the learned start and
            # ANLS rounds to rel obj 1e-4, CGLS, and x^h of one slice; buffers are reused.
            x, _, s = hsn.hsn_fhr_step(y, yo, V, D, CGLS_ITERS, vox=(0, sc.n_cols * sc.n_cols), bins=(0, n_k),
                                       bufs=learned_bufs, check_every=BULK, polish_rounds=POLISH_CAP,
                                       polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star, **paths[path])
            last_x["x"] = x
            if record is not None:
                record.append(s)
            return s
        else:
            p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
            s = hsn.hsn_subspace_nmf(p, pb, n_k, V, D, check_every=BULK, polish_rounds=POLISH_CAP,
                                     polish_algo=hsn.ALGO_ANLS, rel_obj_tol=REL_OBJ, f_ref=f_star, **paths[path])
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
    log(f"learned path: {ms_step:.3f} ms/step, NMF {nmf_ms:.3f} ms, rounds {recs[-1]['polish_done']}, "
        f"rel obj {recs[-1]['rel_obj']:.3e}")

    # Material decomposition tail (Alg. 2, eq. 7-9) on the reconstructed
    # subspace volume, with the phantom's pure-material voxels as the region
    # labels (timed on its own; not part of the step).
    fmd = None
    if not full:
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

    # "FHR with FBP" against DHR (Section V, Table II): the paper's baseline
    # reconstructs every wavelength bin by FBP; FHR reconstructs the K
    # subspace sinograms and rehydrates x^h = x^s D^T (eq. 6) for every voxel
    # and bin.  Both from the counts, timed once after a warm-up each; SNR as
    # in the paper's SNR_FHR (mean over bins and materials of (region mean /
    # background deviation)^2), with the phantom's pure-material voxels as
    # the material regions and its empty voxels inside the field of view as
    # the background.  Not part of the headline step.
    fbp_cmp = None
    if not full:
        fbp_cmp = fbp_comparison(sc, y, yo, mlp, V, D, paths["learned"], f_star, last_x["x"])
        log(f"fbp comparison: FHR with FBP {fbp_cmp['fhr_fbp_ms']:.2f} ms, DHR {fbp_cmp['dhr_fbp_ms']:.2f} ms "
            f"({fbp_cmp['speedup']:.1f}x); SNR FHR-FBP {fbp_cmp['snr_db']['fhr_fbp']:.2f} dB, "
            f"DHR {fbp_cmp['snr_db']['dhr_fbp']:.2f} dB, FHR-CGLS {fbp_cmp['snr_db']['fhr_cgls']:.2f} dB")

    compare = {}
    compare_prof = {}
    for path in ("plain_fp32", "cold_bf16"):
        step(path)
        ms_p, rp, _ = timed(path, args.compare_steps, False)
        _, rpp, pp = timed(path, args.compare_steps, True)
        compare_prof[path] = (pp, rpp)
        nm = float(np.mean([r["ms"] for r in rp]))
        compare[path] = {"ms_per_step": ms_p, "nmf_ms": nm, "nmf_vpb_per_s": vpb / (nm * 1e-3),
                         "mu_iters": rp[-1]["iters"], "anls_rounds": rp[-1]["polish_done"],
                         "rel_obj": rp[-1]["rel_obj"], "reached": all(r["rel_obj"] <= REL_OBJ for r in rp)}
        log(f"{path}: {ms_p:.3f} ms/step, NMF {nm:.3f} ms, {rp[-1]['iters']} MU + {rp[-1]['polish_done']} ANLS, "
            f"rel obj {rp[-1]['rel_obj']:.3e}")

    # Roofline of each profiled kernel kind over the timed region: algorithmic
    # bytes (or flops) per launch / average launch time.
    rounds = sum(r["polish_done"] for r in recs_prof)
    elems = float(n_p) * n_k
    vb = 4.0 * n_p * K
    taps = 2.0 * float(np.mean([max(abs(math.cos(v * math.pi / sc.n_views)), abs(math.sin(v * math.pi / sc.n_views)))
                                for v in range(sc.n_views)]))
    triples = float(sc.n_views) * sc.n_rows * sc.n_cols * sc.n_cols * K
    mlp_flops_row = 2.0 * (256 * 128 + 128 * 128 + 128 * 16)
    work = {  # kind -> (name, total algorithmic units over the timed region, bound, unit)
        hsn.KERN_NORMALIZE: ("normalize_u16_kernel (u16 counts -> f32 p + pooled network input)",
                             args.steps * (6.0 * elems + 2.0 * sc.n_rows * sc.n_cols * n_k +
                                           (512.0 if mlp.precision == hsn.PREC_BF16 else 1024.0) * n_p), "hbm"),
        hsn.KERN_NMF_PASS: ("pass_f32_kernel (N_V / N_D passes over f32 p)",
                            args.steps * (4.0 * elems + vb) + rounds * 2 * (4.0 * elems + vb), "hbm"),
        hsn.KERN_MLP_POOL: ("pool_kernel (bf16 p -> 256-bin pooled rows)",
                            args.steps * (2.0 * elems + 512.0 * n_p), "hbm"),
        hsn.KERN_MLP_ROWS: ("mlp_infer2_kernel (network inference, bf16 MFMA)",
                            args.steps * mlp_flops_row * n_p, "mfma"),
        hsn.KERN_PROJECT: ("project_lds_kernel (A, Joseph footprint, K channels, LDS-staged)", None, "alu"),
        hsn.KERN_BACKPROJECT: ("backproject_lds_kernel (A^T, LDS-staged)", None, "alu"),
    }
    # Float32 passes that did work: one N_D pass for D0 per step and two passes
    # per ANLS round; passes queued after the stop test fired return at once,
    # their time stays in the total (so the rate is conservative).
    real = {hsn.KERN_NMF_PASS: args.steps + 2 * rounds}
    roof = {}
    for kk, (name, units, bound) in work.items():
        ms, n = prof.get(kk, (0.0, 0))
        if n == 0:
            continue
        queued = n
        n = real.get(kk, n)
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
    traffic = load_traffic() if args.workload == "mid" else {}
    for name, r in roof.items():
        r["traffic"] = traffic.get(name.split(" ")[0])
    # The comparison paths' streaming passes (their bulk is the largest HBM
    # stream of the method): MU pass = p once + V read and written; each ANLS
    # round = two passes of p once + V (or N_V) once.
    for path, (pp, rp) in compare_prof.items():
        it_ = sum(r["iters"] for r in rp)
        rd_ = sum(r["polish_done"] for r in rp)
        bf = path == "cold_bf16"
        kinds = [(hsn.KERN_NMF_PASS_BF16, it_ * (2.0 * elems + 2 * vb), it_)] if bf else []
        kinds.append((hsn.KERN_NMF_PASS, (0 if bf else it_ * (4.0 * elems + 2 * vb)) + rd_ * 2 * (4.0 * elems + vb),
                      (0 if bf else it_) + 2 * rd_))
        ent = {}
        for kk, by, nl in kinds:
            ms, nq = pp.get(kk, (0.0, 0))
            if nl and ms > 0:
                ach = by / (ms * 1e-3) / 1e9
                ent["bf16 MU pass" if kk == hsn.KERN_NMF_PASS_BF16 else "f32 passes"] = {
                    "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "avg_launch_ms": ms / nl, "launches": nl, "queued": nq}
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
                   "nmf": f"learned start (bf16 MFMA network, {n_train} training spectra) + ANLS polish until "
                          f"rel obj {REL_OBJ:g}",
                   "recon": f"CGLS {CGLS_ITERS} pairs", "parallelism": "single GPU"},
        "nmf": {"vpb_per_s": vpb / (nmf_ms * 1e-3), "ms": nmf_ms, "anls_rounds": recs[-1]["polish_done"],
                "rel_obj": recs[-1]["rel_obj"], "reached": reached, "f_star": f_star, "references": refs},
        "compare": compare,
        "speedup_vs_plain_fp32": {"nmf": compare["plain_fp32"]["nmf_ms"] / nmf_ms,
                                  "step": compare["plain_fp32"]["ms_per_step"] / ms_step},
        "fmd_tail": fmd,
        "fbp_comparison": fbp_cmp,
        "network": {"train_spectra": n_train, "epochs": args.mlp_epochs, "train_s": t_train,
                    "loss_first": loss_hist[0], "loss_last": loss_hist[-1]},
        "projector": {"voxel_rays_per_s_A": triples / (prj["avg_launch_ms"] * 1e-3) if prj else None,
                      "voxel_rays_per_s_AT": triples / (bpj["avg_launch_ms"] * 1e-3) if bpj else None,
                      "ms_A": prj["avg_launch_ms"] if prj else None, "ms_AT": bpj["avg_launch_ms"] if bpj else None},
        "roofline": {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                     "unit": d["unit"], "frac": d["frac"], "traffic": d["traffic"],
                     "avg_launch_ms": d["avg_launch_ms"], "launches": d["launches"],
                     "alg_per_launch": d["alg_per_launch"], "all_kernels": roof},
    }
    if not args.no_cpu_baseline and not full:
        out["cpu_baseline"] = cpu_baseline(sc, compare["plain_fp32"]["mu_iters"],
                                           compare["plain_fp32"]["anls_rounds"])
    print(json.dumps(out), flush=True)


def load_traffic():
    """kernel -> HBM bytes per launch (mid workload) from profiles/pmc_traffic_mid.json
    (rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the copy probe), for kernels
    whose source file still hashes to the value recorded with the counters."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_mid.json")
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


def run_batched(args):
    """32 uneven decompositions (views 30-180, columns 64-256, bins 512-2048,
    K 2-6, one slice each): float32 MU bulk (200 iterations) then ANLS rounds
    until each instance's relative objective reaches 1e-4, from seeded random
    starts.  Timed: 32 per-instance calls one after the other, and the batched
    call (one launch per phase) without graphs, with graphs, and with graphs
    and the autotuned partition."""
    import torch
    import synth
    from paper_2410_22500_amd import hsn

    t0 = time.time()
    scans = synth.batched_scans(32, 3)
    insts = []
    for i, sc in enumerate(scans):
        y = torch.from_numpy(sc.y.view(np.int16)).cuda()
        yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
        p, _, _, _ = hsn.hsn_normalize(y, yo)
        V0, D0 = synth.random_factors(sc.n_p, sc.n_bins, sc.n_mat, 500 + i)
        insts.append(dict(p=p, n_k=sc.n_bins, V0=torch.from_numpy(V0.astype(np.float32)).cuda(),
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

    def per_instance():
        out = []
        for x, f in zip(insts, f_ref):
            out.append(hsn.hsn_subspace_nmf(x["p"], None, x["n_k"], x["V"], x["D"], polish_algo=hsn.ALGO_ANLS,
                                            f_ref=f, **kw))
        return out

    def batched(flags):
        return hsn.hsn_subspace_nmf_batched([(x["p"], x["n_k"], x["V"], x["D"], f) for x, f in zip(insts, f_ref)],
                                            flags=flags, **kw)

    runs = {"per_instance": per_instance, "batched": lambda: batched(0),
            "batched_graph": lambda: batched(hsn.BATCH_GRAPH),
            "batched_graph_autotuned": lambda: batched(hsn.BATCH_GRAPH | hsn.BATCH_AUTOTUNE)}
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
    best = res["batched_graph_autotuned"]
    out = {
        "metric": "view*pixel*bins decomposed/s at rel obj 1e-4 (32 uneven decompositions)",
        "value": best["vpb_per_s"], "unit": "vpb/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded phantoms, Bragg-edge-like spectra, Poisson counts)",
        "config": {"workload": "batched: 32 instances, views 30-180, columns 64-256, bins 512-2048, K 2-6, "
                               "one slice each, flux 1e4", "nmf": f"f32 MU {BULK} + ANLS until rel obj {REL_OBJ:g}",
                   "parallelism": "single GPU"},
        "runs": res,
        "speedup_vs_per_instance": res["per_instance"]["ms"] / best["ms"],
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(sc, mu_iters, polish_rounds):
    """The FP64 oracle as it stands, on a bounded sample of the same workload:
    detector row 0 (1 of N_r slices), running the plain method (NNDSVDa, MU,
    ANLS) with the iteration counts the plain FP32 GPU path needed.
    Normalisation, NNDSVDa, CGLS and the expansion run in full on that slice;
    the NMF iterations are timed on the first quarter of the slice's rays (10
    MU iterations, 1 ANLS round) and extrapolated linearly in rows and per
    iteration.  Rate in vpb/s of the slice."""
    from threadpoolctl import threadpool_info
    from oracle import cgls as ocgls
    from oracle import expand as oexp
    from oracle import nmf as onmf
    from oracle.normalize import normalize as onorm

    K = sc.n_mat
    ysub = sc.y[:, :1]
    yosub = sc.yo[:1]
    t0 = time.perf_counter()
    p, _, _ = onorm(ysub, yosub)
    t_norm = time.perf_counter() - t0
    t0 = time.perf_counter()
    V, D = onmf.nndsvd(p, K, variant="a")
    t_init = time.perf_counter() - t0
    q = max(1, p.shape[0] // 4)
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
    t = t_norm + t_init + t_mu * mu_iters + t_an * polish_rounds + t_rec
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    vpb = p.shape[0] * p.shape[1]
    return {"value": vpb / t, "unit": "vpb/s", "cores": threads, "kind": "oracle",
            "sample": f"detector row 0 of {sc.n_rows} ({p.shape[0]} x {p.shape[1]}): normalise, NNDSVDa, "
                      f"CGLS {CGLS_ITERS}, expansion in full; NMF iterations timed on {q} rays ({n_mu} MU, "
                      f"1 ANLS) and extrapolated to {mu_iters} MU + {polish_rounds} ANLS on the slice; "
                      f"{t:.1f}s total (estimate) on {os.cpu_count()} host cpus "
                      f"({platform.processor() or platform.machine()})",
            "seconds": t}


if __name__ == "__main__":
    main()
