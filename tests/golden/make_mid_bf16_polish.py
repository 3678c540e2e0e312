"""Writes mid_bf16_polish.json: the float64 oracle's run of the mid
workload's BF16 schedule, against which the GPU's bfloat16 MFMA bulk plus
float32 polish is checked (1e-2 relative on the canonical coefficients).

Schedule (all float64, oracle only): p = the oracle's normalisation of the
mid scan (16 slices of 128^2, 60 views, 1024 bins, 4 materials, flux 2e3),
rounded to float32; the start synth.random_factors(122880, 1024, 4, seed 52)
rounded to float32; 100 multiplicative-update iterations on the
bfloat16-rounded p (round to nearest even), then 15 ANLS rounds on p.
Stored: the canonical D (unit columns matched to the material library), the
canonical V on every 240th row, and the final objective f(V, D) on p.
About 15 minutes on the host.  Run from the repository root:
    python tests/golden/make_mid_bf16_polish.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import nmf as onmf  # noqa: E402
from oracle.metrics import canonical  # noqa: E402
from oracle.normalize import normalize as onorm  # noqa: E402

ROW_STEP = 240
SEED = 52


def bf16_round(a32):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a32, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def main():
    sc = synth.config_scan("mid")
    p, _, _ = onorm(sc.y, sc.yo)
    p32 = p.astype(np.float32)
    p64 = p32.astype(np.float64)
    pq = bf16_round(p32)
    n_p, n_k = p.shape
    V0, D0 = synth.random_factors(n_p, n_k, sc.n_mat, SEED)
    V = V0.astype(np.float32).astype(np.float64)
    D = D0.astype(np.float32).astype(np.float64)
    for it in range(100):
        V, D, _, _ = onmf.mu_step(pq, V, D)
        if (it + 1) % 20 == 0:
            print("mu", it + 1, flush=True)
    for r in range(15):
        V, D, _, f = onmf.anls_round(p64, V, D)
        print("anls", r + 1, f, flush=True)
    f_end = onmf.objective(p64, V, D)
    Vc, Dc = canonical(V, D, library=sc.mu)
    out = {"workload": "mid scan (config_scan('mid')), K = 4",
           "schedule": "start synth.random_factors(n_p, n_k, 4, 52) in float32; 100 MU on the bf16-rounded p; "
                       "15 ANLS rounds on the float32 p (float64 arithmetic)",
           "how": "tests/golden/make_mid_bf16_polish.py (oracle only)",
           "row_step": ROW_STEP, "f_end": f_end,
           "D_canonical": np.round(Dc, 10).tolist(),
           "V_canonical_rows": np.round(Vc[::ROW_STEP], 10).tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mid_bf16_polish.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, f_end)


if __name__ == "__main__":
    main()
