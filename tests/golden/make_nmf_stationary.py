"""Writes nmf_tiny_stationary.json: the stationary objective f* that the
MU + ANLS-polish GPU test must reach within rel obj 1e-4, computed by the
float64 oracle alone (oracle.nmf.stationary_reference: ANLS rounds, then the
projected quasi-Newton refinement, then ANLS rounds; about 15 minutes on one
core, too slow to repeat inside a GPU test).  The KKT residuals of the
returned point are stored beside f* and must be <= 1e-9.

Input: p of the tiny synthetic scan (oracle normalisation), the start
synth.random_factors(5760, 256, 3, seed 10) rounded to float32.
Run from the repository root:  python tests/golden/make_nmf_stationary.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import nmf as onmf  # noqa: E402
from oracle.normalize import normalize as onorm  # noqa: E402


def main():
    sc = synth.config_scan("tiny")
    p, _, _ = onorm(sc.y, sc.yo)
    p = np.asarray(p, np.float32).astype(np.float64)
    V0, D0 = synth.random_factors(p.shape[0], p.shape[1], 3, 10)
    V0 = np.asarray(V0, np.float32).astype(np.float64)
    D0 = np.asarray(D0, np.float32).astype(np.float64)
    f_star, Vs, Ds = onmf.stationary_reference(p, V0, D0)
    kv, kd = onmf.kkt_residual(p, Vs, Ds)
    assert kv <= 1e-9 and kd <= 1e-9, (kv, kd)
    out = {"f_star": f_star, "workload": "tiny scan, K = 3, start synth.random_factors(..., 3, 10) in float32",
           "how": "oracle.nmf.stationary_reference (ANLS to relative change 1e-12, L-BFGS-B refinement, ANLS)",
           "kkt_residual": [kv, kd]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "nmf_tiny_stationary.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, f_star)


if __name__ == "__main__":
    main()
