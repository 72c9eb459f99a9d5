"""Write the stored expected values for the full-size parity tests.

Calls only the CPU oracle (and the seeded input generator). For each case it
runs the oracle's exact-SVT inexact ALM (the plain form: a full one-sided
Jacobi SVD per iteration) and stores what a GPU run at the same size can be
checked against without rerunning the oracle: seeded sampled entries of A and
E, the singular values of A, norms, the nonzero count of E, the iteration
count and rank.

    python tests/golden/make_golden.py rpca_n2000_s0
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    # config: RPCA(2000, 2000, rank 100, 10% corruption U[-500, 500]), lambda = 1/sqrt(2000)
    "rpca_n2000_s0": dict(m=2000, n=2000, r=100, frac=0.10, amp=500.0, seed=0, tol=1e-7),
    # smaller case in the same regime (Table 1, m = 500 row shape)
    "rpca_n500_s0": dict(m=500, n=500, r=50, frac=0.10, amp=500.0, seed=0, tol=1e-7),
}

SAMPLES = 4096
SAMPLE_SEED = 12345


def make(name: str) -> dict:
    c = CASES[name]
    inst = synth.rpca_instance(c["m"], c["n"], c["r"], c["frac"], c["amp"], c["seed"])
    t0 = time.time()
    out = oracle.rpca(inst["D"], mode="exact", tol=c["tol"])
    secs = time.time() - t0
    A, E = out["A"], out["E"]
    pos = synth.sample_positions(c["m"], c["n"], SAMPLES, SAMPLE_SEED)
    _, sA, _ = oracle.jacobi_svd(A)
    info = out["info"]
    return {
        "case": name,
        "source": "oracle exact-SVT inexact ALM (one-sided Jacobi SVD per iteration)",
        "params": c,
        "iters": info["iters"],
        "rank": info["rank"],
        "nnz_E": info["nnz_E"],
        "rel_residual": info["rel_residual"],
        "norm2_D": info["norm2_D"],
        "norm_A": float(np.linalg.norm(A)),
        "norm_E": float(np.linalg.norm(E)),
        "sigma_A": [float(x) for x in sA[: c["r"] + 16]],
        "rel_err_vs_A0": float(np.linalg.norm(A - inst["A0"]) / np.linalg.norm(inst["A0"])),
        "sample_seed": SAMPLE_SEED,
        "sample_pos": [int(p) for p in pos],
        "A_samples": [float(x) for x in A.reshape(-1)[pos]],
        "E_samples": [float(x) for x in E.reshape(-1)[pos]],
        "svp_trace": [int(x) for x in out["svp"]],
        "oracle_seconds": secs,
    }


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        g = make(name)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json")
        with open(path, "w") as f:
            json.dump(g, f, indent=0)
        print(name, "iters", g["iters"], "rank", g["rank"], "secs", round(g["oracle_seconds"], 1))
