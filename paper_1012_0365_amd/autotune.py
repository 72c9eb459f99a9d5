"""Autotuner for the split-K plans of the W-product GEMMs.

For every precision (FP64, FP32, BF16), product size s (W is s x s) and block
width N of a grid, time W X and W^T X under each candidate workgroup target
and keep the fastest (sum of both). The result is written as the C table
compiled into the library (csrc/tuned_plans.inc); rebuild afterwards. Run on
the GPU the library is for:

    python -m paper_1012_0365_amd.autotune [--out PATH] [--quick]
"""

from __future__ import annotations

import argparse
import os
import sys

SIZES = [500, 1000, 2000, 3000, 4000, 5000]
WIDTHS = [16, 48, 112, 208, 256, 400]
TARGETS = [128, 192, 256, 384, 512, 768, 1024]
PRECS = [(0, "FP64"), (1, "FP32"), (2, "BF16")]


def time_product(ctx, prec, W, X, C, trans, reps):
    if prec == 0:
        f = lambda: ctx.gemm_f64(W, X, C, trans_a=trans)  # noqa: E731
    else:
        f = lambda: ctx.gemm_lp(W, X, C, trans_a=trans)  # noqa: E731
    f()
    ctx.timing(True)
    for _ in range(reps):
        f()
    rec = ctx.timing_get("gemm_diag")
    ctx.timing(False)
    return rec["ms"] / rec["launches"] * 1e3


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--out", default=os.path.join(here, "csrc", "tuned_plans.inc"))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="a small grid (smoke run)")
    a = ap.parse_args(argv)
    import torch

    import paper_1012_0365_amd as blws
    from paper_1012_0365_amd import _native

    lib = _native.lib()
    sizes, widths = (SIZES[:2], WIDTHS[:2]) if a.quick else (SIZES, WIDTHS)
    ctx = blws.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(0)
    rows = []
    try:
        for prec, pname in PRECS:
            for s in sizes:
                W64 = torch.randn(s, s, dtype=torch.float64, device="cuda", generator=gen)
                W = W64 if prec == 0 else W64.float()
                if prec == 2:  # BF16 bits (truncated: the timing does not depend on them)
                    W = (W.view(torch.int32) >> 16).to(torch.int16)
                dt = torch.float64 if prec == 0 else torch.float32
                for n in widths:
                    X = torch.randn(s, n, dtype=dt, device="cuda", generator=gen)
                    C = torch.empty(s, n, dtype=dt, device="cuda")
                    best = None
                    for t in TARGETS:
                        if lib.blws_set_plan_target(t) != 0:
                            raise RuntimeError("blws_set_plan_target failed")
                        us = sum(time_product(ctx, prec, W, X, C, tr, a.reps) for tr in (False, True))
                        if best is None or us < best[1]:
                            best = (t, us)
                    rows.append((prec, s, n, best[0], best[1]))
                    print(f"{pname} size {s} N {n}: target {best[0]} ({best[1] / 2:.1f} us per product)",
                          flush=True)
                del W, W64
                torch.cuda.empty_cache()
    finally:
        lib.blws_set_plan_target(0)
        ctx.close()
    with open(a.out, "w") as f:
        f.write("// Written by autotune.py: precision (0 FP64, 1 FP32, 2 BF16), product size\n"
                "// sqrt(M K), block width N, workgroup target of the fastest split-K plan\n"
                f"// (candidates {', '.join(map(str, TARGETS))}; time per product in us).\n")
        for prec, s, n, t, us in rows:
            f.write(f"{{{prec}, {s}, {n}, {t}}},  // {us / 2:.1f}\n")
    print(f"wrote {a.out} ({len(rows)} entries)", file=sys.stderr)


if __name__ == "__main__":
    main()
