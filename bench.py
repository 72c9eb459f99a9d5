"""Benchmark: inexact-ALM robust PCA with BLWS singular value thresholding on
one MI355X, at the n = 2000 configuration (D = L R^T + E0, L, R 2000 x 100
N(0, 1), 10% of entries corrupted with U[-500, 500], lambda = 1/sqrt(2000),
stop at ||D - A - E||_F / ||D||_F < 1e-7).

A step is one full solve (all ALM iterations, each one BLWS SVT step plus the
fused epilogue), with D resident in HBM. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec f64|f32|bf16] [--no-cpu] [--no-plain]
    python bench.py --workload serving [--requests R]   # the request-server mix
    python bench.py --workload rpca4000   # n = 4000 FP64 solve, epilogue bytes and rate
    python bench.py --workload mc5000     # MC n = 5000 FP32 solve, sparse kernels' rates

The roofline entry is for the kernel family with the largest total time in
the timed region, from HIP events recorded around each launch on the stream
it runs on; `kernels` lists every family.
"""

from __future__ import annotations

import argparse
import json
import re
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20  # counter calibration copy
METRIC = "RPCA solve s & SVT calls/s at n=2000 vs plain (≤1e-6 rel err); p50/p99 lat"
M = N = 2000
RANK = 100
FRAC = 0.10
AMP = 500.0
SEED = 0

# Table 1, BLWS-ADM rows (two quad-core Xeon E5540, MATLAB): relative error of A,
# rank, iterations, seconds; context beside the rpca_table1 leg, not a target
PAPER_TABLE1 = {
    500: {"rel_err": 9.64e-6, "rank": 50, "iters": 30, "time_s": 2.07},
    1000: {"rel_err": 6.05e-6, "rank": 100, "iters": 30, "time_s": 9.25},
    2000: {"rel_err": 4.30e-6, "rank": 200, "iters": 30, "time_s": 53.37},
    3000: {"rel_err": 3.90e-6, "rank": 300, "iters": 30, "time_s": 149.19},
}

# Table 2, BLWS-SVT columns (same machine): seconds, iterations, relative error
PAPER_TABLE2 = {
    (5000, 10): {"time_s": 20.02, "iters": 123, "rel_err": 1.74e-4},
    (5000, 50): {"time_s": 279.08, "iters": 108, "rel_err": 1.55e-4},
    (5000, 100): {"time_s": 1175.91, "iters": 122, "rel_err": 1.74e-4},
    (10000, 10): {"time_s": 42.80, "iters": 123, "rel_err": 1.70e-4},
    (10000, 50): {"time_s": 736.01, "iters": 110, "rel_err": 1.60e-4},
    (20000, 10): {"time_s": 101.47, "iters": 124, "rel_err": 1.68e-4},
    (30000, 10): {"time_s": 171.40, "iters": 125, "rel_err": 1.69e-4},
}

# MI355X published peaks
PEAK = {
    "hbm": 8000.0,        # GB/s
    "mfma_f64": 78.6,     # TFLOP/s dense
    "mfma_f32": 157.3,
    "mfma_bf16": 2500.0,
    "valu_f64": 78.6,
}

# kernel family -> (bound, peak key or None for "by precision", unit)
FAMILY_BOUND = {
    "gemm_w": ("mfma", None, "TFLOP/s"),
    "gemm_ts": ("mfma", "mfma_f64", "TFLOP/s"),
    "gemm_lr": ("mfma", "mfma_f64", "TFLOP/s"),
    "alm_epilogue": ("hbm", "hbm", "GB/s"),
    "svt_reconstruct": ("hbm", "hbm", "GB/s"),
    "spmm": ("hbm", "hbm", "GB/s"),
    "mc_update": ("hbm", "hbm", "GB/s"),
}
COMPOSITE = {"small_svd"}  # timed around several other families
# families whose launches are several different kernels (a split-K product and
# its reduction, of several shapes): listed, but not a "dominant kernel"
MULTI_KERNEL = {"gemm_ts"}


def family_bound(name, prec):
    if name in FAMILY_BOUND:
        bound, key, unit = FAMILY_BOUND[name]
    else:  # one-workgroup / latency-bound FP64 kernels: vector ALU
        bound, key, unit = "alu", "valu_f64", "TFLOP/s"
    if key is None:
        key = {"f64": "mfma_f64", "f32": "mfma_f32", "bf16": "mfma_bf16"}[prec]
    return bound, key, unit


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["f64", "f32", "bf16"], default="f64")
    ap.add_argument("--workload", choices=["rpca", "serving", "copy", "rpca4000", "mc5000"],
                    default="rpca",
                    help="copy: one device copy of 256 MiB (counter calibration)")
    ap.add_argument("--requests", type=int, default=64, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=8, help="serving: solves in flight")
    ap.add_argument("--group-window", type=int, default=200,
                    help="serving: microseconds a ready solve waits for others to group with")
    ap.add_argument("--no-group", action="store_true",
                    help="serving: one launch per W-product instead of grouped launches")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the full-SVD comparator")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU baseline: repeat oracle solves until this much time has passed")
    ap.add_argument("--no-legs", action="store_true",
                    help="rpca: skip the extra measurements (FP32 / BF16 solves, the SVT "
                         "snapshot, n = 4000, matrix completion, the serving mix)")
    ap.add_argument("--leg-requests", type=int, default=24,
                    help="rpca legs: requests in the serving-mix leg")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(family):
    """HBM bytes per launch of a kernel family from the committed rocprofv3 PMC
    summaries (profiles/*_traffic.md, FETCH_SIZE and WRITE_SIZE scaled by a
    copy of known size), or None when there is none or the kernel's source has
    changed since the counters were taken."""
    import glob
    import hashlib

    here = os.path.dirname(os.path.abspath(__file__))
    pat = re.compile(r"^traffic: kernel=(\S+) bytes_per_launch=(\d+) source=(\S+) sha256=(\w+)")
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*_traffic.md"))):
        for line in open(path):
            m = pat.match(line.strip())
            if not m or m.group(1) != family:
                continue
            src = os.path.join(here, m.group(3))
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(4):
                return None
            return int(m.group(2))
    return None


def roofline_entry(name, rec, prec):
    bound, key, unit = family_bound(name, prec)
    n = max(1, rec["launches"])
    avg_s = rec["ms"] / n / 1e3
    if bound == "hbm":
        achieved = rec["bytes"] / n / avg_s / 1e9 if avg_s > 0 else 0.0
    else:
        achieved = rec["flops"] / n / avg_s / 1e12 if avg_s > 0 else 0.0
    peak = PEAK[key]
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": measured_traffic(name), "avg_us": avg_s * 1e6,
            "algorithmic_per_launch": (rec["bytes"] if bound == "hbm" else rec["flops"]) / n}


def pct(vals, p):
    v = sorted(vals)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(math.ceil(p / 100.0 * len(v))) - 1))
    return v[i]


def bench_rpca(args):
    import numpy as np
    import torch

    import paper_1012_0365_amd as blws
    import synth

    dt = torch.float64 if args.prec == "f64" else torch.float32
    bf16 = args.prec == "bf16"
    t0 = time.time()
    inst = synth.rpca_instance(M, N, RANK, FRAC, AMP, SEED)
    log(f"[bench] data generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    D = torch.tensor(inst["D"], dtype=dt, device=dev)
    A0 = torch.tensor(inst["A0"], dtype=torch.float64, device=dev)
    A = torch.empty_like(D)
    E = torch.empty_like(D)
    ctx = blws.Context(0)

    for i in range(args.warmup):
        _, _, info = ctx.rpca_solve(D, A=A, E=E, bf16=bf16)
        log(f"[bench] warmup {i}: {info['iters']} iters, {info['seconds']:.3f}s")
    torch.cuda.synchronize()

    # Per-family breakdown: one more solve with every launch timed (two event
    # records per launch), before and outside the timed region.
    ctx.timing(True)
    ctx.rpca_solve(D, A=A, E=E, bf16=bf16)
    torch.cuda.synchronize()
    fams = {}
    for name in ctx.timing_families():
        rec = ctx.timing_get(name)
        if rec["launches"]:
            fams[name] = rec
    ctx.timing(False)
    leaves = {k: v for k, v in fams.items() if k not in COMPOSITE}
    kernel_ms = sum(r["ms"] for r in leaves.values())
    single = {k: v for k, v in leaves.items() if k not in MULTI_KERNEL}
    dominant = max(single, key=lambda k: single[k]["ms"])
    kernels = {}
    for name, rec in sorted(fams.items(), key=lambda kv: -kv[1]["ms"]):
        e = roofline_entry(name, rec, args.prec)
        kernels[name] = {"ms_per_step": rec["ms"],
                         "share": (rec["ms"] / kernel_ms if kernel_ms and name not in COMPOSITE
                                   else None),
                         "launches_per_step": rec["launches"],
                         "avg_us": e["avg_us"], "achieved": e["achieved"], "unit": e["unit"],
                         "frac": e["frac"], "bound": e["bound"],
                         "composite": name in COMPOSITE}

    # Timed region: only the dominant family's launches carry HIP events.
    ctx.timing(True, only=[dominant])
    lat, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        _, _, info = ctx.rpca_solve(D, A=A, E=E, bf16=bf16)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
        iters.append(info["iters"])
        log(f"[bench] step {k}: {info['iters']} iters, {lat[-1]:.3f}s, rank {info['rank']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    dom = ctx.timing_get(dominant)
    ctx.timing(False)
    roof = roofline_entry(dominant, dom, args.prec)
    roof["kernel"] = dominant
    roof["launches_per_step"] = dom["launches"] / args.steps

    # accuracy of the last solve
    Ad = A.double()
    rel_A0 = float(torch.linalg.norm(Ad - A0) / torch.linalg.norm(A0))
    rel_oracle = None
    gpath = os.path.join(ROOT, "tests", "golden", "rpca_n2000_s0.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            g = json.load(f)
        pos = torch.tensor(g["sample_pos"], device=dev)
        As = Ad.reshape(-1)[pos].cpu().numpy()
        ref = np.array(g["A_samples"])
        rel_oracle = float(np.linalg.norm(As - ref) / np.linalg.norm(ref))

    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "rpca_inexact_alm_blws_n2000", "m": M, "n": N, "rank": RANK,
                   "corruption": FRAC, "corruption_amp": AMP, "lambda": 1.0 / math.sqrt(N),
                   "tol": 1e-7, "seed": SEED, "precision": args.prec},
        "solve_s_p50": pct(lat, 50),
        "solve_s_p99": pct(lat, 99),
        "iters": iters[-1],
        "iters_bf16": info.get("iters_bf16"),
        "svt_calls_per_s": sum(iters) / total,
        "rel_err_vs_A0": rel_A0,
        "rel_err_vs_oracle_samples": rel_oracle,
        "kernel_ms_per_step": kernel_ms,
        "roofline": roof,
        "kernels": kernels,
        "kernels_from": "one extra solve before the timed region, every launch timed",
    }

    if not args.no_legs:
        out["legs"] = rpca_legs(args, ctx, D if args.prec == "f64" else D.double(),
                                total / args.steps, A0)

    if not args.no_plain:
        # Plain comparator: the same ALM with a full SVD per iteration on the same
        # GPU (torch.linalg.svd). Bounded sample: the best of two full SVDs of a
        # 2000 x 2000 matrix of the solve's type, times the iteration count.
        W = D.clone()
        torch.linalg.svd(W, full_matrices=False)
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            t1 = time.perf_counter()
            torch.linalg.svd(W, full_matrices=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        plain = min(ts) * iters[-1]
        out["plain_gpu_solve_s_est"] = plain
        out["plain_sample"] = (f"torch.linalg.svd of one {M}x{N} {dt} matrix, best of 2, "
                               f"x {iters[-1]} iterations")
        out["speedup_vs_plain"] = plain / (total / args.steps)

    if not args.no_cpu:
        import oracle

        oracle.build(force=False)
        cores = len(os.sched_getaffinity(0))
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        t1 = time.perf_counter()
        n_solves, n_it = 0, 0
        while True:
            res = oracle.rpca(inst["D"], mode="blws")
            n_solves += 1
            n_it = res["info"]["iters"]
            if time.perf_counter() - t1 >= args.cpu_seconds:
                break
        tc = time.perf_counter() - t1
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        cpu_model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        out["cpu_baseline"] = {
            "value": n_solves / tc, "unit": "solves/s", "cores": min(threads, cores),
            "kind": "oracle", "cpu": cpu_model,
            "sample": (f"oracle BLWS inexact ALM (FP64 plain loops, OpenMP), {n_solves} full "
                       f"n=2000 solve(s) of {n_it} iterations in {tc:.1f}s"),
        }
    return out


def golden_error(name, A, E=None, planted=False):
    """Sampled relative error of A (and E) against the stored oracle values."""
    import numpy as np
    import torch

    with open(os.path.join(ROOT, "tests", "golden", name + ".json")) as f:
        g = json.load(f)
    pos = torch.tensor(g["sample_pos"], device=A.device)
    As = A.double().reshape(-1)[pos].cpu().numpy()
    ref = np.array(g["A_samples"])
    out = {"A": float(np.linalg.norm(As - ref) / np.linalg.norm(ref))}
    if E is not None:
        Es = E.double().reshape(-1)[pos].cpu().numpy()
        refe = np.array(g["E_samples"])
        out["E"] = float(np.linalg.norm(Es - refe) / np.linalg.norm(refe))
    return out, g


def timed_solves(ctx, D, reps, **kw):
    import torch

    ts, info = [], None
    A = torch.empty_like(D)
    E = torch.empty_like(D)
    for _ in range(reps):
        t1 = time.perf_counter()
        _, _, info = ctx.rpca_solve(D, A=A, E=E, **kw)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    return sorted(ts)[len(ts) // 2], info, A, E


def snapshot_state(ctx, D):
    """The state of the n = 2000 solve at iteration 15: 14 ALM iterations
    driven from here (blws_svt plus the elementwise updates in torch, outside
    any timed region) give W and eps of iteration 15 and the warm block (U, V)
    of width b that iteration 14's step returned."""
    import torch

    m, n = D.shape
    lam = 1.0 / math.sqrt(max(m, n))
    s1 = float(torch.linalg.matrix_norm(D, 2))
    J = max(s1, float(D.abs().max()) / lam)
    Y = D / J
    E = torch.zeros_like(D)
    mu, rho = 1.25 / s1, 1.5
    sv, b = 10, 0
    U = V = None
    for it in range(1, 15):
        W = D - E + Y / mu
        bn = min(((sv + 15) // 16) * 16, min(m, n) // 2)
        cold = b == 0 or bn != b
        if cold:
            # a cold block of the new width (this state is for the steady
            # state, not the block-resize rule)
            U = torch.empty(m, bn, dtype=D.dtype, device=D.device)
            V = torch.empty(n, bn, dtype=D.dtype, device=D.device)
        b = bn
        A = torch.empty_like(D)
        S, rank = ctx.svt(W, 1.0 / mu, U, V, warm=not cold, A=A)
        svp = int(rank.item())
        sv = svp + 1 if svp < sv else min(svp + round(0.05 * min(m, n)), min(m, n))
        T = D - A + Y / mu
        E = torch.sign(T) * torch.clamp(T.abs() - lam / mu, min=0.0)
        Y = Y + mu * (D - A - E)
        mu = min(rho * mu, 1.25e7 / s1)
    W = (D - E + Y / mu).contiguous()
    eps = 1.0 / mu
    bn = min(((sv + 15) // 16) * 16, min(m, n) // 2)
    A = torch.empty_like(W)
    if bn != b:
        U = torch.empty(m, bn, dtype=D.dtype, device=D.device)
        V = torch.empty(n, bn, dtype=D.dtype, device=D.device)
        ctx.svt(W, eps, U, V, warm=False, A=A)
    torch.cuda.synchronize()
    return W, eps, U, V


def svt_snapshot_leg(ctx, state):
    """SVT calls/s on the iteration-15 state of the n = 2000 solve (b = 112):
    five blws_svt calls on that W settle the warm block, then back-to-back
    calls, each fed the previous call's Ritz vectors as its warm block."""
    import torch

    W, eps, U0, V0 = state
    U, V = U0.clone(), V0.clone()
    m, n = W.shape
    b = U.shape[1]
    S = torch.empty(b, dtype=torch.float64, device=W.device)
    rank = torch.zeros(1, dtype=torch.int32, device=W.device)
    A = torch.empty_like(W)
    for _ in range(5):
        ctx.svt(W, eps, U, V, A=A, S=S, rank=rank)
    torch.cuda.synchronize()
    calls = 40
    t1 = time.perf_counter()
    for _ in range(calls):
        ctx.svt(W, eps, U, V, A=A, S=S, rank=rank)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    r = int(rank.item())
    flops = 6.0 * m * n * b + 2.0 * m * n * r
    return {"calls_per_s": calls / el, "us_per_call": 1e6 * el / calls, "b": b, "rank": r,
            "gflop_per_s": flops * calls / el / 1e9,
            "flops_per_call": flops, "note": "W and the warm block of iteration 15"}


ABLATIONS = [("split", 2), ("aug", 2), ("left", 2), ("right", 2), ("aug", 3), ("split", 3)]


def ablation_leg(ctx, state, D, A0):
    """The Sec. 4.1 start-block ablations at n = 2000 (blws_svt_lanczos).
    Per call, on the iteration-15 state and from its warm block: the error of
    the top Ritz values and of A = T_eps(W) against a full FP64 SVD of W
    (torch.linalg.svd, a measurement reference only), the rank, the W-products
    and the time per call. Then whole robust-PCA solves with every SVT taken
    this way: iterations, time and the error against the planted A0."""
    import torch

    import paper_1012_0365_amd as blws

    W, eps, U0, V0 = state
    b = U0.shape[1]
    Uf, sf, Vhf = torch.linalg.svd(W, full_matrices=False)
    r_ex = int((sf > eps).sum().item())
    A_ex = (Uf[:, :r_ex] * (sf[:r_ex] - eps)) @ Vhf[:r_ex]
    na = float(torch.linalg.norm(A_ex))
    out = {"config": ("W and eps of iteration 15 of the n = 2000 solve, warm block from "
                      "iteration 14's step"),
           "b": b, "exact_rank": r_ex, "per_call": {}, "solves": {}}
    A = torch.empty_like(W)

    def measure(name, call, products):
        U, V = U0.clone(), V0.clone()
        S, rank = call(U, V)
        torch.cuda.synchronize()
        r = int(rank.item())
        q = min(b, r_ex)
        serr = float(((S[:q] - sf[:q]).abs().max() / sf[0]).item())
        aerr = float(torch.linalg.norm(A - A_ex).item() / na)
        reps = 10
        t1 = time.perf_counter()
        for _ in range(reps):
            call(U, V)
        torch.cuda.synchronize()
        out["per_call"][name] = {"sigma_err_rel_s1": serr, "A_err_rel": aerr, "rank": r,
                                 "w_products": products,
                                 "ms_per_call": 1e3 * (time.perf_counter() - t1) / reps}

    measure("default_step", lambda U, V: ctx.svt(W, eps, U, V, A=A), 3)
    for start, k in ABLATIONS:
        measure(f"{start}_k{k}",
                lambda U, V, st=start, kk=k: ctx.svt_lanczos(W, eps, U, V, start=st, k=kk, A=A),
                2 * k - 1)
    na0 = float(torch.linalg.norm(A0))
    for start, k in [("aug", 2), ("split", 3), ("left", 2)]:
        opts = blws.default_alm_opts(svt_start=blws.STARTS[start], k_blocks=k)
        t, info, Ah, _ = timed_solves(ctx, D, 1, opts=opts)
        out["solves"][f"{start}_k{k}"] = {
            "solve_s": t, "iters": info["iters"], "status": info["status"], "rank": info["rank"],
            "rel_err_vs_A0": float(torch.linalg.norm(Ah - A0).item() / na0)}
    return out


def plain_alm_leg(D, iters_total, iters_timed=3):
    """The plain form on the same GPU: the same inexact ALM with the SVT from a
    full SVD (torch.linalg.svd), timed over its first iterations and scaled
    to the BLWS solve's iteration count."""
    import torch

    m, n = D.shape
    lam = 1.0 / math.sqrt(max(m, n))
    s1 = float(torch.linalg.matrix_norm(D, 2))
    J = max(s1, float(D.abs().max()) / lam)
    Y = D / J
    E = torch.zeros_like(D)
    mu = 1.25 / s1
    torch.linalg.svd(D[:64, :64])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(iters_timed):
        W = D - E + Y / mu
        Uf, Sf, Vh = torch.linalg.svd(W, full_matrices=False)
        Sf = torch.clamp(Sf - 1.0 / mu, min=0.0)
        A = (Uf * Sf) @ Vh
        T = D - A + Y / mu
        E = torch.sign(T) * torch.clamp(T.abs() - lam / mu, min=0.0)
        Y = Y + mu * (D - A - E)
        mu = 1.5 * mu
    torch.cuda.synchronize()
    per_it = (time.perf_counter() - t1) / iters_timed
    return {"solve_s_est": per_it * iters_total, "s_per_iteration": per_it,
            "sample": f"{iters_timed} ALM iterations with torch.linalg.svd ({D.dtype}), "
                      f"x {iters_total} iterations"}


def rpca_legs(args, ctx, D64, fp64_s, A0):
    """Extra measurements beside the headline FP64 line (each bounded)."""
    import torch

    import paper_1012_0365_amd as blws
    import synth

    legs = {}

    def leg(name, fn):
        t1 = time.time()
        try:
            legs[name] = fn()
        except Exception as e:  # a failed leg is reported, the headline line stands
            legs[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] leg {name}: {time.time() - t1:.1f}s")

    def low_prec():
        out = {}
        D32 = D64.float()
        for prec in ("f32", "bf16", "bf16_x3"):
            kw = {"bf16": prec != "f32"}
            if prec == "bf16_x3":  # BF16, then BF16 x 3 down to 1e-6, then FP32
                kw["opts"] = blws.default_alm_opts(ladder3_tol=1e-6)
            timed_solves(ctx, D32, 1, **kw)
            t, info, A, E = timed_solves(ctx, D32, 3, **kw)
            err, _ = golden_error("rpca_n2000_s0", A, E)
            out[prec] = {"solve_s": t, "solves_per_s": 1.0 / t, "iters": info["iters"],
                         "iters_bf16": info["iters_bf16"],
                         "iters_bf16x3": info["iters_bf16x3"], "status": info["status"],
                         "rel_err_vs_oracle_samples": err, "vs_f64_speed": fp64_s / t}
        return out

    def w_products():
        """W V at the benchmark shape (2000 x 2000 times 2000 x 112) in each
        product mode, 20 back-to-back launches each."""
        import numpy as np

        m, n = D64.shape
        b = 112
        X = torch.randn(n, b, dtype=torch.float64, device=D64.device)
        W32, X32 = D64.float(), X.float()
        hi = torch.empty(m, n, dtype=torch.int16, device=D64.device)
        lo = torch.empty_like(hi)
        # the split of W in torch: hi = bf16(W) (nearest even), lo = bf16(W - hi)
        hb = W32.to(torch.bfloat16)
        hi.copy_(hb.view(torch.int16))
        lo.copy_((W32 - hb.float()).to(torch.bfloat16).view(torch.int16))
        C64 = torch.empty(m, b, dtype=torch.float64, device=D64.device)
        C32 = torch.empty(m, b, dtype=torch.float32, device=D64.device)
        ref = D64 @ X
        modes = {
            "f64": (lambda: ctx.gemm_f64(D64, X, C64), 8.0, C64),
            "f32": (lambda: ctx.gemm_lp(W32, X32, C32), 4.0, C32),
            "bf16": (lambda: ctx.gemm_lp(hi, X32, C32), 2.0, C32),
            "bf16_x3": (lambda: ctx.gemm_bf16x3(hi, lo, X32, C32), 4.0, C32),
        }
        out = {"shape": "W (2000 x 2000) times X (2000 x 112)"}
        for name, (fn, wbytes, C) in modes.items():
            fn()
            torch.cuda.synchronize()
            err = float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref))
            reps = 20
            t1 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            us = 1e6 * (time.perf_counter() - t1) / reps
            out[name] = {"us": us, "rel_err": err,
                         "hbm_GB_per_s": wbytes * m * n / (us * 1e3),
                         "tflop_per_s": 2.0 * m * n * b / (us * 1e6)}
        return out

    leg("n2000_low_precision", low_prec)
    leg("w_products_n2000", w_products)
    state = snapshot_state(ctx, D64)
    leg("svt_snapshot_n2000_f64", lambda: svt_snapshot_leg(ctx, state))
    leg("ablations_sec41_n2000_f64", lambda: ablation_leg(ctx, state, D64, A0))
    del state

    def n4000():
        inst = synth.rpca_instance(4000, 4000, 200, 0.10, AMP, 0)
        out = {"config": "m = n = 4000, rank 200, 10% U[-500, 500], rho 1.2, tol 1e-7"}
        opts = blws.default_alm_opts(rho=1.2)
        for prec in ("f64", "f32", "bf16"):
            D = torch.tensor(inst["D"], dtype=torch.float64 if prec == "f64" else torch.float32,
                             device="cuda")
            timed_solves(ctx, D, 1, opts=opts, bf16=prec == "bf16")
            t, info, A, E = timed_solves(ctx, D, 1, opts=opts, bf16=prec == "bf16")
            err, g = golden_error("rpca_n4000_s0", A, E)
            sv = torch.linalg.svdvals(A.double())[:200].cpu()
            import numpy as np

            sref = np.array(g["sigma_A"][:200])
            out[prec] = {"solve_s": t, "iters": info["iters"], "rank": info["rank"],
                         "iters_bf16": info["iters_bf16"],
                         "rel_err_vs_oracle_samples": err,
                         "sigma_rel_err_top200": float(np.max(np.abs(sv.numpy() - sref) / sref))}
            del D, A, E
        return out

    leg("rpca_n4000", n4000)

    def table1():
        # the paper's RPCA experiment: m x m, rank 0.1 m, 10% of entries
        # corrupted with U[-500, 500], lambda = 1/sqrt(m), stopped at 1e-7
        out = {"config": "m x m, rank 0.1 m, 10% corrupted U[-500, 500], lambda = 1/sqrt(m), "
                         "tol 1e-7, FP64; rho 1.5 (and 1.2 where 1.5 leaves A0 unrecovered)"}
        for mm in (500, 1000, 2000, 3000):
            inst = synth.rpca_instance(mm, mm, mm // 10, 0.10, AMP, 0)
            D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
            A0 = torch.tensor(inst["A0"], dtype=torch.float64, device="cuda")
            row = {}
            for rho in (1.5, 1.2):
                opts = blws.default_alm_opts(rho=rho)
                timed_solves(ctx, D, 1, opts=opts)
                t, info, A, E = timed_solves(ctx, D, 1, opts=opts)
                err = float(torch.linalg.norm(A - A0) / torch.linalg.norm(A0))
                row[f"rho_{rho}"] = {"solve_s": t, "iters": info["iters"], "rank": info["rank"],
                                     "status": info["status"], "rel_err_vs_A0": err,
                                     "nnz_E": int((E != 0).sum())}
                del A, E
                if err < 1e-4:
                    break
            row["paper_blws_adm"] = PAPER_TABLE1[mm]
            out[str(mm)] = row
            del D, A0
        return out

    leg("rpca_table1", table1)

    def mc5000():
        import numpy as np

        inst = synth.mc_instance(5000, 5000, 50, 0.10, 0)
        rp = torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda")
        ci = torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda")
        vals = torch.tensor(inst["values"], dtype=torch.float32, device="cuda")
        opts = blws.default_mc_opts()
        ctx.mc_solve(5000, 5000, rp, ci, vals, opts=opts, r_cap=256)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        U, S, V, info = ctx.mc_solve(5000, 5000, rp, ci, vals, opts=opts, r_cap=256)
        torch.cuda.synchronize()
        t = time.perf_counter() - t1
        with open(os.path.join(ROOT, "tests", "golden", "mc_n5000_s0.json")) as f:
            g = json.load(f)
        pos = np.array(g["sample_pos"])
        rows = torch.tensor(pos // 5000, device="cuda")
        cols = torch.tensor(pos % 5000, device="cuda")
        a_s = ((U.double()[rows] * S) * V.double()[cols]).sum(1).cpu().numpy()
        ref = np.array(g["A_samples"])
        msm = np.array(g["M_samples"])
        return {"config": "m = n = 5000, rank 50, 10% sampled, FP32, rho 1.05, tol 1e-6",
                "solve_s": t, "iters": info["iters"], "rank": info["rank"],
                "rel_err_vs_oracle_samples": float(np.linalg.norm(a_s - ref) / np.linalg.norm(ref)),
                "rel_err_vs_planted_samples": float(np.linalg.norm(a_s - msm) / np.linalg.norm(msm))}

    leg("mc_n5000_f32", mc5000)

    def table2():
        """Table 2's r = 10 rows (m x m, s / d_r = 6): the SVT host with BLWS
        thresholding, FP64, error of the completed matrix vs the planted one
        from the factors (no dense product)."""
        out = {"config": "m x m, rank 10, s = 6 r (2 m - r) samples, tau = 5 m, "
                         "delta = 1.2 m^2 / s, tol 1e-4, FP64"}
        # m = 30000 (sampling ratio 0.004) over five seeds: there the SVT iteration
        # converges on some instances and oscillates on others
        for m, seed in [(5000, 0), (10000, 0), (20000, 0)] + [(30000, k) for k in range(5)]:
            s = 6 * 10 * (2 * m - 10)
            inst = synth.mc_instance(m, m, 10, s / float(m * m), seed)
            rp = torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda")
            ci = torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda")
            vals = torch.tensor(inst["values"], dtype=torch.float64, device="cuda")
            if m == 5000:
                ctx.mc_svt_solve(m, m, rp, ci, vals, r_cap=64)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            U, S, V, info = ctx.mc_svt_solve(m, m, rp, ci, vals, r_cap=64)
            torch.cuda.synchronize()
            t = time.perf_counter() - t1
            L = torch.tensor(inst["L"], device="cuda")
            R = torch.tensor(inst["R"], device="cuda")
            nM2 = float(((L.T @ L) * (R.T @ R)).sum())
            ip = float((((U * S).T @ L) * (V.T @ R)).sum())
            err = math.sqrt(max(float((S * S).sum()) + nM2 - 2.0 * ip, 0.0) / nM2)
            out[str(m) if m < 30000 else f"{m}_seed{seed}"] = {
                "nnz": s, "solve_s": t, "iters": info["iters"], "rank": info["rank"],
                "status": info["status"], "rel_err_vs_planted": err,
                "paper_blws_svt": PAPER_TABLE2.get((m, 10))}
        return out

    leg("mc_svt_table2_r10", table2)

    def table2_wide():
        """Table 2's r = 50 and r = 100 rows (s / d_r = 5 and 4), the same host
        and error measure as the r = 10 rows."""
        out = {"config": "m x m, rank r, s = c r (2 m - r) samples (c = 5 for r = 50, 4 for "
                         "r = 100), tau = 5 m, delta = 1.2 m^2 / s, tol 1e-4, FP64"}
        for m, r, c in [(5000, 50, 5), (5000, 100, 4), (10000, 50, 5)]:
            s = c * r * (2 * m - r)
            inst = synth.mc_instance(m, m, r, s / float(m * m), 0)
            rp = torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda")
            ci = torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda")
            vals = torch.tensor(inst["values"], dtype=torch.float64, device="cuda")
            cap = 2 * r + 64
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            U, S, V, info = ctx.mc_svt_solve(m, m, rp, ci, vals, r_cap=cap)
            torch.cuda.synchronize()
            t = time.perf_counter() - t1
            L = torch.tensor(inst["L"], device="cuda")
            R = torch.tensor(inst["R"], device="cuda")
            nM2 = float(((L.T @ L) * (R.T @ R)).sum())
            ip = float((((U * S).T @ L) * (V.T @ R)).sum())
            err = math.sqrt(max(float((S * S).sum()) + nM2 - 2.0 * ip, 0.0) / nM2)
            out[f"{m}_r{r}"] = {"nnz": s, "solve_s": t, "iters": info["iters"],
                                "rank": info["rank"], "status": info["status"],
                                "rel_err_vs_planted": err,
                                "paper_blws_svt": PAPER_TABLE2.get((m, r))}
            del rp, ci, vals, U, S, V, L, R
        return out

    leg("mc_svt_table2_r50_r100", table2_wide)
    if not args.no_plain:
        leg("plain_alm_n2000_f64", lambda: plain_alm_leg(D64, 23))

    def serving():
        sa = argparse.Namespace(requests=args.leg_requests, slots=8, group_window=200,
                                no_group=False, no_plain=False)
        r = bench_serving(sa)
        return {k: r[k] for k in ("value", "unit", "latency_s_p50", "latency_s_p99",
                                  "sequential_fp64_solves_per_s", "speedup_vs_sequential_fp64",
                                  "failed", "config")}

    leg("serving_mix", serving)
    return legs


def serving_mix(nreq, seed=2024):
    """Seeded request mix: 70% RPCA / 30% MC, m ~ U[500, 3000], n = m U[0.75, 1.25]
    rounded to 64, rank 0.05 min(m, n), RPCA corruption 5-10% U[-500, 500], MC
    sampling 10-20%, Poisson arrivals."""
    import numpy as np

    g = np.random.default_rng(seed)
    reqs = []
    for i in range(nreq):
        m = int(g.integers(500, 3001))
        n = max(64, int(round(m * g.uniform(0.75, 1.25) / 64.0)) * 64)
        r = max(1, int(round(0.05 * min(m, n))))
        if g.uniform() < 0.7:
            reqs.append(("rpca", m, n, r, float(g.uniform(0.05, 0.10)), 1000 + i))
        else:
            reqs.append(("mc", m, n, r, float(g.uniform(0.10, 0.20)), 1000 + i))
    return reqs


def bench_serving(args):
    import torch

    import paper_1012_0365_amd as blws
    import synth

    reqs = serving_mix(args.requests)
    log(f"[bench] serving: generating {len(reqs)} requests")
    data = []
    for kind, m, n, r, frac, seed in reqs:
        if kind == "rpca":
            inst = synth.rpca_instance(m, n, r, frac, AMP, seed)
            data.append((kind, m, n, torch.tensor(inst["D"], dtype=torch.float32, device="cuda")))
        else:
            inst = synth.mc_instance(m, n, r, frac, seed)
            data.append((kind, m, n,
                         torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda"),
                         torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda"),
                         torch.tensor(inst["values"], dtype=torch.float32, device="cuda")))
    torch.cuda.synchronize()
    mc_opts = blws.default_mc_opts()
    srv = blws.Server(0, max_slots=args.slots, group_products=not args.no_group,
                      group_window_us=args.group_window)
    # warm-up: one request of each kind
    for item in data[:2]:
        t = (srv.submit_rpca(item[3]) if item[0] == "rpca"
             else srv.submit_mc(item[1], item[2], item[3], item[4], item[5], opts=mc_opts))
        srv.wait(t)
    import numpy as np

    g = np.random.default_rng(7)
    gaps = g.exponential(1.0, len(data))  # Poisson arrivals, rate set below
    t_start = time.perf_counter()
    tickets = []
    # submit at the arrival times; mean gap 20 ms keeps the server loaded
    arrival = 0.0
    for (item, gap) in zip(data, gaps):
        arrival += 0.02 * gap
        while time.perf_counter() - t_start < arrival:
            time.sleep(0.0005)
        if item[0] == "rpca":
            tickets.append(srv.submit_rpca(item[3]))
        else:
            tickets.append(srv.submit_mc(item[1], item[2], item[3], item[4], item[5],
                                         opts=mc_opts))
    lat, iters, fails = [], 0, 0
    for t in tickets:
        try:
            res = srv.wait(t)
            lat.append(res[-1]["seconds"])
            iters += res[-1]["iters"]
        except blws.BlwsError:
            fails += 1
    total = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    seq = None
    if not args.no_plain:
        # the same requests one at a time, blocking FP64 solves (no server)
        ctx = blws.Context(0)
        t0 = time.perf_counter()
        for item in data:
            if item[0] == "rpca":
                ctx.rpca_solve(item[3].double())
            else:
                ctx.mc_solve(item[1], item[2], item[3], item[4], item[5].double(), opts=mc_opts)
        torch.cuda.synchronize()
        seq = len(data) / (time.perf_counter() - t0)
        ctx.close()
    return {
        "metric": "serving mix: solves/s with p50/p99 latency",
        "value": len(lat) / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 2,
        "ms_per_step": 1e3 * total / max(1, len(lat)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_mix_rpca70_mc30", "requests": len(reqs),
                   "m_range": [500, 3000], "arrivals": "poisson, mean gap 20 ms",
                   "max_slots": args.slots, "grouped_products": not args.no_group,
                   "group_window_us": args.group_window},
        "sequential_fp64_solves_per_s": seq,
        "speedup_vs_sequential_fp64": (len(lat) / total) / seq if seq else None,
        "latency_s_p50": pct(lat, 50),
        "latency_s_p99": pct(lat, 99),
        "svt_calls_per_s": iters / total,
        "failed": fails,
        "server_stats": st,
    }


def bench_copy():
    """One device-to-device copy of COPY_BYTES: the reference for HBM byte
    counters (FETCH_SIZE should read COPY_BYTES, WRITE_SIZE the same)."""
    import torch

    n = COPY_BYTES // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    assert bool((y[-16:] == x[-16:]).all())
    return {"workload": "copy", "bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES}


def bench_rpca4000():
    """The n = 4000 FP64 solve (rank 200, 10% U[-500, 500], rho 1.2, tol 1e-7),
    where D, Y, E and W (512 MB) exceed the 256 MB last-level cache: one warm
    solve, then one with every launch timed; reports the ALM epilogue's
    algorithmic bytes and rate (read D and Y, write E, Y and W per call)."""
    import torch

    import paper_1012_0365_amd as blws
    import synth

    inst = synth.rpca_instance(4000, 4000, 200, FRAC, AMP, 0)
    D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
    del inst
    ctx = blws.Context(0)
    opts = blws.default_alm_opts(rho=1.2)
    ctx.rpca_solve(D, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.rpca_solve(D, opts=opts)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.timing(True)
    t0 = time.perf_counter()
    _, _, info = ctx.rpca_solve(D, opts=opts)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    fams = {n: ctx.timing_get(n) for n in ctx.timing_families()}
    ctx.timing(False)
    out = {"workload": "rpca_inexact_alm_blws_n4000", "m": 4000, "n": 4000, "rank": 200,
           "precision": "f64", "solve_s": t_plain, "solve_s_with_events": t,
           "iters": info["iters"], "final_rank": info["rank"], "status": info["status"],
           "families_ms": {k: round(r["ms"], 3) for k, r in
                           sorted(fams.items(), key=lambda kv: -kv[1]["ms"]) if r["launches"]}}
    for name in ("alm_epilogue", "gemm_w"):
        rec = fams.get(name)
        if rec and rec["launches"]:
            e = roofline_entry(name, rec, "f64")
            e.pop("traffic")
            out[name] = dict(e, launches=rec["launches"])
    ctx.close()
    return out


def bench_mc5000():
    """Matrix completion by the ALM host at m = n = 5000, rank 50, 10% sampled,
    FP32 (rho 1.05, tol 1e-6): one warm solve, one untimed, then one with every
    launch timed; the sparse products' and the update's rates."""
    import torch

    import paper_1012_0365_amd as blws
    import synth

    inst = synth.mc_instance(5000, 5000, 50, 0.10, 0)
    rp = torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda")
    ci = torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda")
    vals = torch.tensor(inst["values"], dtype=torch.float32, device="cuda")
    ctx = blws.Context(0)
    opts = blws.default_mc_opts()
    ctx.mc_solve(5000, 5000, rp, ci, vals, opts=opts, r_cap=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.mc_solve(5000, 5000, rp, ci, vals, opts=opts, r_cap=256)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.timing(True)
    _, _, _, info = ctx.mc_solve(5000, 5000, rp, ci, vals, opts=opts, r_cap=256)
    torch.cuda.synchronize()
    fams = {n: ctx.timing_get(n) for n in ctx.timing_families()}
    ctx.timing(False)
    out = {"workload": "mc_alm_blws_n5000_r50_f32", "nnz": int(vals.numel()),
           "solve_s": t_plain, "iters": info["iters"], "rank": info["rank"],
           "status": info["status"],
           "families_ms": {k: round(r["ms"], 3) for k, r in
                           sorted(fams.items(), key=lambda kv: -kv[1]["ms"]) if r["launches"]}}
    for name in ("spmm", "mc_update"):
        rec = fams.get(name)
        if rec and rec["launches"]:
            e = roofline_entry(name, rec, "f32")
            e.pop("traffic")
            out[name] = dict(e, launches=rec["launches"])
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solve is a "
              "single-GPU path and no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        out = bench_copy()
    elif args.workload == "rpca4000":
        out = bench_rpca4000()
    elif args.workload == "mc5000":
        out = bench_mc5000()
    else:
        out = bench_serving(args) if args.workload == "serving" else bench_rpca(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
