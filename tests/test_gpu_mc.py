"""GPU parity of blws_mc_solve (ALM matrix completion + BLWS, W applied as low
rank plus sparse) against the oracle.

Small cases run live against the oracle: the BLWS ALM (same algorithm, same
iteration count and rank, the iterate to 1e-8), the exact-SVT ALM (the plain
form: the same optimum to 1e-6) and the planted matrix. The full-size case
(n = 5000, rank 50, 10% sampled, FP32) is checked against stored oracle
values on seeded sampled entries.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
OPTS = dict(rho=1.1, tol=1e-8, mu0_scale=1.0)
GPU_NORM_STEPS = 8  # the library's default norm_steps


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "these tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def blws():
    import paper_1012_0365_amd as blws

    return blws


@pytest.fixture(scope="module")
def ctx(torch, blws):
    c = blws.Context(0)
    yield c
    c.close()


def _dev(torch, inst, dtype):
    return (torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["values"], dtype=dtype, device="cuda"))


def _dense(U, S, V):
    return (U * S) @ V.T


CASES = [(200, 150, 5, 0.3, 0), (300, 250, 8, 0.25, 1)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}x{c[1]}r{c[2]}")
def case(request):
    m, n, r, frac, seed = request.param
    inst = synth.mc_instance(m, n, r, frac, seed)
    # the oracle's BLWS form with the GPU's reading of the ||D||_2 estimate (at
    # most 8 BLWS steps), so that both follow the same iterates
    bl = oracle.mc(m, n, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                   r_cap=64, norm_steps=GPU_NORM_STEPS, **OPTS)
    return inst, bl


def test_mc_fp64_matches_oracle(torch, blws, ctx, case):
    inst, bl = case
    m, n = inst["m"], inst["n"]
    rp, ci, vals = _dev(torch, inst, torch.float64)
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, vals, opts=blws.default_mc_opts(**OPTS), r_cap=64)
    torch.cuda.synchronize()
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    assert info["status"] == 0 and info["rel_residual"] < 1e-8
    # same algorithm as the oracle's BLWS ALM: same trajectory
    assert info["iters"] == bl["info"]["iters"]
    assert info["rank"] == bl["rank"] == len(bl["S"])
    assert abs(info["norm2_D"] - bl["info"]["norm2_D"]) <= 1e-12 * bl["info"]["norm2_D"]
    assert np.max(np.abs(S - bl["S"]) / bl["S"]) < 1e-8
    A = _dense(U, S, V)
    A_or = _dense(bl["U"], bl["S"], bl["V"])
    assert np.linalg.norm(A - A_or) / np.linalg.norm(A_or) < 1e-8
    # factors: orthonormal columns
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-12
    # recovery of the planted matrix
    M = inst["L"] @ inst["R"].T
    assert np.linalg.norm(A - M) / np.linalg.norm(M) < 1e-6


def test_mc_fp64_matches_exact_form(torch, blws, ctx):
    m, n, r, frac, seed = CASES[0]
    inst = synth.mc_instance(m, n, r, frac, seed)
    ex = oracle.mc(m, n, inst["row_ptr"], inst["col_idx"], inst["values"], mode="exact",
                   r_cap=64, **OPTS)
    rp, ci, vals = _dev(torch, inst, torch.float64)
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, vals, opts=blws.default_mc_opts(**OPTS), r_cap=64)
    A = _dense(U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy())
    A_ex = _dense(ex["U"], ex["S"], ex["V"])
    assert info["rank"] == ex["rank"]
    assert np.linalg.norm(A - A_ex) / np.linalg.norm(A_ex) < 1e-6


@pytest.fixture(scope="module")
def wide_case():
    """Rank 30 at 25% sampling, rho 1.05 (the library's MC default, with which
    the oracle recovers the planted rank here): the block grows to 32 columns
    over the solve, so the columns added on widening are drawn as well."""
    m, n, r, frac, seed = 800, 700, 30, 0.25, 2
    inst = synth.mc_instance(m, n, r, frac, seed)
    bl = oracle.mc(m, n, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                   r_cap=96, norm_steps=GPU_NORM_STEPS, rho=1.05, tol=1e-8, mu0_scale=1.0)
    return inst, bl


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mc_rank30_matches_oracle(torch, blws, ctx, wide_case, prec):
    inst, bl = wide_case
    m, n = inst["m"], inst["n"]
    dt = torch.float64 if prec == "f64" else torch.float32
    rp, ci, vals = _dev(torch, inst, dt)
    tol = 1e-8 if prec == "f64" else 1e-6
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, vals,
                                 opts=blws.default_mc_opts(rho=1.05, tol=tol, mu0_scale=1.0),
                                 r_cap=96)
    torch.cuda.synchronize()
    U, S, V = U.double().cpu().numpy(), S.cpu().numpy(), V.double().cpu().numpy()
    A = _dense(U, S, V)
    A_or = _dense(bl["U"], bl["S"], bl["V"])
    err = np.linalg.norm(A - A_or) / np.linalg.norm(A_or)
    M = inst["L"] @ inst["R"].T
    rec = np.linalg.norm(A - M) / np.linalg.norm(M)
    print(f"mc rank 30 {prec}: iters={info['iters']} (oracle {bl['info']['iters']}) "
          f"rank={info['rank']} err vs oracle {err:.2e} vs planted {rec:.2e}", flush=True)
    assert info["status"] == 0 and info["rank"] == bl["rank"] == 30
    if prec == "f64":
        # the same algorithm: same trajectory
        assert info["iters"] == bl["info"]["iters"]
        assert np.max(np.abs(S - bl["S"]) / bl["S"]) < 1e-8
        assert err < 1e-8 and rec < 1e-6
    else:
        # FP32 stopped at 1e-6 (the FP32 bar of the other MC solves)
        assert err < 1e-5


def test_mc_fp32_small(torch, blws, ctx, case):
    inst, bl = case
    m, n = inst["m"], inst["n"]
    rp, ci, vals = _dev(torch, inst, torch.float32)
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, vals,
                                 opts=blws.default_mc_opts(rho=1.1, tol=1e-6, mu0_scale=1.0),
                                 r_cap=64)
    A = _dense(U.double().cpu().numpy(), S.cpu().numpy(), V.double().cpu().numpy())
    A_or = _dense(bl["U"], bl["S"], bl["V"])
    err = np.linalg.norm(A - A_or) / np.linalg.norm(A_or)
    print(f"mc fp32 {m}x{n}: iters={info['iters']} rank={info['rank']} err={err:.3e}")
    assert info["status"] == 0 and info["rank"] == bl["rank"]
    assert err < 1e-5


def test_mc_row_order_of_entries_irrelevant(torch, blws, ctx):
    """Columns within a row in any order: the transposed pattern is rebuilt in
    row order, so only the summation order of the row products changes."""
    m, n, r, frac, seed = CASES[0]
    inst = synth.mc_instance(m, n, r, frac, seed)
    rp_h, ci_h, v_h = inst["row_ptr"], inst["col_idx"].copy(), inst["values"].copy()
    g = np.random.default_rng(5)
    for i in range(m):
        a, z = rp_h[i], rp_h[i + 1]
        p = g.permutation(z - a)
        ci_h[a:z] = ci_h[a:z][p]
        v_h[a:z] = v_h[a:z][p]
    opts = blws.default_mc_opts(**OPTS)
    rp, ci, vals = _dev(torch, inst, torch.float64)
    U1, S1, V1, i1 = ctx.mc_solve(m, n, rp, ci, vals, opts=opts, r_cap=64)
    ci2 = torch.tensor(ci_h, dtype=torch.int32, device="cuda")
    v2 = torch.tensor(v_h, dtype=torch.float64, device="cuda")
    U2, S2, V2, i2 = ctx.mc_solve(m, n, rp, ci2, v2, opts=opts, r_cap=64)
    assert i1["iters"] == i2["iters"] and i1["rank"] == i2["rank"]
    A1 = _dense(U1.cpu().numpy(), S1.cpu().numpy(), V1.cpu().numpy())
    A2 = _dense(U2.cpu().numpy(), S2.cpu().numpy(), V2.cpu().numpy())
    assert np.linalg.norm(A1 - A2) / np.linalg.norm(A1) < 1e-10


def test_mc_deterministic(torch, blws, ctx):
    m, n, r, frac, seed = CASES[0]
    inst = synth.mc_instance(m, n, r, frac, seed)
    rp, ci, vals = _dev(torch, inst, torch.float64)
    opts = blws.default_mc_opts(**OPTS)
    a = ctx.mc_solve(m, n, rp, ci, vals, opts=opts, r_cap=64)
    b = ctx.mc_solve(m, n, rp, ci, vals, opts=opts, r_cap=64)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def test_mc_rejects_bad_pattern(torch, blws, ctx):
    m, n, r, frac, seed = CASES[0]
    inst = synth.mc_instance(m, n, r, frac, seed)
    rp, ci, vals = _dev(torch, inst, torch.float64)
    bad_c = ci.clone()
    bad_c[7] = n  # column out of range
    with pytest.raises(blws.BlwsError) as e:
        ctx.mc_solve(m, n, rp, bad_c, vals)
    assert e.value.status == -1 and "column" in str(e.value)
    bad_r = rp.clone()
    bad_r[5] = bad_r[7] + 1  # not nondecreasing
    with pytest.raises(blws.BlwsError) as e:
        ctx.mc_solve(m, n, bad_r, ci, vals)
    assert e.value.status == -1 and "row_ptr" in str(e.value)


def test_mc_zero_samples(torch, blws, ctx):
    m, n = 40, 30
    rp = torch.zeros(m + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    vals = torch.zeros(0, dtype=torch.float64, device="cuda")
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, vals, r_cap=8)
    assert info["status"] == 0 and info["rank"] == 0 and U.shape == (m, 0)


def test_mc_n5000_fp32_matches_stored_oracle(torch, blws, ctx):
    path = os.path.join(HERE, "golden", "mc_n5000_s0.json")
    with open(path) as f:
        g = json.load(f)
    p = g["params"]
    inst = synth.mc_instance(p["m"], p["n"], p["r"], p["frac"], p["seed"])
    rp, ci, vals = _dev(torch, inst, torch.float32)
    opts = blws.default_mc_opts(tol=p["tol"], rho=p["rho"], mu0_scale=p["mu0_scale"])
    U, S, V, info = ctx.mc_solve(p["m"], p["n"], rp, ci, vals, opts=opts, r_cap=256)
    torch.cuda.synchronize()
    pos = np.array(g["sample_pos"])
    rows = torch.tensor(pos // p["n"], device="cuda")
    cols = torch.tensor(pos % p["n"], device="cuda")
    a_s = ((U.double()[rows] * S) * V.double()[cols]).sum(1).cpu().numpy()
    a_ref = np.array(g["A_samples"])
    m_ref = np.array(g["M_samples"])
    err = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    rec = np.linalg.norm(a_s - m_ref) / np.linalg.norm(m_ref)
    r = p["r"]
    s_ref = np.array(g["sigma_A"])
    s_err = np.max(np.abs(S.cpu().numpy()[:r] - s_ref[:r]) / s_ref[:r])
    print(f"mc n5000 fp32: iters={info['iters']} (oracle {g['iters']}) rank={info['rank']} "
          f"(oracle {g['rank']}) sampled rel err vs oracle {err:.3e}, vs planted {rec:.3e}, "
          f"top-{r} sigma {s_err:.3e}, {info['seconds']:.3f}s")
    # the planted rank; the iteration counts differ by the GPU's 8-step
    # ||D||_2 estimate (it sets mu_0), which moves the iterates, not the optimum
    assert info["status"] == 0 and info["rank"] == g["rank"] == r
    assert abs(info["iters"] - g["iters"]) <= 8
    assert err < 1e-6 and s_err < 1e-6
    # recovery of the planted matrix at the level the tolerance allows
    assert rec < 1e-5
