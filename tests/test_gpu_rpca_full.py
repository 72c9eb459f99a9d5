"""GPU parity of blws_rpca_solve at full size (m = n = 2000, rank 100, 10%
corruption U[-500, 500], lambda = 1/sqrt(2000), tol 1e-7): the workload the
benchmark times, in the same launch configuration.

The oracle's exact-SVT solve at this size takes minutes, so its result is
stored (tests/golden/rpca_n2000_s0.json, written by make_golden.py from the
oracle alone): 4096 seeded sampled entries of A and E, the singular values of
A, norms, rank and nonzero count. The GPU solve is checked on the samples
entry by entry and on the properties that hold at any size (rank, spectrum,
residual, the E support count).
"""

import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "rpca_n2000_s0.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "these tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_1012_0365_amd as blws

    c = blws.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def instance(golden):
    p = golden["params"]
    return synth.rpca_instance(p["m"], p["n"], p["r"], p["frac"], p["amp"], p["seed"])


def _solve(torch, ctx, inst, dtype):
    D = torch.tensor(inst["D"], dtype=dtype, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    return A.double(), E.double(), info


def test_rpca_n2000_fp64_matches_oracle(torch, ctx, golden, instance):
    A, E, info = _solve(torch, ctx, instance, torch.float64)
    print(f"n2000 fp64: iters={info['iters']} rank={info['rank']} b={info['b_final']} "
          f"nnz_E={info['nnz_E']} residual={info['rel_residual']:.3e}")
    assert info["status"] == 0 and info["rel_residual"] < 1e-7
    assert info["rank"] == golden["rank"] == 100
    # same convex optimum: the two runs differ only in the ||D||_2 estimate that
    # seeds Y0 and mu0, so the iteration count may differ by a step or two
    assert abs(info["iters"] - golden["iters"]) <= 2
    pos = torch.tensor(golden["sample_pos"], device="cuda")
    a_s = A.reshape(-1)[pos].cpu().numpy()
    e_s = E.reshape(-1)[pos].cpu().numpy()
    a_ref = np.array(golden["A_samples"])
    e_ref = np.array(golden["E_samples"])
    err_a = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    err_e = np.linalg.norm(e_s - e_ref) / np.linalg.norm(e_ref)
    print(f"  sampled rel err A {err_a:.3e}  E {err_e:.3e}")
    assert err_a < 1e-6 and err_e < 1e-6
    # entrywise, against the largest sampled magnitude
    assert np.max(np.abs(a_s - a_ref)) < 1e-5 * np.max(np.abs(a_ref))
    # whole-matrix properties against the stored spectrum and norms
    sA = torch.linalg.svdvals(A).cpu().numpy()
    sref = np.array(golden["sigma_A"])
    r = golden["rank"]
    err_s = np.max(np.abs(sA[:r] - sref[:r]) / sref[:r])
    print(f"  max rel err of the top {r} singular values {err_s:.3e}")
    assert err_s < 1e-6
    assert np.all(sA[r:r + 16] < 1e-9 * sA[0])
    assert abs(float(torch.linalg.norm(A)) - golden["norm_A"]) < 1e-6 * golden["norm_A"]
    assert abs(float(torch.linalg.norm(E)) - golden["norm_E"]) < 1e-6 * golden["norm_E"]
    # support of E: entries that sit at the shrinkage threshold may flip
    assert abs(info["nnz_E"] - golden["nnz_E"]) <= 40
    # planted-matrix recovery at the level of the oracle's own solution
    A0 = torch.tensor(instance["A0"], device="cuda")
    rec = float(torch.linalg.norm(A - A0) / torch.linalg.norm(A0))
    assert rec < 2 * golden["rel_err_vs_A0"] + 1e-7


def test_rpca_n2000_fp32_matches_oracle(torch, ctx, golden, instance):
    """FP32 storage (products on FP32 matrix cores; Gram, Cholesky, small SVD
    and the reconstruction in FP64): the converged solve to 1e-6 of the
    oracle's exact solution on the sampled entries of A and E, the same rank,
    and the top singular values of A. (The BF16 ladder: test_gpu_precision.)"""
    mode = "f32"
    D = torch.tensor(instance["D"], dtype=torch.float32, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    A, E = A.double(), E.double()
    pos = torch.tensor(golden["sample_pos"], device="cuda")
    a_s = A.reshape(-1)[pos].cpu().numpy()
    e_s = E.reshape(-1)[pos].cpu().numpy()
    a_ref = np.array(golden["A_samples"])
    e_ref = np.array(golden["E_samples"])
    err_a = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    err_e = np.linalg.norm(e_s - e_ref) / np.linalg.norm(e_ref)
    r = golden["rank"]
    sA = torch.linalg.svdvals(A).cpu().numpy()
    sref = np.array(golden["sigma_A"])
    err_s = np.max(np.abs(sA[:r] - sref[:r]) / sref[:r])
    print(f"n2000 {mode}: iters={info['iters']} rank={info['rank']} status={info['status']} "
          f"residual={info['rel_residual']:.3e} sampled rel err A {err_a:.3e} E {err_e:.3e} "
          f"top-{r} sigma {err_s:.3e}")
    assert info["status"] == 0 and info["rel_residual"] < 1e-7
    assert info["rank"] == golden["rank"]
    assert err_a < 1e-6 and err_e < 1e-6 and err_s < 1e-6


# n = 4000, rank 200, 10% corruption U[-500, 500], rho = 1.2: the precision
# variant's size. Stored values from the oracle's BLWS form (same algorithm).
@pytest.fixture(scope="module")
def golden4k():
    with open(os.path.join(HERE, "golden", "rpca_n4000_s0.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("mode", ["f64", "bf16"])
def test_rpca_n4000_matches_oracle(torch, ctx, golden4k, mode):
    import paper_1012_0365_amd as blws

    p = golden4k["params"]
    inst = synth.rpca_instance(p["m"], p["n"], p["r"], p["frac"], p["amp"], p["seed"])
    D = torch.tensor(inst["D"], dtype=torch.float64 if mode == "f64" else torch.float32,
                     device="cuda")
    A, E, info = ctx.rpca_solve(D, opts=blws.default_alm_opts(rho=p["rho"]), bf16=mode == "bf16")
    torch.cuda.synchronize()
    pos = torch.tensor(golden4k["sample_pos"], device="cuda")
    a_s = A.double().reshape(-1)[pos].cpu().numpy()
    e_s = E.double().reshape(-1)[pos].cpu().numpy()
    a_ref = np.array(golden4k["A_samples"])
    e_ref = np.array(golden4k["E_samples"])
    err_a = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    err_e = np.linalg.norm(e_s - e_ref) / np.linalg.norm(e_ref)
    r = p["r"]
    sA = torch.linalg.svdvals(A.double()).cpu().numpy()
    sref = np.array(golden4k["sigma_A"])
    err_s = np.max(np.abs(sA[:r] - sref[:r]) / sref[:r])
    print(f"n4000 {mode}: iters={info['iters']} (oracle {golden4k['iters']}) rank={info['rank']} "
          f"(oracle {golden4k['rank']}) bf16 iters={info['iters_bf16']} sampled rel err A "
          f"{err_a:.3e} E {err_e:.3e}, top-{r} sigma {err_s:.3e}, {info['seconds']:.3f}s")
    assert info["status"] == 0
    assert abs(info["rank"] - golden4k["rank"]) <= 2
    assert abs(info["iters"] - golden4k["iters"]) <= 2
    assert err_a < 1e-6 and err_e < 1e-6 and err_s < 1e-6
