"""GPU parity of blws_rpca_solve (inexact ALM + BLWS) against the oracle.

Small configuration (m = n = 200, rank 10, 5% corruption U[-50, 50]), run live
against the oracle: FP64 must match the exact-SVT ALM (the plain form) to 1e-6
relative Frobenius error in A and E at tol 1e-7, and the oracle's BLWS ALM (the
same algorithm) iteration for iteration.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module", params=[0, 1])
def small_case(request):
    inst = synth.rpca_instance(200, 200, 10, 0.05, 50.0, request.param)
    ex = oracle.rpca(inst["D"], mode="exact")
    # the oracle's BLWS form with the GPU's reading of the ||D||_2 estimate (at
    # most 8 BLWS steps, the library's default norm_steps), so that both follow
    # the same iterates; the exact form above is the plain solve
    bl = oracle.rpca(inst["D"], mode="blws", norm_steps=8)
    return inst, ex, bl


def test_rpca_fp64_small_matches_oracle(torch, ctx, small_case):
    inst, ex, bl = small_case
    D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    A, E = A.cpu().numpy(), E.cpu().numpy()
    assert info["status"] == 0 and info["rel_residual"] < 1e-7
    assert info["rank"] == ex["info"]["rank"] == 10
    # the unique optimum of the convex program, reached by the plain form
    assert rel(A, ex["A"]) < 1e-6 and rel(E, ex["E"]) < 1e-6
    # the same algorithm: same iteration count, rank trajectory and iterate
    assert info["iters"] == bl["info"]["iters"]
    assert abs(info["norm2_D"] - bl["info"]["norm2_D"]) <= 1e-12 * bl["info"]["norm2_D"]
    # (rounding differences of two FP64 implementations grow over ~20 ALM steps)
    assert rel(A, bl["A"]) < 1e-8 and rel(E, bl["E"]) < 1e-8
    assert info["nnz_E"] == bl["info"]["nnz_E"]
    # exact recovery of the planted matrix (Table 1 regime)
    assert rel(A, inst["A0"]) < 2e-6


@pytest.mark.parametrize("m", [500, 1000])
def test_rpca_table1_rows_match_oracle(torch, ctx, m):
    """Table 1's m = 500 and 1000 rows (rank m / 10, 10% of entries corrupted
    with U[-500, 500], lambda = 1/sqrt(m)): the GPU's FP64 solve follows the
    oracle's BLWS solve (same iterations, rank and support of E, A to 1e-8) and
    lands on the paper's row (rank m / 10, ||E||_0 within 0.05% of m^2 / 10,
    the planted A to 5e-5)."""
    r, k = m // 10, m * m // 10
    inst = synth.rpca_instance(m, m, r, 0.10, 500.0, 0)
    bl = oracle.rpca(inst["D"], mode="blws", norm_steps=8)
    D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    A, E = A.cpu().numpy(), E.cpu().numpy()
    print(f"table 1 m={m}: iters {info['iters']} (oracle {bl['info']['iters']}), rank "
          f"{info['rank']}, nnz(E) {info['nnz_E']}, |A - A0| / |A0| {rel(A, inst['A0']):.2e}",
          flush=True)
    assert info["status"] == 0 == bl["info"]["status"]
    assert info["iters"] == bl["info"]["iters"] and info["rank"] == bl["info"]["rank"] == r
    assert info["nnz_E"] == bl["info"]["nnz_E"] and abs(info["nnz_E"] - k) <= 5e-4 * k
    assert rel(A, bl["A"]) < 1e-8 and rel(E, bl["E"]) < 1e-8
    assert rel(A, inst["A0"]) < 5e-5


def test_rpca_fp32_small(torch, ctx, small_case):
    inst, ex, bl = small_case
    D = torch.tensor(inst["D"], dtype=torch.float32, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    A = A.double().cpu().numpy()
    assert info["status"] == 0 and info["rel_residual"] < 1e-7
    assert info["rank"] == 10
    err = rel(A, ex["A"])
    err_bl = rel(A, bl["A"])
    print(f"fp32 small: iters={info['iters']} rel err vs oracle-exact={err:.3e} "
          f"vs oracle-blws={err_bl:.3e} residual={info['rel_residual']:.3e}", flush=True)
    # the FP32 bar: 1e-6 relative to the oracle's solution
    assert err < 1e-6 and err_bl < 1e-6


def test_rpca_zero_and_nan_inputs(torch, ctx):
    import paper_1012_0365_amd as blws

    D = torch.zeros(64, 48, dtype=torch.float64, device="cuda")
    A, E, info = ctx.rpca_solve(D)
    torch.cuda.synchronize()
    assert info["status"] == 0 and torch.count_nonzero(A) == 0 and torch.count_nonzero(E) == 0
    D[3, 4] = float("nan")
    with pytest.raises(blws.BlwsError) as e:
        ctx.rpca_solve(D)
    assert e.value.status == -4
