"""GPU parity of the FP32 / BF16 matrix-core products and of the BF16
precision ladder of the RPCA solve.

The low-precision W-product kernel is checked element by element against the
FP64 product of the same inputs (for BF16: the inputs rounded to BF16 in
numpy, so only the FP32 accumulation differs), within the componentwise bound
of FP32 accumulation. The ladder solve is checked against the oracle: live at
m = n = 200 and, at the n = 2000 size, against the stored oracle solution, to
the 1e-6 relative error the FP32 and BF16 forms must reach.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
U32 = 2.0 ** -24


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


def bf16_bits(x):
    """Round float32 values to BF16 (nearest even); returns the uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


SHAPES = [(2000, 112, 2000), (130, 37, 77), (64, 256, 4096), (1000, 16, 3000), (5, 200, 300)]


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_gemm_lp_fp32(torch, ctx, shape, trans):
    M, N, K = shape
    g = np.random.default_rng(M + N + K)
    A = g.standard_normal((K, M) if trans else (M, K)).astype(np.float32)
    B = g.standard_normal((K, N)).astype(np.float32)
    C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
    ctx.gemm_lp(torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda"), C, trans_a=trans)
    opA = (A.T if trans else A).astype(np.float64)
    ref = opA @ B.astype(np.float64)
    bound = 2 * K * U32 * (np.abs(opA) @ np.abs(B.astype(np.float64))) + 1e-30
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_gemm_lp_bf16(torch, ctx, shape, trans):
    M, N, K = shape
    g = np.random.default_rng(7 * M + N + K)
    A = g.standard_normal((K, M) if trans else (M, K)).astype(np.float32)
    B = g.standard_normal((K, N)).astype(np.float32)
    Ab = bf16_bits(A)
    C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
    ctx.gemm_lp(torch.tensor(Ab.view(np.int16), device="cuda"), torch.tensor(B, device="cuda"), C,
                trans_a=trans)
    Av = bf16_value(Ab)
    Bv = bf16_value(bf16_bits(B))
    opA = Av.T if trans else Av
    ref = opA @ Bv
    bound = 2 * K * U32 * (np.abs(opA) @ np.abs(Bv)) + 1e-30
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


def test_rpca_bf16_ladder_small(torch, ctx):
    inst = synth.rpca_instance(200, 200, 10, 0.05, 50.0, 0)
    ex = oracle.rpca(inst["D"], mode="exact")
    D = torch.tensor(inst["D"], dtype=torch.float32, device="cuda")
    A, E, info = ctx.rpca_solve(D, bf16=True)
    A = A.double().cpu().numpy()
    err = np.linalg.norm(A - ex["A"]) / np.linalg.norm(ex["A"])
    print(f"bf16 ladder 200: iters={info['iters']} bf16 iters={info['iters_bf16']} "
          f"refined={info['refined']} err={err:.3e}")
    assert info["status"] == 0 and info["rank"] == 10
    assert info["iters_bf16"] >= 1
    assert err < 1e-6


def test_rpca_bf16_ladder_n2000_matches_oracle(torch, ctx):
    with open(os.path.join(HERE, "golden", "rpca_n2000_s0.json")) as f:
        g = json.load(f)
    p = g["params"]
    inst = synth.rpca_instance(p["m"], p["n"], p["r"], p["frac"], p["amp"], p["seed"])
    D = torch.tensor(inst["D"], dtype=torch.float32, device="cuda")
    A, E, info = ctx.rpca_solve(D, bf16=True)
    torch.cuda.synchronize()
    pos = torch.tensor(g["sample_pos"], device="cuda")
    a_s = A.double().reshape(-1)[pos].cpu().numpy()
    e_s = E.double().reshape(-1)[pos].cpu().numpy()
    a_ref, e_ref = np.array(g["A_samples"]), np.array(g["E_samples"])
    err_a = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    err_e = np.linalg.norm(e_s - e_ref) / np.linalg.norm(e_ref)
    print(f"bf16 ladder n2000: iters={info['iters']} bf16 iters={info['iters_bf16']} "
          f"refined={info['refined']} sampled rel err A {err_a:.3e} E {err_e:.3e}")
    assert info["status"] == 0 and info["rank"] == g["rank"]
    assert info["iters_bf16"] >= 1
    assert err_a < 1e-6 and err_e < 1e-6
