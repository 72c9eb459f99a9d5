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


# ---------------------------------------------------------------------------
# Split-precision BF16 x 3 products: A = A_hi + A_lo, B = B_hi + B_lo (each
# half BF16), C = A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation.
# ---------------------------------------------------------------------------


def split_bf16(x):
    """(hi bits, lo bits) with hi = bf16(x), lo = bf16(x - hi), in numpy."""
    hi = bf16_bits(x)
    lo = bf16_bits(np.asarray(x, dtype=np.float32) - bf16_value(hi).astype(np.float32))
    return hi, lo


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_gemm_bf16x3(torch, ctx, shape, trans):
    M, N, K = shape
    g = np.random.default_rng(11 * M + N + K)
    A = g.standard_normal((K, M) if trans else (M, K)).astype(np.float32)
    B = g.standard_normal((K, N)).astype(np.float32)
    Ah, Al = split_bf16(A)
    C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
    ctx.gemm_bf16x3(torch.tensor(Ah.view(np.int16), device="cuda"),
                    torch.tensor(Al.view(np.int16), device="cuda"),
                    torch.tensor(B, device="cuda"), C, trans_a=trans)
    got = C.cpu().numpy().astype(np.float64)
    Bh, Bl = split_bf16(B)
    ah, al = bf16_value(Ah), bf16_value(Al)
    bh, bl = bf16_value(Bh), bf16_value(Bl)
    if trans:
        ah, al = ah.T, al.T
    # the three BF16 products are exact in FP32 pieces: only the FP32
    # accumulation of 3K terms differs from the FP64 sum
    ref = ah @ bh + ah @ bl + al @ bh
    mag = np.abs(ah) @ np.abs(bh) + np.abs(ah) @ np.abs(bl) + np.abs(al) @ np.abs(bh)
    err = np.abs(got - ref)
    bound = 2 * 3 * K * U32 * mag + 1e-30
    assert np.all(err <= bound), float(np.max(err / bound))
    # against the FP32 inputs themselves: the splits leave |x - hi - lo| <=
    # 2^-17 |x| and the dropped A_lo B_lo term is below 2^-16 |A||B|
    opA = (A.T if trans else A).astype(np.float64)
    full = opA @ B.astype(np.float64)
    absprod = np.abs(opA) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(got - full) <= (2 ** -14 + 6 * K * U32) * absprod + 1e-30)


def test_svt_bf16x3_matches_oracle(torch, ctx):
    """One warm BLWS step with BF16 x 3 W products against the oracle's FP64
    step: Ritz values and A to about 16 significant bits of the products."""
    sigma = np.r_[np.linspace(100, 50, 5), np.geomspace(5, 0.01, 195)]
    W, _, _ = synth.prescribed_spectrum(300, 200, sigma, seed=5)
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(6)
    b = 16
    U = np.linalg.qr(U0[:, :b] + 1e-3 * g.standard_normal((300, b)))[0]
    V = np.linalg.qr(V0t[:b].T + 1e-3 * g.standard_normal((200, b)))[0]
    _, _, So, Ao, ro = oracle.blws_step(W, 3.5, U, V)
    Wd = torch.tensor(W, dtype=torch.float32, device="cuda")
    Ud = torch.tensor(U, dtype=torch.float32, device="cuda")
    Vd = torch.tensor(V, dtype=torch.float32, device="cuda")
    A = torch.empty_like(Wd)
    S, rank = ctx.svt(Wd, 3.5, Ud, Vd, A=A, bf16x3=True)
    torch.cuda.synchronize()
    Sg, Ag = S.cpu().numpy(), A.double().cpu().numpy()
    derr = np.abs(Sg - So).max() / So[0]
    aerr = np.linalg.norm(Ag - Ao) / np.linalg.norm(Ao)
    print(f"bf16x3 svt: sigma err {derr:.2e}, A err {aerr:.2e}")
    assert int(rank.cpu()[0]) == ro
    # 16-bit products: a few units of 2^-16 (1.5e-5) of sigma_1 on the values
    assert derr < 1e-4 and aerr < 1e-4


def test_rpca_bf16_ladder3_small(torch, ctx):
    inst = synth.rpca_instance(200, 200, 10, 0.05, 50.0, 0)
    ex = oracle.rpca(inst["D"], mode="exact")
    D = torch.tensor(inst["D"], dtype=torch.float32, device="cuda")
    import paper_1012_0365_amd as blws

    A, E, info = ctx.rpca_solve(D, bf16=True, opts=blws.default_alm_opts(ladder3_tol=1e-5))
    A = A.double().cpu().numpy()
    err = np.linalg.norm(A - ex["A"]) / np.linalg.norm(ex["A"])
    print(f"bf16 x3 ladder 200: iters={info['iters']} bf16 {info['iters_bf16']} "
          f"bf16x3 {info['iters_bf16x3']} refined={info['refined']} err={err:.3e}")
    assert info["status"] == 0 and info["rank"] == 10
    assert info["iters_bf16"] >= 1 and info["iters_bf16x3"] >= 1
    assert err < 1e-6


def test_rpca_bf16_ladder3_n2000_matches_oracle(torch, ctx):
    with open(os.path.join(HERE, "golden", "rpca_n2000_s0.json")) as f:
        g = json.load(f)
    p = g["params"]
    inst = synth.rpca_instance(p["m"], p["n"], p["r"], p["frac"], p["amp"], p["seed"])
    D = torch.tensor(inst["D"], dtype=torch.float32, device="cuda")
    import paper_1012_0365_amd as blws

    A, E, info = ctx.rpca_solve(D, bf16=True, opts=blws.default_alm_opts(ladder3_tol=1e-5))
    torch.cuda.synchronize()
    pos = torch.tensor(g["sample_pos"], device="cuda")
    a_s = A.double().reshape(-1)[pos].cpu().numpy()
    e_s = E.double().reshape(-1)[pos].cpu().numpy()
    a_ref, e_ref = np.array(g["A_samples"]), np.array(g["E_samples"])
    err_a = np.linalg.norm(a_s - a_ref) / np.linalg.norm(a_ref)
    err_e = np.linalg.norm(e_s - e_ref) / np.linalg.norm(e_ref)
    print(f"bf16 x3 ladder n2000: iters={info['iters']} bf16 {info['iters_bf16']} "
          f"bf16x3 {info['iters_bf16x3']} refined={info['refined']} "
          f"sampled rel err A {err_a:.3e} E {err_e:.3e}")
    assert info["status"] == 0 and info["rank"] == g["rank"]
    assert info["iters_bf16x3"] >= 1
    assert err_a < 1e-6 and err_e < 1e-6
