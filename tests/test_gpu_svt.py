"""GPU parity of the BLWS SVT step (blws_svt) against the oracle's plain-loop
BLWS step on the same W and warm block, FP64 path.

Bars: Ritz values above the threshold to 1e-10 relative; A to 1e-9 relative
Frobenius; the output blocks orthonormal; the retained subspaces equal
(projectors) when the spectral gap allows. Singular vectors are compared
through projectors only: they are unique up to sign (and rotation for ties).
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


def dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def run_gpu(torch, ctx, W, eps, U, V, warm=True, dtype=None):
    dtype = dtype or torch.float64
    Wd, Ud, Vd = dev(torch, W, dtype), dev(torch, U, dtype), dev(torch, V, dtype)
    A = torch.empty_like(Wd)
    S, rank = ctx.svt(Wd, eps, Ud, Vd, warm=warm, A=A)
    torch.cuda.synchronize()
    return host(Ud).astype(np.float64), host(Vd).astype(np.float64), host(S), \
        host(A).astype(np.float64), int(host(rank)[0])


def proj(X):
    return X @ X.T


def compare(gpu, ref, eps, tol_s=1e-10, tol_a=1e-9):
    Ug, Vg, Sg, Ag, rg = gpu
    Uo, Vo, So, Ao, ro = ref
    b = So.size
    assert rg == ro
    above = So > eps
    assert np.all(np.abs(Sg[above] - So[above]) <= tol_s * So[above]), \
        np.max(np.abs(Sg[above] - So[above]) / So[above])
    # below-threshold Ritz values (warm-start only): normwise agreement
    assert np.all(np.abs(Sg - So) <= 1e-10 * So[0])
    na = np.linalg.norm(Ao)
    if na > 0:
        assert np.linalg.norm(Ag - Ao) <= tol_a * na, np.linalg.norm(Ag - Ao) / na
    else:
        assert np.abs(Ag).max() == 0.0
    assert np.abs(Ug.T @ Ug - np.eye(b)).max() < 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(b)).max() < 1e-12
    if 0 < ro < b and So[ro - 1] - So[ro] > 1e-3 * So[0]:
        assert np.abs(proj(Ug[:, :ro]) - proj(Uo[:, :ro])).max() < 1e-9
        assert np.abs(proj(Vg[:, :ro]) - proj(Vo[:, :ro])).max() < 1e-9


def warm_block(W, b, delta, seed):
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(seed)
    m, n = W.shape
    Ui = np.linalg.qr(U0[:, :b] + delta * g.standard_normal((m, b)))[0]
    Vi = np.linalg.qr(V0t[:b].T + delta * g.standard_normal((n, b)))[0]
    return Ui, Vi


CASES = [
    # (m, n, b, eps, kind)
    (60, 50, 8, 3.5, "spectrum"),
    (200, 200, 16, 30.0, "rpca"),
    (301, 157, 24, 5.0, "random"),
    (157, 301, 24, 5.0, "random"),
    (513, 700, 64, 12.0, "random"),
    (64, 64, 1, 1.0, "random"),
]


def make_w(m, n, kind, seed):
    if kind == "spectrum":
        sigma = np.r_[np.linspace(100, 50, 5), np.geomspace(5, 0.01, min(m, n) - 5)]
        return synth.prescribed_spectrum(m, n, sigma, seed)[0]
    if kind == "rpca":
        return synth.rpca_instance(m, n, 10, 0.05, 50.0, seed)["D"]
    return synth.gaussian((m, n), seed) + 3.0 * synth.gaussian((m, 5), seed + 1) @ \
        synth.gaussian((5, n), seed + 2)


@pytest.mark.parametrize("m,n,b,eps,kind", CASES)
def test_svt_warm_matches_oracle(torch, ctx, m, n, b, eps, kind):
    W = make_w(m, n, kind, seed=m + n)
    U, V = warm_block(W, b, 1e-2, seed=1)
    ref = oracle.blws_step(W, eps, U, V)
    gpu = run_gpu(torch, ctx, W, eps, U, V)
    compare(gpu, ref, eps)


def spectrum_w(m, n, r, seed):
    """r values spread over [50, 100] above a geometric tail from 5 to 0.01."""
    sigma = np.r_[np.linspace(100, 50, r), np.geomspace(5, 0.01, min(m, n) - r)]
    return synth.prescribed_spectrum(m, n, sigma, seed)[0]


# The block widths the solvers run at: b = 112 (the projected matrix is
# 224 x 224: the one-workgroup bidiagonalisation; one Cholesky-QR block),
# b = 128 and b = 208 (256 x 256 and 416 x 416: 32 and 192 cooperative
# bidiagonalisation steps, then the one-workgroup kernel on the trailing
# 224 x 224; at b = 208 blocks wider than 128 columns, orthonormalised in two
# chunks with block Gram-Schmidt between them).
WIDE = [(600, 560, 112, 100, 20.0), (600, 560, 128, 100, 20.0), (1000, 900, 208, 200, 20.0)]


@pytest.mark.parametrize("m,n,b,r,eps", WIDE)
def test_svt_warm_production_widths(torch, ctx, m, n, b, r, eps):
    W = spectrum_w(m, n, r, seed=m)
    U, V = warm_block(W, b, 1e-2, seed=3)
    ref = oracle.blws_step(W, eps, U, V)
    compare(run_gpu(torch, ctx, W, eps, U, V), ref, eps)


@pytest.fixture(scope="module")
def snapshot2000():
    """Iteration 15 of the oracle's BLWS solve of the benchmark problem (n = 2000,
    rank 100, 10% corruption U[-500, 500]): that iteration's W, eps = 1/mu and
    warm block (b = 112, 100 Ritz values above eps: the steady state)."""
    inst = synth.rpca_instance(2000, 2000, 100, 0.10, 500.0, 0)
    W, U, V, eps = oracle.rpca_snapshot(inst["D"], 15)
    ref = oracle.blws_step(W, eps, U, V)
    return W, U, V, eps, ref


def test_svt_benchmark_snapshot_fp64(torch, ctx, snapshot2000):
    W, U, V, eps, ref = snapshot2000
    assert U.shape[1] == 112 and ref[4] == 100
    compare(run_gpu(torch, ctx, W, eps, U, V), ref, eps)


def test_svt_benchmark_snapshot_fp32(torch, ctx, snapshot2000):
    """FP32 storage of W, U, V (products on FP32 matrix cores, FP64 Gram,
    Cholesky and small SVD): values above eps to 1e-6 relative, the rank
    exact, A to 1e-5, the blocks orthonormal to 1e-6."""
    W, U, V, eps, (Uo, Vo, So, Ao, ro) = snapshot2000
    Ug, Vg, Sg, Ag, rg = run_gpu(torch, ctx, W, eps, U, V, dtype=torch.float32)
    above = So > eps
    err_s = np.max(np.abs(Sg[above] - So[above]) / So[above])
    err_a = np.linalg.norm(Ag - Ao) / np.linalg.norm(Ao)
    print(f"snapshot fp32: sigma {err_s:.2e}  A {err_a:.2e}")
    assert rg == ro and err_s < 1e-6 and err_a < 1e-5
    assert np.abs(Ug.T @ Ug - np.eye(112)).max() < 1e-6
    assert np.abs(Vg.T @ Vg - np.eye(112)).max() < 1e-6


@pytest.mark.parametrize("m,n,b,eps,kind", CASES[:5])
def test_svt_fp32_warm_matches_oracle(torch, ctx, m, n, b, eps, kind):
    """FP32 path (W, U, V stored in FP32; Gram matrices, Cholesky and the small
    SVD in FP64): its second Cholesky-QR pass takes the near-identity form
    (||G - I||_2 <= 2.5e-4), which leaves the blocks orthonormal to FP32
    rounding. Bars scaled to FP32: Ritz values to 1e-5 of the largest, A to
    1e-4, orthonormality to 1e-6."""
    W = make_w(m, n, kind, seed=m + n)
    U, V = warm_block(W, b, 1e-2, seed=1)
    Uo, Vo, So, Ao, ro = oracle.blws_step(W, eps, U, V)
    Ug, Vg, Sg, Ag, rg = run_gpu(torch, ctx, W, eps, U, V, dtype=torch.float32)
    assert np.abs(Ug.T @ Ug - np.eye(b)).max() < 1e-6
    assert np.abs(Vg.T @ Vg - np.eye(b)).max() < 1e-6
    assert np.abs(Sg - So).max() <= 1e-5 * So[0], np.abs(Sg - So).max() / So[0]
    na = np.linalg.norm(Ao)
    if na > 0:
        assert np.linalg.norm(Ag - Ao) <= 1e-4 * na, np.linalg.norm(Ag - Ao) / na
    # the rank can differ only where a Ritz value sits within FP32 error of eps
    if rg != ro:
        assert np.min(np.abs(So - eps)) <= 1e-5 * So[0]


@pytest.mark.parametrize("m,n,b,eps,kind", CASES[:4])
def test_svt_cold_matches_oracle(torch, ctx, m, n, b, eps, kind):
    W = make_w(m, n, kind, seed=m + 2 * n)
    Uo, Vo = oracle.cold_block(W, b, pow_steps=2, seed=20101202, stream_v=1)
    ref = oracle.blws_step(W, eps, Uo, Vo)
    gpu = run_gpu(torch, ctx, W, eps, np.zeros((m, b)), np.zeros((n, b)), warm=False)
    compare(gpu, ref, eps)


@pytest.mark.parametrize("pow_steps", [0, 1, 2])
def test_cold_block_spans_match_oracle(torch, ctx, pow_steps):
    m, n, b = 157, 301, 24
    W = make_w(m, n, "random", seed=m + 2 * n)
    Uo, Vo = oracle.cold_block(W, b, pow_steps=pow_steps, seed=20101202, stream_v=1)
    Ug, Vg = ctx.cold_block(dev(torch, W), b, pow_steps=pow_steps)
    torch.cuda.synchronize()
    Ug, Vg = host(Ug), host(Vg)
    assert np.abs(Ug.T @ Ug - np.eye(b)).max() < 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(b)).max() < 1e-12
    assert np.abs(proj(Vg) - proj(Vo)).max() < 1e-10
    assert np.abs(proj(Ug) - proj(Uo)).max() < 1e-10


def test_svt_from_oracle_cold_block(torch, ctx):
    """The BLWS step from the oracle's cold block (passed as a warm block)."""
    m, n, b, eps = 157, 301, 24, 5.0
    W = make_w(m, n, "random", seed=m + 2 * n)
    Uo, Vo = oracle.cold_block(W, b, pow_steps=2, seed=20101202, stream_v=1)
    ref = oracle.blws_step(W, eps, Uo, Vo)
    compare(run_gpu(torch, ctx, W, eps, Uo, Vo), ref, eps)


def test_svt_exact_warm_start_breakdown(torch, ctx):
    """R_1 = 0: the new block is rounding noise; the result must still be the
    exact top-b and T_eps(W)."""
    sigma = np.r_[np.linspace(100, 50, 5), np.geomspace(5, 0.01, 45)]
    W, _, _ = synth.prescribed_spectrum(60, 50, sigma, seed=3)
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    b = 8
    Ug, Vg, Sg, Ag, rg = run_gpu(torch, ctx, W, 3.5, U0[:, :b], V0t[:b].T)
    assert np.allclose(Sg, sigma[:b], rtol=1e-12)
    Aex, _, rex = oracle.svt_exact(W, 3.5)
    assert rg == rex
    assert np.linalg.norm(Ag - Aex) <= 1e-11 * np.linalg.norm(Aex)
    assert np.abs(Ug.T @ Ug - np.eye(b)).max() < 1e-12


@pytest.mark.parametrize("side", ["V", "U"])
@pytest.mark.parametrize("kappa", [1e4, 1e6, 1e8, 1e10, 1e12])
def test_svt_ill_conditioned_krylov_block(torch, ctx, side, kappa):
    """The new block F0 (side V) or G0 (side U) with condition number kappa
    after column scaling, not singular. Up to kappa ~ 3e6 the two Cholesky-QR
    passes keep the near-dependent pair; beyond it the first pass finds the
    scaled pivot (about 4 / kappa^2) below 1e-13 and the fallback pass
    re-forms that column from the vectors (Gram-Schmidt with
    reorthogonalisation), so the block's span holds the pair to rounding as
    the oracle's Householder QR does. Every singular pair above eps lies in
    the span, so the values above eps, A and the retained subspaces are
    those of W and the oracle's."""
    c = synth.ill_conditioned_block(200, 180, 12, kappa, side, seed=11)
    W, sig, eps = c["W"], c["sigma"], 30.0
    gpu = run_gpu(torch, ctx, W, eps, c["U"], c["V"])
    Ug, Vg, Sg, Ag, rg = gpu
    Uo, Vo, So, Ao, ro = oracle.blws_step(W, eps, c["U"], c["V"])
    print(f"ill-conditioned {side} kappa {kappa:.0e}: |dS|/s1 "
          f"{np.abs(Sg[:rg] - sig[:rg]).max() / sig[0]:.1e}, |A - A_oracle| / |A_oracle| "
          f"{np.linalg.norm(Ag - Ao) / np.linalg.norm(Ao):.1e}", flush=True)
    assert rg == ro == 11
    assert np.abs(Sg[:rg] - sig[:rg]).max() <= 1e-12 * sig[0]
    assert np.abs(Sg[:rg] - So[:ro]).max() <= 1e-12 * sig[0]
    assert np.linalg.norm(Ag - Ao) <= 1e-11 * np.linalg.norm(Ao)
    assert np.abs(Ug.T @ Ug - np.eye(12)).max() < 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(12)).max() < 1e-12
    assert np.abs(proj(Ug[:, :rg]) - proj(Uo[:, :ro])).max() < 1e-10
    assert np.abs(proj(Vg[:, :rg]) - proj(Vo[:, :ro])).max() < 1e-10


def test_svt_exactly_low_rank_w(torch, ctx):
    """rank(W) < 2b: the Krylov block is rank deficient (dependent columns are
    replaced and reorthogonalised); values and A still match the oracle."""
    g = np.random.default_rng(4)
    W = g.standard_normal((90, 3)) @ g.standard_normal((3, 70))
    U = np.linalg.qr(g.standard_normal((90, 6)))[0]
    V = np.linalg.qr(g.standard_normal((70, 6)))[0]
    Ug, Vg, Sg, Ag, rg = run_gpu(torch, ctx, W, 0.5, U, V)
    sv = np.linalg.svd(W, compute_uv=False)
    assert np.allclose(Sg[:3], sv[:3], rtol=1e-11)
    assert np.all(Sg[3:] <= 1e-11 * sv[0])
    Aex, _, _ = oracle.svt_exact(W, 0.5)
    assert np.linalg.norm(Ag - Aex) <= 1e-10 * np.linalg.norm(Aex)
    assert np.abs(Ug.T @ Ug - np.eye(6)).max() < 1e-11


def test_svt_threshold_above_spectrum_and_zero_matrix(torch, ctx):
    W = synth.gaussian((80, 60), seed=5)
    U, V = warm_block(W, 4, 1e-3, seed=2)
    s1 = np.linalg.norm(W, 2)
    _, _, Sg, Ag, rg = run_gpu(torch, ctx, W, 1.5 * s1, U, V)
    assert rg == 0 and np.abs(Ag).max() == 0.0
    Ug, Vg, Sg, Ag, rg = run_gpu(torch, ctx, np.zeros((80, 60)), 0.0, U, V)
    assert rg == 0 and np.all(Sg == 0.0) and np.abs(Ag).max() == 0.0
    assert np.abs(Ug.T @ Ug - np.eye(4)).max() < 1e-12


def test_svt_rejects_bad_arguments(torch, ctx):
    import paper_1012_0365_amd as blws

    W = torch.zeros(20, 10, dtype=torch.float64, device="cuda")
    U = torch.zeros(20, 6, dtype=torch.float64, device="cuda")
    V = torch.zeros(10, 6, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        ctx.svt(W, 1.0, U, V)  # 2b > min(m, n)
    assert e.value.status == -1
    U = torch.zeros(20, 2, dtype=torch.float64, device="cuda")
    V = torch.zeros(10, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError):
        ctx.svt(W, -1.0, U, V)
    with pytest.raises(blws.BlwsError):
        ctx.svt(W, float("nan"), U, V)
