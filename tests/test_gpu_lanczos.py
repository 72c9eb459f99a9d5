"""GPU parity of blws_svt_lanczos, the start-block ablations of Sec. 4.1
(Algorithms 2-3 taken literally on [[0, W], [W^T, 0]] from the split, aug and
half-information starts, with k blocks), and of robust PCA run with it,
against the oracle's form on the explicitly formed augmented matrix."""

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


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def signed_warm(W, b, delta, seed):
    """Noisy top-b singular subspaces keeping the exact vectors' signs (the
    pairing of u_j with v_j that the aug start relies on)."""
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(seed)
    m, n = W.shape

    def orth_signed(X):
        Q, R = np.linalg.qr(X)
        return Q * np.sign(np.diag(R))

    return (orth_signed(U0[:, :b] + delta * g.standard_normal((m, b))),
            orth_signed(V0t[:b].T + delta * g.standard_normal((n, b))))


def make_w(m, n, seed):
    p = min(m, n)
    sigma = np.r_[np.linspace(100.0, 40.0, p // 4), np.geomspace(20.0, 1e-3, p - p // 4)]
    return synth.prescribed_spectrum(m, n, sigma, seed)[0]


CASES = [
    # (m, n, b, start, k): k c covers the three small-SVD paths of T_k + c I
    (90, 70, 8, "split", 2),
    (90, 70, 8, "aug", 2),
    (90, 70, 8, "left", 2),
    (90, 70, 8, "right", 2),
    (131, 97, 8, "aug", 3),
    (131, 97, 8, "split", 3),
    (131, 97, 8, "left", 4),
    (64, 64, 1, "aug", 2),
    (300, 260, 56, "aug", 4),    # k c = 224: one-workgroup bidiagonalisation
    (300, 260, 40, "split", 3),  # k c = 240: 16 cooperative steps, then one workgroup
    (400, 380, 100, "aug", 3),   # k c = 300: 76 cooperative steps, then one workgroup
]


@pytest.mark.parametrize("m,n,b,start,k", CASES)
def test_lanczos_step_matches_oracle(torch, ctx, m, n, b, start, k):
    W = make_w(m, n, seed=m + 7 * k)
    U, V = signed_warm(W, b, 1e-2, seed=b)
    sv = np.linalg.svd(W, compute_uv=False)
    eps = 0.5 * (sv[b // 2] + sv[max(b // 2 - 1, 0)]) if b > 1 else 0.5 * sv[0]
    Uo, Vo, So, Ao, ro = oracle.lanczos_svt(W, eps, U, V, start, k)
    Wd, Ud, Vd = dev(torch, W), dev(torch, U), dev(torch, V)
    A = torch.empty_like(Wd)
    S, rank = ctx.svt_lanczos(Wd, eps, Ud, Vd, start=start, k=k, A=A)
    torch.cuda.synchronize()
    Sg, Ag, rg = S.cpu().numpy(), A.cpu().numpy(), int(rank.cpu().numpy()[0])
    Ug, Vg = Ud.cpu().numpy(), Vd.cpu().numpy()
    print(f"lanczos {start} k={k} m={m} n={n} b={b}: |dS|/s1 {np.abs(Sg - So).max() / sv[0]:.1e}",
          flush=True)
    assert rg == ro
    assert np.abs(Sg - So).max() <= 1e-10 * sv[0]
    assert np.linalg.norm(Ag - Ao) <= 1e-9 * np.linalg.norm(Ao)
    if start != "aug":  # split and half starts: the halves of the Ritz vectors are exact halves
        assert np.abs(Ug.T @ Ug - np.eye(b)).max() < 1e-11
        assert np.abs(Vg.T @ Vg - np.eye(b)).max() < 1e-11
    # the Ritz vectors above eps, one by one up to sign (distinct values here)
    for j in range(ro):
        sgn = np.sign(Ug[:, j] @ Uo[:, j])
        assert np.abs(sgn * Ug[:, j] - Uo[:, j]).max() < 1e-8
        assert np.abs(sgn * Vg[:, j] - Vo[:, j]).max() < 1e-8


def test_lanczos_split_k2_equals_default_step(torch, ctx):
    """The literal form from blockdiag(U, V) with k = 2 and the default step
    (which skips the zero blocks) are the same method: same Ritz values and SVT."""
    m, n, b = 250, 210, 24
    W = make_w(m, n, seed=3)
    U, V = signed_warm(W, b, 1e-3, seed=4)
    eps = 30.0
    Wd = dev(torch, W)
    U1, V1, U2, V2 = dev(torch, U), dev(torch, V), dev(torch, U), dev(torch, V)
    A1, A2 = torch.empty_like(Wd), torch.empty_like(Wd)
    S1, r1 = ctx.svt(Wd, eps, U1, V1, A=A1)
    S2, r2 = ctx.svt_lanczos(Wd, eps, U2, V2, start="split", k=2, A=A2)
    torch.cuda.synchronize()
    assert int(r1.cpu()[0]) == int(r2.cpu()[0])
    S1, S2 = S1.cpu().numpy(), S2.cpu().numpy()
    assert np.abs(S1 - S2).max() <= 1e-11 * S1[0]
    assert torch.linalg.norm(A1 - A2).item() <= 1e-10 * torch.linalg.norm(A1).item()


def test_lanczos_argument_errors(torch, ctx):
    import paper_1012_0365_amd as blws

    W = dev(torch, make_w(700, 700, seed=1))
    U = torch.zeros(700, 300, dtype=torch.float64, device="cuda")
    V = torch.zeros(700, 300, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:  # k c = 1200 > 1024
        ctx.svt_lanczos(W, 1.0, U, V, start="split", k=2)
    assert "1024" in str(e.value)
    Ws = dev(torch, make_w(40, 30, seed=2))
    Us = torch.zeros(40, 4, dtype=torch.float64, device="cuda")
    Vs = torch.zeros(30, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError):  # k c = 80 > m + n = 70
        ctx.svt_lanczos(Ws, 1.0, Us, Vs, start="aug", k=20)


@pytest.fixture(scope="module")
def rpca_case():
    return synth.rpca_instance(200, 200, 10, 0.1, 500.0, 1)


@pytest.mark.parametrize("start,k", [("aug", 2), ("split", 3)])
def test_rpca_ablation_matches_oracle(torch, ctx, rpca_case, start, k):
    """Whole inexact-ALM solves with each SVT taken by the literal procedure:
    the same iterates as the oracle's solve with the same start and k (and the
    GPU's 8-step reading of the ||D||_2 estimate)."""
    import paper_1012_0365_amd as blws

    inst = rpca_case
    bl = oracle.rpca(inst["D"], mode="blws", norm_steps=8, svt_start=oracle.STARTS[start],
                     k_blocks=k)
    D = dev(torch, inst["D"])
    opts = blws.default_alm_opts(svt_start=oracle.STARTS[start], k_blocks=k)
    A, E, info = ctx.rpca_solve(D, opts=opts)
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    print(f"rpca {start} k={k}: iters {info['iters']} (oracle {bl['info']['iters']}), "
          f"err vs A0 {np.linalg.norm(A - inst['A0']) / np.linalg.norm(inst['A0']):.2e}",
          flush=True)
    assert info["status"] == bl["info"]["status"] == 0
    assert info["iters"] == bl["info"]["iters"]
    assert info["rank"] == bl["info"]["rank"]
    # the aug start's Ritz vectors are only nearly orthonormal (U = sqrt(2)
    # Y_top) and feed the next start block, so rounding differences between the
    # two implementations grow faster over the solve than with the split start
    tol = 1e-5 if start == "aug" else 1e-7
    assert np.linalg.norm(A - bl["A"]) <= tol * np.linalg.norm(bl["A"])
    assert np.linalg.norm(A - inst["A0"]) <= 1e-5 * np.linalg.norm(inst["A0"])


def test_rpca_ablation_rejected_outside_fp64_rpca(torch, ctx, rpca_case):
    import paper_1012_0365_amd as blws

    D = torch.tensor(rpca_case["D"], dtype=torch.float32, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        ctx.rpca_solve(D, opts=blws.default_alm_opts(svt_start=1))
    assert "FP64" in str(e.value)
