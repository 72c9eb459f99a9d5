"""GPU parity of the library's building blocks, called through the C ABI."""

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


def test_counter_generator_is_bit_exact(torch, ctx):
    for rows, cols, seed, stream in [(1, 1, 0, 0), (37, 5, 20101202, 3), (300, 64, 7, 1 << 20)]:
        X = torch.empty(rows, cols, dtype=torch.float64, device="cuda")
        ctx.fill_uniform(X, seed, stream)
        ref = oracle.fill_uniform(rows, cols, seed, stream)
        assert np.array_equal(host(X), ref)


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 16, 32), (130, 112, 2000), (2000, 112, 2000),
                                   (17, 200, 45), (224, 224, 1999), (5, 3, 70000),
                                   # tall-skinny forms: NN with K <= 512, TN with M, N <= 512
                                   (2000, 112, 112), (1999, 511, 512), (33, 300, 3),
                                   (5000, 256, 224), (112, 112, 2000), (448, 448, 2001),
                                   (512, 512, 4096), (100, 37, 130),
                                   # TN split-K sums over 16 or more splits: 128 splits
                                   # and 3700 outputs (not a multiple of 64), 32 splits
                                   # and 1500 outputs, 17 splits (quarters of 5, 5, 5, 2)
                                   (100, 37, 4096), (50, 30, 1000), (112, 112, 540)])
def test_gemm_matches_numpy(torch, ctx, trans, M, N, K):
    g = np.random.default_rng(M * 7 + N * 3 + K)
    A = g.standard_normal((K, M) if trans else (M, K))
    B = g.standard_normal((K, N))
    C0 = g.standard_normal((M, N))
    ref = 0.75 * ((A.T if trans else A) @ B) - 0.5 * C0
    C = dev(torch, C0)
    ctx.gemm_f64(dev(torch, A), dev(torch, B), C, trans_a=trans, alpha=0.75, beta=-0.5)
    torch.cuda.synchronize()
    scale = np.abs(A).max() * np.abs(B).max() * K + np.abs(C0).max()
    assert np.abs(host(C) - ref).max() <= 1e-14 * scale


@pytest.mark.parametrize("M", [700, 224])
def test_gemm_is_deterministic(torch, ctx, M):
    # split-K sums are reduced in chunk order: the same bits on every call
    g = np.random.default_rng(1)
    A, B = dev(torch, g.standard_normal((3000, M))), dev(torch, g.standard_normal((3000, 96)))
    outs = []
    for _ in range(3):
        C = torch.zeros(M, 96, dtype=torch.float64, device="cuda")
        ctx.gemm_f64(A, B, C, trans_a=True)
        outs.append(host(C))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


@pytest.mark.parametrize("N", [1, 2, 7, 32, 64, 224, 225, 240, 256, 257, 272, 300, 320, 352, 416, 512, 640, 1024])
def test_small_svd_matches_oracle_jacobi(torch, ctx, N):
    g = np.random.default_rng(N)
    B = g.standard_normal((N, N)) * np.geomspace(1.0, 1e-6, N)[None, :]
    UB, S, VB = ctx.small_svd_f64(dev(torch, B))
    torch.cuda.synchronize()
    UB, S, VB = host(UB), host(S), host(VB)
    _, So, _ = oracle.jacobi_svd(B)
    assert np.all(np.abs(S - So) <= 1e-13 * So[0] + 1e-12 * So)
    assert np.abs(UB.T @ UB - np.eye(N)).max() < 1e-13
    assert np.abs(VB.T @ VB - np.eye(N)).max() < 1e-13
    assert np.linalg.norm(UB * S @ VB.T - B) <= 1e-13 * np.linalg.norm(B)


@pytest.mark.parametrize("N", [224, 256, 352, 416, 512])
@pytest.mark.parametrize("kind", ["repeated", "clustered"])
def test_small_svd_multiple_and_clustered_values(torch, ctx, N, kind):
    """B = Q1 diag(sigma) Q2^T with nonzero values repeated (groups of 4 equal
    values) or clustered (groups of 4 within 1e-12 relative): the inverse
    iteration branch. Values to 1e-13 against the oracle's Jacobi and against
    the prescribed sigma; vectors through orthonormality, the reconstruction
    and the spectral projectors of whole groups (the vectors inside a group are
    not unique)."""
    g = np.random.default_rng(N + len(kind))
    base = np.geomspace(100.0, 1e-3, N // 4)
    if kind == "repeated":
        sigma = np.repeat(base, 4)
    else:
        sigma = (base[:, None] * (1.0 + 1e-12 * np.arange(4))[None, :]).reshape(-1)
    sigma = np.sort(sigma)[::-1]
    B, q1, q2 = synth.prescribed_spectrum(N, N, sigma, seed=N)
    UB, S, VB = ctx.small_svd_f64(dev(torch, B))
    torch.cuda.synchronize()
    UB, S, VB = host(UB), host(S), host(VB)
    _, So, _ = oracle.jacobi_svd(B)
    assert np.all(np.abs(S - So) <= 1e-13 * So[0] + 1e-12 * So)
    assert np.all(np.abs(S - sigma) <= 1e-13 * sigma[0] + 1e-12 * sigma)
    assert np.abs(UB.T @ UB - np.eye(N)).max() < 1e-13
    assert np.abs(VB.T @ VB - np.eye(N)).max() < 1e-13
    # backward error of a stable SVD: a small multiple of N u ||B||_F. The
    # vectors of a multiple value come from inverse iteration on the
    # Golub-Kahan tridiagonal and a Cholesky-QR polish of each side, which can
    # turn the two sides of a group of equal values by slightly different
    # rotations: 2 to 34 N u ||B||_F measured over N = 192 .. 416 with
    # repeated values, below 0.1 N u ||B||_F with clustered ones
    nb = np.linalg.norm(B)
    bound = (64 if kind == "repeated" else 16) * N * 2.0**-53 * nb
    assert np.linalg.norm(UB * S @ VB.T - B) <= bound
    for k in range(0, N, 4):
        Pg = UB[:, k:k + 4] @ UB[:, k:k + 4].T
        Pq = q1[:, k:k + 4] @ q1[:, k:k + 4].T
        # group gap over the group scale bounds the projector error (Davis-Kahan)
        gap = min(abs(sigma[k - 1] - sigma[k]) if k else np.inf,
                  abs(sigma[k + 3] - sigma[k + 4]) if k + 4 < N else np.inf)
        assert np.abs(Pg - Pq).max() <= 1e-13 * nb / gap + 1e-12


def test_small_svd_rank_deficient(torch, ctx):
    g = np.random.default_rng(3)
    B = g.standard_normal((40, 3)) @ g.standard_normal((3, 40))
    B[:, 5] = 0.0
    UB, S, VB = ctx.small_svd_f64(dev(torch, B))
    torch.cuda.synchronize()
    UB, S, VB = host(UB), host(S), host(VB)
    assert np.all(S[3:] <= 1e-13 * S[0])
    assert np.abs(UB.T @ UB - np.eye(40)).max() < 1e-12
    assert np.abs(VB.T @ VB - np.eye(40)).max() < 1e-12
