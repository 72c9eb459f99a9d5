"""blws_svt_noalloc (static scratch, no allocation inside the call) against
blws_svt on the same inputs, calls in a row each smaller than the last, in
FP64 (Ritz values above eps to 1e-10 relative, A to 1e-9, ranks equal) and
FP32 (values to 1e-6 of the largest, A to 1e-5); and its size limit."""

import numpy as np
import pytest

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


def _case(m, n, b, r, seed):
    sigma = np.r_[np.linspace(100, 50, r), np.geomspace(5, 0.01, min(m, n) - r)]
    W = synth.prescribed_spectrum(m, n, sigma, seed)[0]
    U0, _, V0t = np.linalg.svd(W, full_matrices=False)
    g = np.random.default_rng(seed)
    U = np.linalg.qr(U0[:, :b] + 1e-2 * g.standard_normal((m, b)))[0]
    V = np.linalg.qr(V0t[:b].T + 1e-2 * g.standard_normal((n, b)))[0]
    return W, U, V


def _run(torch, ctx, W, U, V, eps, dtype, noalloc):
    Wd = torch.tensor(W, dtype=dtype, device="cuda")
    Ud = torch.tensor(U, dtype=dtype, device="cuda")
    Vd = torch.tensor(V, dtype=dtype, device="cuda")
    A = torch.empty_like(Wd)
    S = torch.empty(U.shape[1], dtype=torch.float64, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.svt(Wd, eps, Ud, Vd, A=A, S=S, rank=rank, noalloc=noalloc)
    torch.cuda.synchronize()
    return S.cpu().numpy(), int(rank.cpu()[0]), A.double().cpu().numpy(), \
        Ud.double().cpu().numpy()


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_noalloc_matches_svt_two_calls(torch, ctx, dtype_name):
    dtype = getattr(torch, dtype_name)
    # each call smaller than the one before: the static scratch keeps the
    # previous call's contents, which must not leak into the next. b = 160
    # (small SVD of N = 320: cooperative steps, then the one-workgroup kernel,
    # the back-transformation's 512-row form) on the single stream here
    # against the two-stream path of blws_svt
    for (m, n, b, r, eps) in [(700, 650, 160, 140, 20.0), (600, 560, 112, 100, 20.0),
                              (300, 250, 24, 20, 20.0)]:
        W, U, V = _case(m, n, b, r, seed=m)
        print(f"noalloc {dtype_name} m={m} n={n} b={b}", flush=True)
        Sr, rr, Ar, Ur = _run(torch, ctx, W, U, V, eps, dtype, noalloc=False)
        Sn, rn, An, Un = _run(torch, ctx, W, U, V, eps, dtype, noalloc=True)
        assert rn == rr == r
        above = Sr > eps
        if dtype == torch.float64:
            assert np.all(np.abs(Sn[above] - Sr[above]) <= 1e-10 * Sr[above])
            assert np.linalg.norm(An - Ar) <= 1e-9 * np.linalg.norm(Ar)
            assert np.abs(Un.T @ Un - np.eye(b)).max() < 1e-12
        else:
            assert np.abs(Sn - Sr).max() <= 1e-6 * Sr[0]
            assert np.linalg.norm(An - Ar) <= 1e-5 * np.linalg.norm(Ar)
            assert np.abs(Un.T @ Un - np.eye(b)).max() < 1e-6


def test_noalloc_rejects_sizes_beyond_the_static_scratch(torch, ctx):
    import paper_1012_0365_amd as blws

    m = n = 4000
    b = 512
    W = torch.zeros(m, n, dtype=torch.float64, device="cuda")
    U = torch.zeros(m, b, dtype=torch.float64, device="cuda")
    V = torch.zeros(n, b, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        ctx.svt(W, 1.0, U, V, noalloc=True)
    assert e.value.status == -1 and "MiB" in str(e.value)
