"""GPU parity of blws_mc_svt_solve (the SVT algorithm for matrix completion,
Table 2's host, with BLWS thresholding on the purely sparse Y) against the
oracle's same algorithm.

The oracle runs with the library's reading of the ||P_Omega(M)||_2 estimate
(at most 8 BLWS steps; it fixes k0 and so Y_0), so both follow the same
iterates: the same iteration count and rank, the completed matrix to 1e-7 in
FP64 (1e-6 in FP32). Recovery of the planted matrix is at Table 2's level.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
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


def _instance(m, n, r, ratio, seed=0):
    s = ratio * r * (m + n - r)  # s / d_r with d_r = r (m + n - r)
    return synth.mc_instance(m, n, r, s / float(m * n), seed)


def _dev(torch, inst, dtype):
    return (torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["values"], dtype=dtype, device="cuda"))


def _rel_planted(U, S, V, L, R):
    nA2 = float(np.sum(S ** 2))
    nM2 = float(np.sum((L.T @ L) * (R.T @ R)))
    ip = float(np.sum(((U * S).T @ L) * (V.T @ R)))
    return np.sqrt(max(nA2 + nM2 - 2.0 * ip, 0.0)) / np.sqrt(nM2)


def _rel_between(Ua, Sa, Va, Ub, Sb, Vb):
    """||A_a - A_b||_F / ||A_b||_F for A = U diag(S) V^T, from the factors."""
    g = lambda U1, S1, V1, U2, S2, V2: float(np.sum(((U1 * S1).T @ (U2 * S2)) * (V1.T @ V2)))
    d2 = g(Ua, Sa, Va, Ua, Sa, Va) + g(Ub, Sb, Vb, Ub, Sb, Vb) - 2.0 * g(Ua, Sa, Va, Ub, Sb, Vb)
    return np.sqrt(max(d2, 0.0)) / np.sqrt(g(Ub, Sb, Vb, Ub, Sb, Vb))


# (m, n, r, s / d_r): the last two at Table 2's r = 50 sampling (s / d_r = 5)
CASES = [(300, 260, 5, 6), (5000, 5000, 10, 6), (1000, 1000, 50, 5), (2000, 2000, 50, 5)]


@pytest.mark.parametrize("m,n,r,ratio", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mc_svt_matches_oracle(torch, blws, ctx, m, n, r, ratio, prec):
    inst = _instance(m, n, r, ratio)
    cap = 64 if r <= 10 else 2 * r + 64  # room for the block to grow past the rank
    ref = oracle.mc_svt(m, n, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                        r_cap=cap, norm_steps=GPU_NORM_STEPS)
    dt = torch.float64 if prec == "f64" else torch.float32
    U, S, V, info = ctx.mc_svt_solve(m, n, *_dev(torch, inst, dt), r_cap=cap)
    torch.cuda.synchronize()
    U, S, V = U.double().cpu().numpy(), S.cpu().numpy(), V.double().cpu().numpy()
    err = _rel_between(U, S, V, ref["U"], ref["S"], ref["V"])
    rec = _rel_planted(U, S, V, inst["L"], inst["R"])
    print(f"mc svt {m}x{n} r{r} {prec}: iters={info['iters']} (oracle {ref['info']['iters']}) "
          f"rank={info['rank']} rel err vs oracle {err:.2e} vs planted {rec:.2e} "
          f"{info['seconds']:.3f}s")
    assert info["status"] == 0 and info["rank"] == ref["rank"] == r
    # the samples are stored in FP32 in the FP32 solve
    tol_s1 = 1e-10 if prec == "f64" else 1e-6
    assert abs(info["norm2_D"] - ref["info"]["norm2_D"]) <= tol_s1 * ref["info"]["norm2_D"]
    # rounding differences of the two implementations grow over ~130 steps of
    # Y_k = Y_{k-1} + delta P_Omega(M - X_k) (observed 2e-8 .. 8e-8)
    if prec == "f64":
        assert info["iters"] == ref["info"]["iters"]
        assert err < 1e-7
    else:
        assert abs(info["iters"] - ref["info"]["iters"]) <= 1
        assert err < 1e-6
    assert rec < 3e-4


def test_mc_svt_default_norm_reaches_the_same_solution(torch, blws, ctx):
    """Against the oracle's own reading (||P_Omega(M)||_2 to 1e-13): k0 and the
    iterates may differ, the completed matrix agrees to the tolerance's scale."""
    m, n, r, ratio = 400, 400, 8, 6
    inst = _instance(m, n, r, ratio)
    ref = oracle.mc_svt(m, n, inst["row_ptr"], inst["col_idx"], inst["values"], mode="blws",
                        r_cap=64)
    U, S, V, info = ctx.mc_svt_solve(m, n, *_dev(torch, inst, torch.float64), r_cap=64)
    torch.cuda.synchronize()
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    assert info["status"] == 0 and info["rank"] == ref["rank"] == r
    assert abs(info["iters"] - ref["info"]["iters"]) <= 3
    assert _rel_between(U, S, V, ref["U"], ref["S"], ref["V"]) < 3e-4


def test_mc_svt_rejects_bad_arguments(torch, blws, ctx):
    inst = _instance(60, 50, 3, 6)
    rp, ci, vals = _dev(torch, inst, torch.float64)
    bad = ci.clone()
    bad[3] = 50
    with pytest.raises(blws.BlwsError) as e:
        ctx.mc_svt_solve(60, 50, rp, bad, vals)
    assert e.value.status == -1
    with pytest.raises(blws.BlwsError):
        ctx.mc_svt_solve(60, 50, rp, ci, vals, opts=blws.default_svt_mc_opts(tol=0.0))
