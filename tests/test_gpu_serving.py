"""The request server (continuous batching of RPCA and MC solves on one GPU).

Every request must compute exactly what the blocking solver computes for the
same arguments, whatever else is in flight: results are compared bit for bit
with solves run alone, with the W-products of solves stepping together in
grouped launches and without, and each served result against the oracle's
solve of the same problem. Also checked: solves overlap (more than one in flight),
admission by the memory budget (a budget below one request's workspace runs
them one at a time), per-request errors, argument checks at submission, and
polling.
"""

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
def blws():
    import paper_1012_0365_amd as blws

    return blws


@pytest.fixture(scope="module")
def ctx(blws, torch):
    c = blws.Context(0)
    yield c
    c.close()


MC_OPTS = dict(rho=1.1, tol=1e-6, mu0_scale=1.0)


def rpca_req(torch, m, n, r, frac, amp, seed, dtype, bf16=False):
    inst = synth.rpca_instance(m, n, r, frac, amp, seed)
    return ("rpca", torch.tensor(inst["D"], dtype=dtype, device="cuda"), bf16)


def mc_req(torch, m, n, r, frac, seed, dtype):
    inst = synth.mc_instance(m, n, r, frac, seed)
    return ("mc", m, n, torch.tensor(inst["row_ptr"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["col_idx"], dtype=torch.int32, device="cuda"),
            torch.tensor(inst["values"], dtype=dtype, device="cuda"))


@pytest.fixture(scope="module")
def mix(torch):
    f64, f32 = torch.float64, torch.float32
    return [
        rpca_req(torch, 300, 300, 15, 0.05, 50.0, 0, f64),
        mc_req(torch, 300, 250, 8, 0.25, 1, f64),
        rpca_req(torch, 420, 360, 20, 0.08, 100.0, 2, f32),
        rpca_req(torch, 512, 512, 25, 0.10, 500.0, 3, f32, bf16=True),
        mc_req(torch, 400, 400, 10, 0.15, 4, f32),
        rpca_req(torch, 640, 576, 30, 0.07, 200.0, 5, f64),
        rpca_req(torch, 200, 260, 10, 0.05, 50.0, 6, f64),
        mc_req(torch, 256, 320, 6, 0.2, 7, f64),
    ]


def solve_alone(ctx, blws, req):
    if req[0] == "rpca":
        A, E, info = ctx.rpca_solve(req[1], bf16=req[2])
        return (A.clone(), E.clone()), info
    _, m, n, rp, ci, v = req
    U, S, V, info = ctx.mc_solve(m, n, rp, ci, v, opts=blws.default_mc_opts(**MC_OPTS))
    return (U.clone(), S.clone(), V.clone()), info


def submit(srv, blws, req):
    if req[0] == "rpca":
        return srv.submit_rpca(req[1], bf16=req[2])
    _, m, n, rp, ci, v = req
    return srv.submit_mc(m, n, rp, ci, v, opts=blws.default_mc_opts(**MC_OPTS))


@pytest.fixture(scope="module")
def alone(torch, ctx, blws, mix):
    out = [solve_alone(ctx, blws, r) for r in mix]
    torch.cuda.synchronize()
    return out


def same(torch, a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_mix_results_equal_solves_alone(torch, blws, mix, alone):
    srv = blws.Server(0, max_slots=4)
    tickets = [submit(srv, blws, r) for r in mix]
    for t, (ref, ref_info), req in zip(tickets, alone, mix):
        res = srv.wait(t)
        outs, info = res[:-1], res[-1]
        assert info["status"] == ref_info["status"] == 0
        assert info["iters"] == ref_info["iters"] and info["rank"] == ref_info["rank"]
        assert same(torch, outs, ref), req[0]
    st = srv.stats()
    print("server stats", st)
    assert st["completed"] == len(mix) and st["failed"] == 0
    assert st["max_active"] >= 2  # solves overlapped on the device
    # the dense W-products of solves stepping together went out grouped
    assert st["grouped_launches"] > 0 and st["max_group"] >= 2
    assert st["grouped_products"] >= st["grouped_launches"]
    srv.close()


def oracle_ref(req):
    """The oracle's BLWS solve of a request on the values the GPU was given
    (FP32 requests: their FP32-rounded entries, in FP64), with the library's
    reading of the ||D||_2 estimate (at most 8 BLWS steps)."""
    import oracle

    if req[0] == "rpca":
        return oracle.rpca(req[1].double().cpu().numpy(), mode="blws", norm_steps=8)
    _, m, n, rp, ci, v = req
    return oracle.mc(m, n, rp.cpu().numpy(), ci.cpu().numpy(), v.double().cpu().numpy(),
                     mode="blws", norm_steps=8, **MC_OPTS)


def test_served_results_match_oracle(torch, blws, mix):
    """Each request as served (grouped launches, four in flight) against the
    oracle's solve of the same problem. FP64 requests follow the oracle's
    trajectory (same iterations and rank, rounding differences of two FP64
    implementations only); FP32 and BF16-ladder RPCA requests end within the
    FP32 bar of 1e-6 of it. The FP32 MC request (400 x 400, 15% sampled,
    stopped at a relative residual of 1e-6) does not recover its planted rank
    10: 91 values stay above the threshold, the smallest 0.04 against 442, and
    over its 93 iterations FP32 rounding moves those near the threshold; it is
    held to 1e-5, the bar of the other FP32 MC solves stopped at 1e-6."""
    srv = blws.Server(0, max_slots=4)
    tickets = [submit(srv, blws, r) for r in mix]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for i, (req, res) in enumerate(zip(mix, served)):
        ref = oracle_ref(req)
        info = res[-1]
        f64 = (req[1] if req[0] == "rpca" else req[5]).dtype == torch.float64
        if req[0] == "rpca":
            A = res[0].double().cpu().numpy()
            A_or = ref["A"]
            rank_or = ref["info"]["rank"]
        else:
            U, S, V = (x.double().cpu().numpy() for x in res[:3])
            r = info["rank"]
            A = (U[:, :r] * S[:r]) @ V[:, :r].T
            A_or = (ref["U"] * ref["S"]) @ ref["V"].T
            rank_or = ref["rank"]
        err = np.linalg.norm(A - A_or) / np.linalg.norm(A_or)
        print(f"request {i} {req[0]} {tuple(A.shape)} {'f64' if f64 else 'f32'}: iters "
              f"{info['iters']} (oracle {ref['info']['iters']}), rank {info['rank']} "
              f"({rank_or}), |A - A_oracle| / |A_oracle| {err:.2e}", flush=True)
        assert info["status"] == ref["info"]["status"] == 0
        if f64:
            assert info["iters"] == ref["info"]["iters"] and info["rank"] == rank_or
            assert err < 1e-8
        else:
            assert err < (1e-6 if req[0] == "rpca" else 1e-5)


def test_mix_without_grouping_is_the_same(torch, blws, mix, alone):
    # one launch per product instead of grouped launches: the same bits
    srv = blws.Server(0, max_slots=4, group_products=False)
    tickets = [submit(srv, blws, r) for r in mix]
    for t, (ref, _) in zip(tickets, alone):
        assert same(torch, srv.wait(t)[:-1], ref)
    st = srv.stats()
    assert st["grouped_launches"] == 0 and st["completed"] == len(mix)
    srv.close()


def test_memory_budget_serialises_admission(torch, blws, mix, alone):
    # a budget below any single workspace: each request runs alone, in order
    srv = blws.Server(0, max_slots=4, mem_budget=1)
    tickets = [submit(srv, blws, r) for r in mix[:4]]
    for t, (ref, _) in zip(tickets, alone[:4]):
        res = srv.wait(t)
        assert same(torch, res[:-1], ref)
    st = srv.stats()
    assert st["max_active"] == 1 and st["completed"] == 4
    assert st["mem_in_use"] == 0 and st["mem_peak"] > 1
    srv.close()


def test_polling_and_continuous_admission(torch, blws, mix, alone):
    srv = blws.Server(0, max_slots=2)
    pending = {submit(srv, blws, r): i for i, r in enumerate(mix)}
    done = {}
    while pending:
        for t in list(pending):
            res = srv.poll(t)
            if res is not None:
                done[pending.pop(t)] = res
    for i, (ref, _) in enumerate(alone):
        assert same(torch, done[i][:-1], ref)
    st = srv.stats()
    assert st["max_active"] == 2 and st["completed"] == len(mix)
    with pytest.raises(blws.BlwsError):
        srv.poll(next(iter(done)))  # retrieved already
    srv.close()


def test_errors_stay_with_their_request(torch, blws, mix, alone):
    srv = blws.Server(0, max_slots=3)
    good = submit(srv, blws, mix[0])
    _, m, n, rp, ci, v = mix[1]
    bad_ci = ci.clone()
    bad_ci[3] = n + 5
    bad = srv.submit_mc(m, n, rp, bad_ci, v)
    nan_D = mix[6][1].clone()
    nan_D[1, 1] = float("nan")
    bad_nan = srv.submit_rpca(nan_D)
    good2 = submit(srv, blws, mix[7])
    with pytest.raises(blws.BlwsError) as e:
        srv.wait(bad)
    assert e.value.status == -1 and "column" in str(e.value)
    with pytest.raises(blws.BlwsError) as e:
        srv.wait(bad_nan)
    assert e.value.status == -4
    assert same(torch, srv.wait(good)[:-1], alone[0][0])
    assert same(torch, srv.wait(good2)[:-1], alone[7][0])
    st = srv.stats()
    assert st["failed"] == 2 and st["completed"] == 2
    srv.close()


def test_submit_checks_arguments(torch, blws):
    srv = blws.Server(0, max_slots=1)
    D = torch.zeros(1, 5, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        srv.submit_rpca(D)
    assert e.value.status == -1
    D = torch.zeros(8, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        srv.submit_rpca(D, opts=blws.default_alm_opts(b_max=600))
    assert e.value.status == -5
    assert srv.stats()["submitted"] == 0
    srv.close()
