"""Graph replay of robust-PCA iterations (blws_alm_opts.graph): once the block
width holds, one iteration (products, Ritz step, epilogue, readback) is
captured into a HIP graph and replayed with the iteration's changing values
(eps, mu, mu', stream-id bases) copied in from pinned host memory at the
start of every replay. Every replay must compute what the eager launches
compute: whole solves with and without graphs are compared bit for bit, with
eager solves (and their synchronisations) run between graph solves, and each
graph solve holds many replays. The solve is also held to the oracle."""

import numpy as np
import pytest

import oracle
import synth

# Withdrawn: the first GPU run of a captured solve (default test order, the
# FP64 case) ended the process with a host segmentation fault inside the
# solve call. Reading the capture path did not show a cause (every fork of the
# second stream joined before the capture ends, no synchronous or allocating
# call while capturing, the pinned parameter block and readback area live),
# so graph replay is not part of the library and these tests stay skipped
# until a cause is found and fixed.
pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="graph replay withdrawn: its first captured solve crashed the host "
                            "process and no cause was found in the code"),
]


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


@pytest.fixture(scope="module")
def inst():
    return synth.rpca_instance(420, 380, 20, 0.08, 100.0, 11)


@pytest.mark.parametrize("dtype,bf16", [("f64", False), ("f32", False), ("f32", True)])
def test_graph_solves_equal_eager_solves(torch, blws, ctx, inst, dtype, bf16):
    D = torch.tensor(inst["D"], dtype=torch.float64 if dtype == "f64" else torch.float32,
                     device="cuda")
    eager = ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=0), bf16=bf16)
    torch.cuda.synchronize()
    for rep in range(2):  # a new capture per solve, eager work in between
        A, E, info = ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=1), bf16=bf16)
        torch.cuda.synchronize()
        print(f"{dtype} bf16={bf16} rep {rep}: iters {info['iters']}, replays "
              f"{info['graph_replays']}, captures {info['graph_captures']}", flush=True)
        assert eager[2]["graph_replays"] == 0 and eager[2]["graph_captures"] == 0
        assert info["graph_captures"] >= 1 and info["graph_replays"] >= 5
        assert info["status"] == eager[2]["status"] == 0
        assert info["iters"] == eager[2]["iters"] and info["rank"] == eager[2]["rank"]
        assert info["fallbacks"] == eager[2]["fallbacks"]
        assert torch.equal(A, eager[0]) and torch.equal(E, eager[1])
        ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=0), bf16=bf16)
        torch.cuda.synchronize()


def test_graph_solve_matches_oracle(torch, blws, ctx, inst):
    bl = oracle.rpca(inst["D"], mode="blws", norm_steps=8)
    D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
    A, E, info = ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=1))
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    assert info["graph_replays"] > 0
    assert info["iters"] == bl["info"]["iters"] and info["rank"] == bl["info"]["rank"]
    assert np.linalg.norm(A - bl["A"]) <= 1e-8 * np.linalg.norm(bl["A"])


def test_no_graphs_while_timing(torch, blws, ctx, inst):
    D = torch.tensor(inst["D"], dtype=torch.float64, device="cuda")
    ctx.timing(True)
    try:
        _, _, info = ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=1))
        torch.cuda.synchronize()
    finally:
        ctx.timing(False)
    assert info["graph_replays"] == 0 and info["graph_captures"] == 0


def test_graph_option_checked(torch, blws, ctx, inst):
    D = torch.tensor(inst["D"][:64, :64], dtype=torch.float64, device="cuda")
    with pytest.raises(blws.BlwsError) as e:
        ctx.rpca_solve(D, opts=blws.default_alm_opts(graph=2))
    assert e.value.status == -1
