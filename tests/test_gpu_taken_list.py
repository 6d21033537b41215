"""The round kernel's two ways of expanding a window's taken nodes: a list of
them in node order (the default, whenever LDS has room for it), and passes
over 1024 consecutive nodes (the fallback for graphs near the size limit,
forced here with the di_set_taken_list switch).  Both must diffuse exactly
the recorded sets: a traced solve is replayed set by set by the oracle from
the same start, on windows of 4096 nodes where early rounds take more than
a pass of nodes per window, and the solve must reach the oracle's limit
within its bound."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
D = 0.85


@pytest.fixture(scope="module")
def di():
    import torch
    from paper_1202_6158_amd import di as _di
    torch.cuda.set_device(0)
    return _di


@pytest.fixture(params=[True, False], ids=["list", "passes"])
def listing(di, request):
    di.set_taken_list(request.param)
    yield request.param
    di.set_taken_list(True)


@pytest.fixture(scope="module")
def graph():
    return wl.random_small(20000, 160000, seed=61, p_dangling=0.15)


@pytest.mark.parametrize("prec,sched,threads", [
    ("fp64", "mean", 1024),
    ("fp32", "op2", 512),
    ("fp64", "op", 512),
])
def test_replay_with_and_without_the_list(di, listing, graph, prec, sched, threads):
    import torch
    g = graph
    G = di.Graph(g)
    dt = torch.float64 if prec == "fp64" else torch.float32
    F = torch.full((g.n,), (1 - D) / g.n, dtype=dt, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    F0 = F.cpu().numpy().astype(np.float64)
    trace = torch.zeros((400, g.n), dtype=torch.uint8, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-8
    _, st = di.solve(G, d=D, tol=tol, precision=prec, state=(F, H), trace=trace,
                     tune=di.make_tune(sched, 1.0, window_log2=12, threads=threads))
    rounds = st["rounds"]
    assert 0 < rounds <= 400
    sets = trace[:rounds].cpu().numpy().astype(bool)
    # some round takes more than one pass of nodes in every full window
    full = (g.n // 4096) * 4096
    per_window = sets[:, :full].reshape(rounds, -1, 4096).sum(axis=2)
    assert per_window.min(axis=1).max() > 1024
    Fo, Ho = F0, np.zeros(g.n)
    for r in range(rounds):
        Fo, Ho = oracle.apply_set(g, D, sets[r], Fo, Ho)
    Fg, Hg = F.cpu().numpy().astype(np.float64), H.cpu().numpy()
    eps = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(Hg - Ho).sum() <= eps
    assert np.abs(Fg - Fo).sum() <= eps
    assert sets.sum() == st["nodes_diffused"]


@pytest.fixture(scope="module")
def limit(graph):
    return oracle.limit(graph, D, tol=1e-14)


def test_limit_with_and_without_the_list(di, listing, graph, limit):
    g, xs = graph, limit
    G = di.Graph(g)
    x, st = di.solve(G, d=D, tol=1e-12, precision="fp64",
                     tune=di.make_tune("op2", 0.125, window_log2=12, threads=1024))
    assert st["residual_l1"] < 1e-12
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + 1e-12
