"""Frontier replay: a traced GPU solve records the set S_r every round takes;
the oracle diffuses exactly those sets, in order, in fp64 from the same start.
The final states must agree (1e-12 for fp64 fluid, 1e-6 for fp32) -- a check
of every round of a whole solve, independent of the threshold schedule, so a
wrong push, a lost record or a missed fold in any round shows up here."""
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


@pytest.mark.parametrize("gname,prec,tol,sched", [
    ("pagerank-10k", "fp64", 1e-10, "mean"),
    ("pagerank-10k", "fp32", 1e-8, "mean"),
    ("pagerank-10k", "fp64", 1e-10, "op"),
    ("rand", "fp64", 1e-10, "op2"),
])
def test_replay_of_recorded_sets(di, gname, prec, tol, sched):
    import torch
    g = wl.recipe(gname) if gname != "rand" else wl.random_small(5000, 40000, seed=41, p_dangling=0.2)
    G = di.Graph(g)
    dt = torch.float64 if prec == "fp64" else torch.float32
    F = torch.full((g.n,), (1 - D) / g.n, dtype=dt, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    F0 = F.cpu().numpy().astype(np.float64)
    trace = torch.zeros((400, g.n), dtype=torch.uint8, device="cuda")
    _, st = di.solve(G, d=D, tol=tol, precision=prec, state=(F, H), trace=trace,
                     tune=di.make_tune(sched, 1.0))
    rounds = st["rounds"]
    assert 0 < rounds <= 400
    sets = trace[:rounds].cpu().numpy().astype(bool)
    assert not trace[rounds:].any().item()
    Fo, Ho = F0, np.zeros(g.n)
    for r in range(rounds):
        Fo, Ho = oracle.apply_set(g, D, sets[r], Fo, Ho)
    Fg, Hg = F.cpu().numpy().astype(np.float64), H.cpu().numpy()
    eps = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(Hg - Ho).sum() <= eps
    assert np.abs(Fg - Fo).sum() <= eps
    # the recorded sets follow the rule: a taken node held fluid when taken
    assert sets.sum() == st["nodes_diffused"]
