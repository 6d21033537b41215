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


def _tune(di, sched, c, win):
    """Windows of the default size (0), the whole-graph window (-1), or the
    one-launch solve ("persist") at the default window."""
    if win == "persist":
        return di.make_tune(sched, c, persist=True)
    return di.make_tune(sched, c, window_log2=win)


@pytest.mark.parametrize("gname,prec,tol,sched", [
    ("pagerank-10k", "fp64", 1e-10, "mean"),
    ("pagerank-10k", "fp32", 1e-8, "mean"),
    ("pagerank-10k", "fp64", 1e-10, "op"),
    ("rand", "fp64", 1e-10, "op2"),
])
@pytest.mark.parametrize("win", [0, -1, "persist"], ids=["windows", "whole", "persist"])
def test_replay_of_recorded_sets(di, gname, prec, tol, sched, win):
    import torch
    g = wl.recipe(gname) if gname != "rand" else wl.random_small(5000, 40000, seed=41, p_dangling=0.2)
    G = di.Graph(g)
    dt = torch.float64 if prec == "fp64" else torch.float32
    F = torch.full((g.n,), (1 - D) / g.n, dtype=dt, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    F0 = F.cpu().numpy().astype(np.float64)
    trace = torch.zeros((400, g.n), dtype=torch.uint8, device="cuda")
    _, st = di.solve(G, d=D, tol=tol, precision=prec, state=(F, H), trace=trace,
                     tune=_tune(di, sched, 1.0, win))
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


def _score(sched, F, outdeg, indeg):
    """The selection scores of Section 4.3 (ALGO-OP: F_i/((#in_i+1)(#out_i+1)),
    ALGO-OP2: F_i/(#out_i+1)) and of the plain threshold variant (F_i), written
    out here from the paper, independent of the library and of the oracle."""
    a = np.abs(F)
    if sched == "op":
        return a / ((indeg + 1.0) * (outdeg + 1.0))
    if sched == "op2":
        return a / (outdeg + 1.0)
    return a


@pytest.mark.parametrize("gname,sched,c", [
    ("pagerank-10k", "op", 1.0),
    ("pagerank-10k", "op2", 1.0),
    ("pagerank-10k", "op", 1.0 / 16),
    ("pagerank-10k", "op2", 1.0 / 32),
    ("pagerank-10k", "mean", 0.25),
    ("rand", "op", 1.0),
    ("rand", "op2", 0.5),
])
@pytest.mark.parametrize("win", [0, -1, "persist"], ids=["windows", "whole", "persist"])
def test_every_round_takes_the_top_of_its_score(di, gname, sched, c, win):
    """Every round of a traced fp64 solve takes an upper set of the schedule's
    score: on the oracle's replay of the recorded sets, each round's lowest
    taken score is at least the highest score of the nodes it left holding
    fluid.  A slip in the device's OP / OP2 weights (a sum for OP's product,
    #in for OP2's #out) breaks this on graphs whose degrees vary."""
    import torch
    g = wl.recipe(gname) if gname != "rand" else wl.random_small(5000, 40000, seed=43, p_dangling=0.2)
    G = di.Graph(g)
    outdeg = g.outdeg.astype(np.float64)
    indeg = np.bincount(g.col_idx, minlength=g.n).astype(np.float64)
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float64, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    F0 = F.cpu().numpy()
    trace = torch.zeros((600, g.n), dtype=torch.uint8, device="cuda")
    _, st = di.solve(G, d=D, tol=1e-10, precision="fp64", state=(F, H), trace=trace,
                     tune=_tune(di, sched, c, win))
    rounds = st["rounds"]
    assert 0 < rounds <= 600
    sets = trace[:rounds].cpu().numpy().astype(bool)
    Fo, Ho = F0, np.zeros(g.n)
    checked = 0
    for r in range(rounds):
        S = sets[r]
        assert np.all(Fo[S] != 0.0), r  # a taken node holds fluid
        sc = _score(sched, Fo, outdeg, indeg)
        left = (~S) & (Fo != 0.0)
        if S.any() and left.any():
            lo, hi = sc[S].min(), sc[left].max()
            assert lo >= hi * (1.0 - 1e-9), (r, lo, hi)
            checked += 1
        Fo, Ho = oracle.apply_set(g, D, S, Fo, Ho)
    assert checked >= rounds // 2
