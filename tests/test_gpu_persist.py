"""GPU tests of the one-launch solve (di_tune.persist): one cooperative launch
runs every round, each window's state held in its workgroup's LDS, rounds
separated by a grid barrier.  Limit parity against the oracle for every
schedule and both precisions at every window size it takes (ragged last
windows included), personalised, unnormalised and weighted solves, resume
(Theorem 1 on the returned state), max_rounds, closed forms and degenerate
graphs, the same rounds as the launch-per-round path, the size limit, and
the barrier's time-out path (forced from the host).  The frontier replay and the score rule of every round are checked in
test_gpu_trace.py."""
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


@pytest.fixture(scope="module")
def c1():
    g = wl.recipe("pagerank-10k")
    return g, oracle.sparse_exact(g, D)[1]


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


@pytest.mark.parametrize("sched,c,win", [("mean", 1.0, 8), ("mean", 0.0625, 9), ("op2", 0.5, 8),
                                         ("op", 0.25, 10), ("op2", 0.03125, 11)])
def test_limit_parity(di, c1, sched, c, win):
    g, xs = c1  # 10^4 nodes: 40 / 20 / 10 / 5 windows, the last one ragged
    G = di.Graph(g)
    tune = di.make_tune(sched, c, win, persist=True)
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune, timing=True)
    assert st["kernel_launches"] == 1
    assert st["residual_l1"] < 1e-14
    assert _l1(x.cpu().numpy(), xs) <= 1e-12
    assert abs(st["mass_drift"]) < 1e-12
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", tune=tune)
    assert st["residual_l1"] < 1e-8
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6
    assert abs(st["mass_drift"]) < 1e-5


@pytest.mark.parametrize("sched,c", [("mean", 1.0), ("op2", 0.125), ("op", 0.0625)])
def test_same_rounds_as_one_launch_per_round(di, c1, sched, c):
    """Round r of the one-launch solve computes what launch r of the windowed
    path computes: same thresholds, same stop, so the same rounds and links
    (up to the order of fp64 additions, which may move a node across θ)."""
    g, _ = c1
    G = di.Graph(g)
    _, sp = di.solve(G, d=D, tol=1e-10, precision="fp64",
                     tune=di.make_tune(sched, c, 8, persist=True))
    _, sw = di.solve(G, d=D, tol=1e-10, precision="fp64", tune=di.make_tune(sched, c, 8))
    assert abs(sp["rounds"] - sw["rounds"]) <= 1
    assert abs(sp["edges_diffused"] - sw["edges_diffused"]) <= 0.01 * sw["edges_diffused"]


def test_personalised_and_unnormalised(di, c1):
    g, _ = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 4, 100, seed=19)
    for b in range(4):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        Y, xs = oracle.sparse_exact(g, D, v=v)
        x, st = di.solve(G, v=v, d=D, tol=1e-12, precision="fp64",
                         tune=di.make_tune("op2", 0.25, persist=True))
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12
        y, st = di.solve(G, v=v, d=D, tol=1e-10, precision="fp64", normalize=False,
                         tune=di.make_tune("mean", 1.0, persist=True))
        gap = Y - y.cpu().numpy()
        assert gap.min() >= -1e-15 and gap.sum() <= st["err_bound_l1"] * (1 + 1e-9) + 1e-15


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-12, 1e-12), ("fp32", 1e-8, 1e-6)])
def test_weighted_graph(di, prec, tol, eps):
    g = wl.random_small(3000, 20000, seed=21, p_dangling=0.15)
    w = wl.random_weights(g, seed=22)
    xs = oracle.dense_exact_weighted(g, w, D)[1]
    G = di.Graph(g, w=w)
    x, st = di.solve(G, d=D, tol=tol, precision=prec, tune=di.make_tune("op", 0.5, persist=True))
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + eps


def test_resume_keeps_theorem1(di, c1):
    import torch
    g, xs = c1
    G = di.Graph(g)
    tune = di.make_tune("op", 0.5, persist=True)
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float64, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    di.solve(G, d=D, tol=1e-4, precision="fp64", state=(F, H), tune=tune)
    x, st = di.solve(G, d=D, tol=1e-11, precision="fp64", state=(F, H), tune=tune)
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy()
    src, dst = g.edges()
    PH = np.bincount(dst, weights=Hn[src] / g.outdeg[src], minlength=g.n)
    np.testing.assert_allclose(Hn + Fn, (1 - D) / g.n + D * PH, rtol=1e-11, atol=1e-18)


def test_max_rounds(di, c1):
    g, xs = c1
    x, st = di.solve(di.Graph(g), d=D, tol=1e-12, precision="fp64", max_rounds=5,
                     tune=di.make_tune("mean", 1.0, persist=True), allow_notconv=True)
    assert st["status"] == di.ENOTCONV and st["rounds"] == 5
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] * (1 + 1e-9)


def test_closed_forms_and_edge_cases(di):
    tune = di.make_tune("mean", 1.0, persist=True)
    k = 5
    n_max = 128 * 2048  # the most nodes it takes: 128 windows of 2^11
    for g, expect in [
        (wl.cycle(7), np.full(7, 1 / 7)),
        (wl.cycle(n_max), np.full(n_max, 1 / n_max)),
        (wl.in_star(k), np.r_[(1 + D * k) / (k + 1 + D * k), np.full(k, 1 / (k + 1 + D * k))]),
        (wl.out_star(k), np.r_[1 / (k + 1 + D), np.full(k, (1 + D / k) / (k + 1 + D))]),
        (wl.from_edges(40, np.array([], np.int64), np.array([], np.int64)), np.full(40, 1 / 40)),
        (wl.from_edges(1, np.array([0]), np.array([0])), np.array([1.0])),
    ]:
        G = di.Graph(g)
        x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune)
        assert _l1(x.cpu().numpy(), expect) <= 1e-12, g.name
    # multigraph with self-loops and dangling nodes, against the dense limit
    g = wl.random_small(700, 5000, seed=5, p_dangling=0.3)
    x, st = di.solve(di.Graph(g), d=D, tol=1e-14, precision="fp64", tune=tune)
    assert _l1(x.cpu().numpy(), oracle.dense_exact(g, D)[1]) <= 1e-12
    # one node more than 128 windows of 2^11 hold, and the whole-graph window
    big = di.Graph(wl.cycle(n_max + 1))
    with pytest.raises(di.DiError) as e:
        di.solve(big, d=D, tol=1e-8, tune=tune)
    assert e.value.status == di.EINVAL
    with pytest.raises(di.DiError) as e:
        di.solve(di.Graph(wl.cycle(7)), d=D, tol=1e-8, tune=di.make_tune("mean", 1.0, -1, persist=True))
    assert e.value.status == di.EINVAL


def test_hub_window_reads_links_from_global_memory(di):
    """A window with more out-links than its LDS link cache holds (24576)
    reads them from global memory; the result is the same limit."""
    n = 4000
    src = np.r_[np.zeros(30000, np.int64), np.arange(1, n, dtype=np.int64)]
    rng = np.random.default_rng(7)
    dst = np.r_[rng.integers(0, n, 30000), rng.integers(0, n, n - 1)]
    g = wl.from_edges(n, src, dst)
    G = di.Graph(g)
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=di.make_tune("op2", 0.5, 8, persist=True))
    assert _l1(x.cpu().numpy(), oracle.sparse_exact(g, D)[1]) <= 1e-12


def test_barrier_wait_limit_ends_the_solve_cleanly(di, c1):
    """The failure path of the grid barrier, forced from the host: with a wait
    limit of 0 a workgroup that finds the others not yet arrived ends the
    solve, every workgroup leaves its loop (the call returns), and the status
    is DI_EDEVICE; the next solve, at the default limit, is exact again."""
    g, xs = c1
    G = di.Graph(g)
    tune = di.make_tune("mean", 1.0, persist=True)
    di.set_persist_wait(0.0)
    try:
        with pytest.raises(di.DiError) as e:
            di.solve(G, d=D, tol=1e-10, precision="fp64", tune=tune)
        assert e.value.status == di.EDEVICE and "barrier" in e.value.message
    finally:
        di.set_persist_wait(2.0)
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune)
    assert _l1(x.cpu().numpy(), xs) <= 1e-12
