"""GPU tests of the whole-graph window (DI_WINDOW_WHOLE): graphs of at most
DI_SMALL_MAX_NODES nodes solved by one workgroup holding the whole fluid
vector in LDS and running every round itself.  Limit parity against the
oracle for every schedule and both precisions, personalised and weighted
solves, resume (Theorem 1 on the returned state), max_rounds, closed forms,
the size limit, and that it runs in one launch and is an autotuner candidate."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
D = 0.85
WHOLE = -1
SMALL_MAX = 16384


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


@pytest.mark.parametrize("sched,c", [("mean", 1.0), ("mean", 0.0625), ("op2", 0.5),
                                     ("op", 0.25), ("op2", 2.0)])
def test_limit_parity(di, c1, sched, c):
    g, xs = c1
    G = di.Graph(g)
    tune = di.make_tune(sched, c, WHOLE)
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune, timing=True)
    assert st["kernel_launches"] == 1
    assert st["residual_l1"] < 1e-14
    assert _l1(x.cpu().numpy(), xs) <= 1e-12
    assert abs(st["mass_drift"]) < 1e-12
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", tune=tune)
    assert st["residual_l1"] < 1e-8
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6
    assert abs(st["mass_drift"]) < 1e-5


def test_whole_window_is_one_launch_and_an_autotuner_candidate(di):
    g = wl.paper_scenario("S2")
    G = di.Graph(g)
    assert di.window_layout(g.n, di.make_tune("mean", 1.0, WHOLE)) == (WHOLE, False)
    x, st = di.solve(G, d=D, tol=1e-10, precision="fp64", timing=True,
                     tune=di.make_tune("mean", 1.0, WHOLE))
    assert st["kernel_launches"] == 1
    assert _l1(x.cpu().numpy(), oracle.sparse_exact(g, D)[1]) <= st["err_bound_l1"] + 1e-12
    # windows run the windowed kernel, one launch per round
    _, sw = di.solve(G, d=D, tol=1e-10, precision="fp64", timing=True,
                     tune=di.make_tune("mean", 1.0, 11))
    assert sw["kernel_launches"] > 1
    _, trials = di.autotune(G, "solve", d=D, tol=1e-8, precision="fp64")
    whole = [t for t in trials if t["window_log2"] == WHOLE]
    assert len(whole) == 21  # every schedule x c; those past the round cap are discarded
    assert any(t["status"] == 0 for t in whole)


def test_personalised_and_unnormalised(di, c1):
    g, _ = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 4, 100, seed=19)
    for b in range(4):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        Y, xs = oracle.sparse_exact(g, D, v=v)
        x, st = di.solve(G, v=v, d=D, tol=1e-12, precision="fp64",
                         tune=di.make_tune("op2", 0.25, WHOLE))
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12
        y, st = di.solve(G, v=v, d=D, tol=1e-10, precision="fp64", normalize=False,
                         tune=di.make_tune("mean", 1.0, WHOLE))
        gap = Y - y.cpu().numpy()
        assert gap.min() >= -1e-15 and gap.sum() <= st["err_bound_l1"] * (1 + 1e-9) + 1e-15


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-12, 1e-12), ("fp32", 1e-8, 1e-6)])
def test_weighted_graph(di, prec, tol, eps):
    g = wl.random_small(3000, 20000, seed=21, p_dangling=0.15)
    w = wl.random_weights(g, seed=22)
    xs = oracle.dense_exact_weighted(g, w, D)[1]
    G = di.Graph(g, w=w)
    x, st = di.solve(G, d=D, tol=tol, precision=prec, tune=di.make_tune("mean", 1.0, WHOLE))
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + eps


def test_resume_keeps_theorem1(di, c1):
    import torch
    g, xs = c1
    G = di.Graph(g)
    tune = di.make_tune("op", 0.5, WHOLE)
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
                     tune=di.make_tune("mean", 1.0, WHOLE), allow_notconv=True)
    assert st["status"] == di.ENOTCONV and st["rounds"] == 5
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] * (1 + 1e-9)


def test_closed_forms_and_edge_cases(di):
    tune = di.make_tune("mean", 1.0, WHOLE)
    k = 5
    for g, expect in [
        (wl.cycle(7), np.full(7, 1 / 7)),
        (wl.cycle(SMALL_MAX), np.full(SMALL_MAX, 1 / SMALL_MAX)),  # the largest graph it holds
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
    # one node more than the window holds
    big = di.Graph(wl.cycle(SMALL_MAX + 1))
    with pytest.raises(di.DiError) as e:
        di.solve(big, d=D, tol=1e-8, tune=tune)
    assert e.value.status == di.EINVAL
    with pytest.raises(di.DiError):
        di.window_layout(SMALL_MAX + 1, tune)
