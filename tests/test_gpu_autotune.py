"""GPU tests of the autotuner (di_autotune): it times every schedule x
threshold factor at the default window plus the neighbouring windows, picks
the fastest converged candidate, caches it in the graph, and solves that
later pass no tune use it and still meet their error bounds against the
oracle."""
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


def test_autotune_solve_picks_fastest_and_caches(di):
    g = wl.recipe("pagerank-10k")
    G = di.Graph(g)
    best, trials = di.autotune(G, "solve", d=D, tol=1e-10, precision="fp64")
    ok = [t for t in trials if t["status"] == 0]
    assert len(trials) >= 15 and len(ok) >= 1
    assert {t["schedule"] for t in trials} == {"mean", "op2", "op"}
    fastest = min(ok, key=lambda t: t["seconds"])
    assert di.tune_dict(best) == {k: fastest[k] for k in ("schedule", "c", "window_log2",
                                                          "check_every", "threads", "tables",
                                                          "persist")}
    assert {t["threads"] for t in trials} == {0, 1024}
    # a 40-window graph: the one-launch solve is a candidate at every
    # schedule x threshold factor
    assert sum(t["persist"] for t in trials) >= 21
    # a solve that passes no tune uses the cached knobs: same rounds as the
    # explicit winner, and the result within its bound of the exact limit
    xs = oracle.sparse_exact(g, D)[1]
    x0, s0 = di.solve(G, d=D, tol=1e-10, precision="fp64")
    x1, s1 = di.solve(G, d=D, tol=1e-10, precision="fp64", tune=best)
    assert abs(s0["rounds"] - s1["rounds"]) <= 1
    for x, s in [(x0, s0), (x1, s1)]:
        assert float(np.abs(x.cpu().numpy() - xs).sum()) <= s["err_bound_l1"] + 1e-12


def test_autotune_batch_then_batch_solves_meet_bounds(di):
    g = wl.recipe("pagerank-10k")
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 16, 100, seed=21)
    best, trials = di.autotune(G, "batch", d=D, tol=1e-6, precision="fp32", seed_ptr=ptr,
                               seeds=seeds)
    assert any(t["status"] == 0 for t in trials)
    x, st = di.solve_batch(G, ptr, seeds, d=D, tol=1e-6, precision="fp32")
    for b in [0, 7, 15]:
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.limit(g, D, v, tol=1e-14)
        assert st[b]["residual_l1"] < 1e-6
        assert float(np.abs(x[b].cpu().numpy() - xs).sum()) <= st[b]["err_bound_l1"] + 1e-6


def test_autotune_discards_candidates_that_do_not_converge(di):
    g = wl.recipe("pagerank-10k")
    G = di.Graph(g)
    with pytest.raises(di.DiError) as e:
        di.autotune(G, "solve", d=D, tol=1e-10, precision="fp64", max_rounds=3)
    assert e.value.status == di.ENOTCONV


def test_autotune_batch_needs_seed_sets(di):
    G = di.Graph(wl.recipe("pagerank-10k"))
    with pytest.raises(di.DiError) as e:
        di.autotune(G, "batch", d=D, tol=1e-6, seed_ptr=np.array([0], np.int64),
                    seeds=np.array([], np.int32))
    assert e.value.status == di.EINVAL
