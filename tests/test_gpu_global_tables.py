"""The round kernel with its per-window segment tables read from global memory
(the layout for graphs with more windows than LDS can hold): forced on the
10k-node graph for limit parity against the oracle (every schedule, fp64 and
fp32 fluid, several window sizes, batches and the server), and chosen by
itself on a 3*10^7-node graph, beyond the LDS-table layout, where Theorem 1 on
the device state and agreement with the power iteration are checked."""
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


@pytest.mark.parametrize("sched", ["mean", "op2", "op"])
@pytest.mark.parametrize("wlog", [8, 13])
def test_forced_global_tables_limit_parity(di, c1, sched, wlog):
    g, xs = c1
    G = di.Graph(g)
    tune = di.make_tune(sched, 0.5, wlog, tables="global")
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune)
    assert _l1(x.cpu().numpy(), xs) <= 1e-12
    assert abs(st["mass_drift"]) < 1e-12
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", tune=tune)
    assert st["residual_l1"] < 1e-8
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6


def test_forced_global_tables_same_rounds_as_lds_tables(di, c1):
    """Same decisions either way: the two layouts only move where the segment
    tables are read from, so an fp64 solve takes the same rounds and links."""
    g, _ = c1
    G = di.Graph(g)
    _, a = di.solve(G, d=D, tol=1e-12, precision="fp64",
                    tune=di.make_tune("op2", 0.25, 9, threads=1024, tables="lds"))
    _, b = di.solve(G, d=D, tol=1e-12, precision="fp64",
                    tune=di.make_tune("op2", 0.25, 9, threads=1024, tables="global"))
    assert abs(a["rounds"] - b["rounds"]) <= 1
    assert abs(a["edges_diffused"] - b["edges_diffused"]) <= 0.01 * a["edges_diffused"]


def test_forced_global_tables_batch_and_server(di, c1):
    g, _ = c1
    G = di.Graph(g)
    tune = di.make_tune("op2", 0.125, 10, tables="global")
    ptr, seeds = wl.ppr_seed_sets(g.n, 6, 100, seed=51)
    x, st = di.solve_batch(G, ptr, seeds, d=D, tol=1e-11, precision="fp64", tune=tune)
    for b in range(6):
        xs = oracle.limit(g, D, wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]]), tol=1e-14)
        assert _l1(x[b].cpu().numpy(), xs) <= st[b]["err_bound_l1"] + 1e-12, b
    srv = di.Server(hbm_budget_bytes=2 << 30, max_slots=4, topk=20, precision="fp64", tune=tune)
    gid = srv.add_graph(G)
    rids = [(seeds[ptr[b]:ptr[b + 1]], srv.submit(gid, seeds[ptr[b]:ptr[b + 1]], d=D, tol=1e-12))
            for b in range(3)]
    for ss, rid in rids:
        r = srv.wait(rid, 60.0)
        assert r is not None and r["status"] == 0
        xs = oracle.limit(g, D, wl.seed_vector(g.n, ss), tol=1e-14)
        assert np.all(np.abs(r["top_x"] - xs[r["top_ids"]]) <= r["err_bound_l1"] + 1e-12)
    srv.close()


def test_tables_knob_is_validated(di, c1):
    g, _ = c1
    G = di.Graph(g)
    with pytest.raises(di.DiError) as e:
        di.solve(G, d=D, tol=1e-8, tune=di.make_tune("mean", 1.0, tables=3))
    assert e.value.status == di.EINVAL


@pytest.fixture(scope="module")
def big(di):
    import time
    t0 = time.time()
    g = wl.powerlaw(n=30_000_000, mean=5.0, dangling=0.10, kmax=1000, seed=61, name="powerlaw-30m")
    print("\npowerlaw-30m: %d nodes, %d links generated in %.0f s" % (g.n, g.m, time.time() - t0),
          flush=True)
    G = di.Graph(g)
    print("powerlaw-30m: resident on the device after %.0f s" % (time.time() - t0), flush=True)
    return g, G


@pytest.mark.timeout(900)
def test_30m_nodes_beyond_lds_tables(di, big):
    """3*10^7 nodes need 3663 windows of 2^13 nodes, more than the LDS-table
    layout holds: the library picks global tables by itself.  Theorem 1 on
    every node of the returned state, the stop, and agreement with the GPU
    power iteration within both bounds."""
    import torch
    g, G = big
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float32, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", state=(F, H))
    print("30m: %d rounds, %.1f ms, %.3g links" % (st["rounds"], 1e3 * st["seconds"],
                                                  st["edges_diffused"]), flush=True)
    assert st["residual_l1"] < 1e-8
    assert abs(st["mass_drift"]) < 1e-5
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n, dtype=np.int32), deg)
    PH = np.bincount(g.col_idx, weights=Hn[src] / deg[src], minlength=g.n)
    del src
    assert np.abs(Hn + Fn - ((1 - D) / g.n + D * PH)).sum() < 1e-6
    xp, sp = di.power_solve(G, d=D, tol=1e-8, precision="fp64")
    assert _l1(x.cpu().numpy(), xp.cpu().numpy()) <= st["err_bound_l1"] + sp["err_bound_l1"] + 1e-6
    # the LDS-table layout cannot hold this graph
    with pytest.raises(di.DiError) as e:
        di.solve(G, d=D, tol=1e-8, tune=di.make_tune("mean", 1.0, tables="lds"))
    assert e.value.status == di.EINVAL
