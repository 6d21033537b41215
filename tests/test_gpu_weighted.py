"""GPU parity on weighted graphs (P with arbitrary non-negative column weights
summing to one, Section 2.1): one round against the oracle's weighted set
step, full solves, the power iteration and personalised batches against the
oracle's dense weighted limit."""
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
def wg():
    g = wl.random_small(3000, 20000, seed=21, p_dangling=0.15)
    w = wl.random_weights(g, seed=22)
    return g, w, oracle.dense_exact_weighted(g, w, D)[1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_weighted_round_matches_oracle(di, wg, prec):
    import torch
    g, w, _ = wg
    G = di.Graph(g, w=w)
    F, H = wl.random_fluid(g.n, seed=23)
    dt = torch.float32 if prec == "fp32" else torch.float64
    Ft = torch.tensor(F, dtype=dt, device="cuda")
    Ht = torch.tensor(H, dtype=torch.float64, device="cuda")
    F64 = Ft.cpu().numpy().astype(np.float64)
    theta = float(np.quantile(F64[F64 > 0], 0.5))
    di.diffuse_round(G, Ft, Ht, theta, d=D)
    Fo, Ho, S = oracle.set_step_weighted(g, w, D, theta, F64, H)
    assert np.array_equal(Ht.cpu().numpy(), Ho)
    src, dst = g.edges()
    push = np.abs(np.where(S[src], D * F64[src] * w, 0.0))
    k = np.bincount(dst, weights=(push > 0).astype(float), minlength=g.n)
    mag = np.abs(np.where(S, 0.0, F64)) + np.bincount(dst, weights=push, minlength=g.n)
    eps = 2.0 ** -24 if prec == "fp32" else 2.0 ** -53
    # the weighted share d*F_i*w_e: one more rounding than the 1/deg share
    assert np.all(np.abs(Ft.cpu().numpy().astype(np.float64) - Fo) <= (k + 3) * 2 * eps * mag + 1e-300)


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-12, 1e-12), ("fp32", 1e-8, 1e-6)])
def test_weighted_solve_and_power_match_dense_limit(di, wg, prec, tol, eps):
    g, w, xs = wg
    G = di.Graph(g, w=w)
    x, st = di.solve(G, d=D, tol=tol, precision=prec)
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + eps
    xp, sp = di.power_solve(G, d=D, tol=tol, precision=prec)
    assert float(np.abs(xp.cpu().numpy() - xs).sum()) <= sp["err_bound_l1"] + eps


def test_weighted_batch_matches_dense_limit(di, wg):
    g, w, _ = wg
    G = di.Graph(g, w=w)
    ptr, seeds = wl.ppr_seed_sets(g.n, 4, 50, seed=24)
    x, st = di.solve_batch(G, ptr, seeds, d=D, tol=1e-12, precision="fp64")
    for b in range(4):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.dense_exact_weighted(g, w, D, v)[1]
        assert float(np.abs(x[b].cpu().numpy() - xs).sum()) <= st[b]["err_bound_l1"] + 1e-12


def test_weighted_server_matches_dense_limit(di, wg):
    """Served PPR on the weighted graph: the top-k values within the reported
    bound of the oracle's dense weighted PPR vector, in rank order."""
    g, w, _ = wg
    G = di.Graph(g, w=w)
    srv = di.Server(hbm_budget_bytes=2 << 30, max_slots=4, topk=20, precision="fp64")
    gid = srv.add_graph(G)
    rng = np.random.default_rng(25)
    reqs = []
    for s in (1, 7, 60):
        seeds = np.sort(rng.choice(g.n, s, replace=False)).astype(np.int32)
        reqs.append((seeds, srv.submit(gid, seeds, d=D, tol=1e-12)))
    for seeds, rid in reqs:
        r = srv.wait(rid, 60.0)
        assert r is not None and r["status"] == 0 and r["residual_l1"] < 1e-12
        xs = oracle.dense_exact_weighted(g, w, D, wl.seed_vector(g.n, seeds))[1]
        ids, vals = r["top_ids"], r["top_x"]
        assert np.all(np.diff(vals) <= 0)
        assert np.all(np.abs(vals - xs[ids]) <= r["err_bound_l1"] + 1e-12)
        assert np.sort(xs)[::-1][len(ids) - 1] <= vals[-1] + 2 * (r["err_bound_l1"] + 1e-12)
    srv.close()


def test_weighted_update_of_link_weights(di, wg):
    """A change of the link weights of 5% of the rows, same links (Section 3.2
    with P' from the new weights): the injected fluid against the oracle's
    F + d(P'-P)H on the dense weighted matrices, then the resumed solve
    against the dense weighted limit of P'."""
    import torch
    g, w0, _ = wg
    rng = np.random.default_rng(26)
    w1 = w0.copy()
    deg = np.diff(g.row_ptr)
    rows = rng.choice(np.flatnonzero(deg > 1), size=int(0.05 * g.n), replace=False)
    w_new = wl.random_weights(g, seed=27)
    for i in rows:
        w1[g.row_ptr[i]:g.row_ptr[i + 1]] = w_new[g.row_ptr[i]:g.row_ptr[i + 1]]
    G0, G1 = di.Graph(g, w=w0), di.Graph(g, w=w1)
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float64, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    di.solve(G0, d=D, tol=1e-5, precision="fp64", state=(F, H))
    F0, H0 = F.cpu().numpy(), H.cpu().numpy()
    di.inject_update(G0, G1, F, H, d=D)
    P0 = oracle.transition_dense_weighted(g, w0)
    P1 = oracle.transition_dense_weighted(g, w1)
    ref = F0 + D * (P1 @ H0) - D * (P0 @ H0)
    mag = np.abs(F0) + D * (P1 @ np.abs(H0)) + D * (P0 @ np.abs(H0))
    assert np.all(np.abs(F.cpu().numpy() - ref) <= 8 * 2.0 ** -53 * mag + 1e-300)
    assert (ref < 0).any()
    x, st = di.solve(G1, d=D, tol=1e-12, precision="fp64", state=(F, H))
    xs = oracle.dense_exact_weighted(g, w1, D)[1]
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + 1e-12
