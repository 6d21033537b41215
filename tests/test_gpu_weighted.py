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
