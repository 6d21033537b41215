"""GPU tests of the graph update (updating equation, Section 3.2): the fluid
injection F += d(P'-P)H against the oracle's, one round on signed fluid
against the oracle's signed set step, and the full flow -- solve on P, change
the graph, inject, resume on P' -- against the exact limit of P' (Theorem 4),
with less work than a fresh solve."""
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
def pair():
    g0 = wl.recipe("pagerank-10k")
    return g0, wl.modify_graph(g0, 0.01, seed=77)


def _state(di, G, g, prec, tol):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    F = torch.full((g.n,), (1 - D) / g.n, dtype=dt, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    di.solve(G, d=D, tol=tol, precision=prec, state=(F, H))
    return F, H


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inject_matches_oracle(di, pair, prec):
    g0, g1 = pair
    G0, G1 = di.Graph(g0), di.Graph(g1)
    F, H = _state(di, G0, g0, prec, 1e-5)
    F0, H0 = F.cpu().numpy().astype(np.float64), H.cpu().numpy()
    di.inject_update(G0, G1, F, H, d=D)
    ref = oracle.inject_update(g0, g1, D, F0, H0)
    got = F.cpu().numpy().astype(np.float64)
    # rounding bound of the fp64 sums: a few ulps of the magnitudes summed
    mag = np.abs(F0) + D * (oracle.transition_sparse(g1) @ np.abs(H0)) \
        + D * (oracle.transition_sparse(g0) @ np.abs(H0))
    slack = 8 * 2.0 ** -53 * mag + 1e-300
    if prec == "fp64":
        assert np.all(np.abs(got - ref) <= slack)
    else:  # plus one rounding of the fp64 value into fp32
        assert np.all(np.abs(got - ref) <= np.spacing(np.abs(ref).astype(np.float32)) + slack)
    assert (ref < 0).any()  # the injection mixes signs
    assert np.array_equal(H.cpu().numpy(), H0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_round_on_signed_fluid_matches_oracle(di, pair, prec):
    import torch
    g0, g1 = pair
    G0, G1 = di.Graph(g0), di.Graph(g1)
    F, H = _state(di, G0, g0, prec, 1e-5)
    di.inject_update(G0, G1, F, H, d=D)
    Fs, Hs = F.cpu().numpy().astype(np.float64), H.cpu().numpy()
    theta = float(np.abs(Fs).sum() / g1.n)
    di.diffuse_round(G1, F, H, theta, d=D)
    Fr, Hr, S = oracle.set_step_signed(g1, D, theta, Fs, Hs)
    Hg, Fg = H.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    assert np.array_equal(Hg, Hr)  # same set taken, F_i added to H_i once in fp64
    # fluid: k pushes into a node, each rounded once, summed in any order
    src, dst = g1.edges()
    share = np.zeros(g1.n)
    share[S] = D * Fs[S] / np.maximum(g1.outdeg[S], 1)
    push = np.abs(share[src])
    k = np.bincount(dst, weights=(push > 0).astype(float), minlength=g1.n)
    mag = np.abs(np.where(S, 0.0, Fs)) + np.bincount(dst, weights=push, minlength=g1.n)
    eps = 2.0 ** -24 if prec == "fp32" else 2.0 ** -53
    assert np.all(np.abs(Fg - Fr) <= (k + 2) * 2 * eps * mag + 1e-300)


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-11, 1e-12), ("fp32", 1e-8, 1e-6)])
def test_update_then_resume_reaches_new_limit(di, pair, prec, tol, eps):
    g0, g1 = pair
    G0, G1 = di.Graph(g0), di.Graph(g1)
    F, H = _state(di, G0, g0, prec, tol)
    di.inject_update(G0, G1, F, H, d=D)
    x, st = di.solve(G1, d=D, tol=tol, precision=prec, state=(F, H))
    xs = oracle.limit(g1, D, tol=1e-14)
    assert st["residual_l1"] < tol
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + eps
    assert abs(st["mass_drift"]) < (1e-12 if prec == "fp64" else 1e-5)
    # a 1% change costs far less than solving P' from scratch
    _, fresh = di.solve(G1, d=D, tol=tol, precision=prec)
    assert st["edges_diffused"] < 0.6 * fresh["edges_diffused"]


def test_inject_rejects_mismatched_graphs(di):
    import torch
    a, b = di.Graph(wl.cycle(10)), di.Graph(wl.cycle(11))
    F = torch.zeros(11, dtype=torch.float64, device="cuda")
    H = torch.zeros(11, dtype=torch.float64, device="cuda")
    # the binding refuses before any library call ...
    with pytest.raises(ValueError):
        di.inject_update(a, b, F, H)
    # ... and the library itself returns DI_EINVAL for the same call
    rc = di._lib.di_inject_update(a.handle, b.handle, di.PRECISION["fp64"], 0.85,
                                  di._ptr(F), di._ptr(H), None)
    assert rc == di.EINVAL


@pytest.mark.timeout(600)
def test_update_at_one_million_nodes(di):
    """The benchmark's update at full size: 1% of the 10^6-node graph's rows get
    new out-links after an fp32 solve; inject + resume to 1e-8.  Theorem 1 for
    P' on every node of the device state, and the result within its bound of
    the oracle's limit of P' (MAT-ITER on every host core to
    ||X_n - X_n-1||_1 < 1e-12, plus that stop's own bound)."""
    g0 = wl.recipe("powerlaw-1m")
    g1 = wl.modify_graph(g0, 0.01, seed=78)
    G0, G1 = di.Graph(g0), di.Graph(g1)
    F, H = _state(di, G0, g0, "fp32", 1e-8)
    di.inject_update(G0, G1, F, H, d=D)
    x, st = di.solve(G1, d=D, tol=1e-8, precision="fp32", state=(F, H))
    assert st["residual_l1"] < 1e-8
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    deg = np.diff(g1.row_ptr)
    src = np.repeat(np.arange(g1.n, dtype=np.int32), deg)
    PH = np.bincount(g1.col_idx, weights=Hn[src] / deg[src], minlength=g1.n)
    assert np.abs(Hn + Fn - ((1 - D) / g1.n + D * PH)).sum() < 1e-6
    ref = oracle.power_omp(g1, D, 1e-12)
    ref_bound = 2 * D * ref["stats"]["residual"] / ((1 - D) * ref["X"].sum())
    l1 = float(np.abs(x.cpu().numpy() - ref["x"]).sum())
    assert l1 <= st["err_bound_l1"] + ref_bound + 1e-6


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-11, 1e-12), ("fp32", 1e-8, 1e-6)])
def test_successive_updates(di, prec, tol, eps):
    """On-line use: five successive changes of 1% of the rows, each injected
    into the state the previous one left and resumed.  The final result is
    within its bound of the exact limit of the last graph, and Theorem 1 holds
    for it on the final state."""
    g = wl.recipe("pagerank-10k")
    graphs = [g]
    for k in range(5):
        graphs.append(wl.modify_graph(graphs[-1], 0.01, seed=200 + k))
    Gs = [di.Graph(x) for x in graphs]
    F, H = _state(di, Gs[0], g, prec, tol)
    for k in range(5):
        di.inject_update(Gs[k], Gs[k + 1], F, H, d=D)
        x, st = di.solve(Gs[k + 1], d=D, tol=tol, precision=prec, state=(F, H))
        assert st["residual_l1"] < tol
    last = graphs[-1]
    xs = oracle.limit(last, D, tol=1e-14)
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + eps
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    PH = oracle.transition_sparse(last) @ Hn
    assert np.abs(Hn + Fn - ((1 - D) / last.n + D * PH)).sum() < (1e-12 if prec == "fp64" else 1e-6)
