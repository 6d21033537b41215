"""GPU parity: the HIP D-iteration and power iteration against the CPU oracle.

Element-wise checks of one threshold round (di_diffuse_round vs the oracle's
set step from the same seeded state), limit parity of full solves against the
oracle's exact solution within the reported bound plus the precision
tolerance (1e-12 all-fp64, 1e-6 fp32 fluid), closed forms, and Theorem 1 on
full-size device states.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

D = 0.85
EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


@pytest.fixture(scope="module")
def di():
    import torch
    from paper_1202_6158_amd import di as _di
    torch.cuda.set_device(0)
    return _di


def _round_case(di, g, F, H, theta, prec):
    import torch
    G = di.Graph(g)
    tdtype = torch.float32 if prec == "fp32" else torch.float64
    Ft = torch.tensor(F, dtype=tdtype, device="cuda")
    Ht = torch.tensor(H, dtype=torch.float64, device="cuda")
    tn, te = di.diffuse_round(G, Ft, Ht, theta, d=D)
    Fo, Ho, taken, st = oracle.set_step(g, D, theta, F.astype(np.float64), H)
    Fg = Ft.cpu().numpy().astype(np.float64)
    Hg = Ht.cpu().numpy()
    # the taken set and the history are decided and updated identically
    assert tn == int(taken.sum())
    assert te == st["edges"]
    np.testing.assert_array_equal(Hg, Ho)
    np.testing.assert_array_equal(Fg[taken & (np.bincount(g.col_idx, minlength=g.n) == 0)], 0.0)
    # fluid: k pushes into a node, each rounded once, summed in any order
    src, dst = g.edges()
    deg = g.outdeg
    share = np.zeros(g.n)
    share[taken] = D * F.astype(np.float64)[taken] / np.maximum(deg[taken], 1)
    push = share[src]
    k = np.bincount(dst, weights=(push > 0).astype(float), minlength=g.n)
    mag = np.abs(np.where(taken, 0.0, F.astype(np.float64))) + np.bincount(dst, weights=push, minlength=g.n)
    eps = EPS32 if prec == "fp32" else EPS64
    tol = (k + 2) * 2 * eps * mag + 1e-300
    bad = np.abs(Fg - Fo) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:10], Fg[bad][:5], Fo[bad][:5])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("gname", ["rand", "rand_ragged", "pagerank-10k", "outstar", "selfloops"])
def test_round_matches_oracle_set_step(di, prec, gname):
    if gname == "rand":
        g = wl.random_small(4096, 30000, seed=1)
    elif gname == "rand_ragged":
        g = wl.random_small(7777, 51234, seed=2, p_dangling=0.3)
    elif gname == "outstar":
        g = wl.out_star(5000)
    elif gname == "selfloops":
        g = wl.from_edges(3000, np.r_[np.arange(3000), np.arange(3000)],
                          np.r_[np.arange(3000), (np.arange(3000) * 7) % 3000])
    else:
        g = wl.recipe(gname)
    F, H = wl.random_fluid(g.n, seed=5)
    if prec == "fp64":
        F = F.astype(np.float64) * (1 + 1e-9 * np.arange(g.n) / g.n)
    for q in [0.0, 0.5, 0.9, 1.0]:
        pos = F[F > 0]
        theta = 0.0 if q == 0 else float(np.quantile(pos, q))
        _round_case(di, g, F, H, theta, prec)


def test_round_edge_cases(di):
    import torch
    # no out-links at all, and a theta above every fluid
    g = wl.from_edges(1000, [], [])
    F, H = wl.random_fluid(1000, seed=3)
    _round_case(di, g, F, H, 0.0, "fp32")
    g = wl.random_small(2000, 9000, seed=4)
    F, H = wl.random_fluid(2000, seed=4)
    _round_case(di, g, F, H, float(F.max()) * 2, "fp32")
    # single node with a self-loop
    g = wl.from_edges(1, [0], [0])
    _round_case(di, g, np.array([0.25], np.float32), np.array([0.5]), 0.0, "fp64")


# --------------------------------------------------------------- full solves

def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


@pytest.mark.parametrize("g", [wl.cycle(1000), wl.in_star(3000), wl.out_star(3000), wl.bi_star(2500),
                               wl.from_edges(1, [0], [0]), wl.from_edges(300, [], [])],
                         ids=["cycle", "instar", "outstar", "bistar", "selfloop1", "alldangling"])
def test_closed_forms_on_gpu(di, g):
    xs = oracle.dense_exact(g, D)[1] if g.n <= 2000 else oracle.sparse_exact(g, D)[1]
    for prec, eps in [("fp64", 1e-12), ("fp32", 1e-6)]:
        x, st = di.solve(di.Graph(g), d=D, tol=1e-13 if prec == "fp64" else 1e-9, precision=prec)
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + eps, (prec, st)
        xp, sp = di.power_solve(di.Graph(g), d=D, tol=1e-13, precision="fp64")
        assert _l1(xp.cpu().numpy(), xs) <= sp["err_bound_l1"] + 1e-12


@pytest.fixture(scope="module")
def c1():
    g = wl.recipe("pagerank-10k")
    Y, xs = oracle.sparse_exact(g, D)
    return g, Y, xs


@pytest.mark.parametrize("sched", ["mean", "op2", "op"])
@pytest.mark.parametrize("c", [0.5, 1.0, 2.0])
def test_c1_fp64_limit_parity(di, c1, sched, c):
    g, Y, xs = c1
    G = di.Graph(g)
    tune = di.make_tune(sched, c)
    x, st = di.solve(G, d=D, tol=1e-10, precision="fp64", tune=tune)
    assert st["residual_l1"] < 1e-10
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12
    assert abs(st["mass_drift"]) < 1e-12
    # dedicated parity run: near-exact residual
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune)
    assert _l1(x.cpu().numpy(), xs) <= 1e-12


@pytest.mark.parametrize("wlog", [8, 10, 12, 14])
@pytest.mark.parametrize("threads", [512, 1024])
def test_launch_shapes_limit_parity(di, c1, wlog, threads):
    """Every window size and both workgroup sizes reach the oracle's limit, in
    fp64 and with fp32 fluid: 2^8 gives 40 windows with a 16-node tail, and
    2^14, clamped to 2^13 by the LDS budget, a window of eight 1024-node tiles
    plus a ragged 1808-node one."""
    g, Y, xs = c1
    G = di.Graph(g)
    tune = di.make_tune("op2", 0.5, wlog, threads=threads)
    x, st = di.solve(G, d=D, tol=1e-14, precision="fp64", tune=tune)
    assert _l1(x.cpu().numpy(), xs) <= 1e-12
    assert abs(st["mass_drift"]) < 1e-12
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", tune=tune)
    assert st["residual_l1"] < 1e-8
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6


@pytest.mark.parametrize("check_every", [1, 3, 64])
def test_fixed_check_intervals_reach_the_limit(di, c1, check_every):
    """The host polls the control blocks every check_every rounds (the next
    chunk already queued): the solve stops on the same round, whatever the
    interval, and reaches the oracle's limit."""
    g, Y, xs = c1
    G = di.Graph(g)
    tune = di.make_tune("op2", 0.5, check_every=check_every)
    x, st = di.solve(G, d=D, tol=1e-12, precision="fp64", tune=tune)
    _, ref = di.solve(G, d=D, tol=1e-12, precision="fp64", tune=di.make_tune("op2", 0.5))
    assert abs(st["rounds"] - ref["rounds"]) <= 1
    assert st["residual_l1"] < 1e-12
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12


def test_c1_fp32_limit_parity(di, c1):
    g, Y, xs = c1
    G = di.Graph(g)
    for tol in [1e-6, 1e-8]:
        x, st = di.solve(G, d=D, tol=tol, precision="fp32")
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6
        assert abs(st["mass_drift"]) < 1e-5


def test_c1_unnormalised_is_below_Y(di, c1):
    """H+F approaches Y = (1-d)(I-dP)^-1 V from below within d||F||/(1-d)."""
    g, Y, xs = c1
    x, st = di.solve(di.Graph(g), d=D, tol=1e-10, precision="fp64", normalize=False)
    y = x.cpu().numpy()
    gap = Y - y
    assert gap.min() >= -1e-15
    assert gap.sum() <= st["err_bound_l1"] * (1 + 1e-9) + 1e-15


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_power_iteration_parity(di, c1, prec):
    g, Y, xs = c1
    ref = oracle.power(g, D, 1e-10)
    x, st = di.power_solve(di.Graph(g), d=D, tol=1e-10, precision=prec)
    eps = 1e-12 if prec == "fp64" else 1e-6
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + eps
    # same number of products as the oracle's MAT-ITER (the residual sums may
    # round differently right at the threshold), and then the same iterate
    assert abs(st["rounds"] - ref["stats"]["rounds"]) <= 1
    if prec == "fp64" and st["rounds"] == ref["stats"]["rounds"]:
        np.testing.assert_allclose(x.cpu().numpy(), ref["x"], rtol=1e-12, atol=1e-18)


def test_personalised_vectors(di):
    g = wl.recipe("pagerank-10k")
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 6, 100, seed=9)
    for b in range(6):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.limit(g, D, v, tol=1e-14)
        x, st = di.solve(G, v=v, d=D, tol=1e-12, precision="fp64")
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-12
        x, st = di.solve(G, v=v, d=D, tol=1e-7, precision="fp32")
        assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6


def test_resume_continues_to_same_limit(di, c1):
    import torch
    g, Y, xs = c1
    G = di.Graph(g)
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float64, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    _, st1 = di.solve(G, d=D, tol=1e-4, precision="fp64", state=(F, H))
    x, st2 = di.solve(G, d=D, tol=1e-11, precision="fp64", state=(F, H))
    assert _l1(x.cpu().numpy(), xs) <= st2["err_bound_l1"] + 1e-12
    # the returned state satisfies Theorem 1: H + F = F0 + d P H
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy()
    src, dst = g.edges()
    PH = np.bincount(dst, weights=Hn[src] / g.outdeg[src], minlength=g.n)
    np.testing.assert_allclose(Hn + Fn, (1 - D) / g.n + D * PH, rtol=1e-11, atol=1e-18)


def test_max_rounds_reports_notconv_with_valid_bound(di, c1):
    g, Y, xs = c1
    x, st = di.solve(di.Graph(g), d=D, tol=1e-12, precision="fp64", max_rounds=5,
                     allow_notconv=True)
    assert st["status"] == di.ENOTCONV
    assert st["rounds"] == 5
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] * (1 + 1e-9)


def test_invalid_vector_rejected(di, c1):
    g, _, _ = c1
    G = di.Graph(g)
    v = np.full(g.n, 1.0 / g.n)
    v[0] = -v[0]
    with pytest.raises(di.DiError):
        di._check(di._lib.di_solve(G.handle, v.ctypes.data, di.ctypes.byref(di.make_opts()), None,
                                   None, None))


@pytest.mark.parametrize("bad", ["negative", "nan", "sum"])
def test_invalid_device_vector_rejected(di, c1, bad):
    """A device V gets the checks a host V gets: DI_EINVAL, nothing solved."""
    import torch
    g, _, _ = c1
    G = di.Graph(g)
    v = np.full(g.n, 1.0 / g.n)
    if bad == "negative":
        v[17] = -v[17]
    elif bad == "nan":
        v[g.n - 1] = np.nan
    else:
        v *= 0.5
    vd = torch.from_numpy(v).cuda()
    for fn in (di.solve, di.power_solve):
        with pytest.raises(di.DiError) as e:
            fn(G, v=vd, d=D, tol=1e-8)
        assert e.value.status == di.EINVAL


def test_host_buffers_match_device_buffers(di, c1):
    """v and x as host arrays (copied by the library) give the device-pointer
    results, for the D-iteration and the power iteration."""
    g, _, _ = c1
    G = di.Graph(g)
    rng = np.random.default_rng(9)
    seeds = np.sort(rng.choice(g.n, 25, replace=False))
    v = wl.seed_vector(g.n, seeds)
    xs = oracle.limit(g, D, v, tol=1e-14)
    for vv in (None, v):
        xh, sh = di.solve(G, v=vv, d=D, tol=1e-12, precision="fp64", host=True)
        xd, sd = di.solve(G, v=vv, d=D, tol=1e-12, precision="fp64")
        assert isinstance(xh, np.ndarray) and abs(sh["rounds"] - sd["rounds"]) <= 1
        assert _l1(xh, xd.cpu().numpy()) <= 1e-13
        ph, _ = di.power_solve(G, v=vv, d=D, tol=1e-12, host=True)
        pd, _ = di.power_solve(G, v=vv, d=D, tol=1e-12)
        assert _l1(ph, pd.cpu().numpy()) <= 1e-13
    assert _l1(xh, xs) <= sh["err_bound_l1"] + 1e-12


@pytest.fixture(scope="module")
def c2():
    return wl.recipe("powerlaw-1m")


def test_c2_fp32_theorem1_and_bound(di, c2):
    """Full-size 1M-node solve at the benchmark setting: Theorem 1 holds for the
    returned device state, ||F||_1 < tol, and H + F is below Y by at most
    d||F||_1/(1-d) (checked against the oracle's MAT-ITER limit)."""
    import torch
    g = c2
    G = di.Graph(g)
    F = torch.full((g.n,), (1 - D) / g.n, dtype=torch.float32, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    x, st = di.solve(G, d=D, tol=1e-8, precision="fp32", state=(F, H))
    assert st["residual_l1"] < 1e-8
    Hn, Fn = H.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    src, dst = g.edges()
    PH = np.bincount(dst, weights=Hn[src] / g.outdeg[src], minlength=g.n)
    lhs, rhs = Hn + Fn, (1 - D) / g.n + D * PH
    # fp32 pushes: each node's value carries rounding of its fp32 fluid history
    assert np.abs(lhs - rhs).sum() < 1e-6
    xs = oracle.power(g, D, 1e-12)["x"]
    assert _l1(x.cpu().numpy(), xs) <= st["err_bound_l1"] + 1e-6
    xp, sp = di.power_solve(G, d=D, tol=1e-8, precision="fp64")
    assert _l1(xp.cpu().numpy(), xs) <= sp["err_bound_l1"] + 1e-12


def test_concurrent_solves_on_one_graph(di, c1):
    """Four host threads, each with its own stream, solve personalised vectors
    on the same resident graph at once (each call takes its own workspace from
    the graph's pool): every result equals the same solve run alone."""
    import threading
    import torch
    g, _, _ = c1
    G = di.Graph(g)
    rng = np.random.default_rng(77)
    vs = [wl.seed_vector(g.n, np.sort(rng.choice(g.n, 30, replace=False))) for _ in range(12)]
    alone = [di.solve(G, v=v, d=D, tol=1e-12, precision="fp64")[0].cpu().numpy() for v in vs]
    out = [None] * len(vs)
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for i in range(k, len(vs), 4):
                    x, _ = di.solve(G, v=vs[i], d=D, tol=1e-12, precision="fp64", stream=s)
                    s.synchronize()
                    out[i] = x.cpu().numpy()
        except Exception as e:  # reported below, on the test's thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    assert not errors, errors
    for i in range(len(vs)):
        assert out[i] is not None and _l1(out[i], alone[i]) <= 1e-13, i
