"""GPU parity of batched personalised PageRank (di_solve_batch) against the
CPU oracle: every vector of a batch within its own error bound of the exact
PPR vector, batched vs one-at-a-time results, weighted seed sets, linearity of
the unnormalised result in V, validation, and the 256-vector workload on the
10^6-node graph on sampled vectors."""
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


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


@pytest.fixture(scope="module")
def c1():
    return wl.recipe("pagerank-10k")


@pytest.mark.parametrize("prec,tol,eps", [("fp64", 1e-11, 1e-12), ("fp32", 1e-6, 1e-6)])
def test_batch_vectors_match_exact_ppr(di, c1, prec, tol, eps):
    g = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 24, 100, seed=11)
    x, stats = di.solve_batch(G, ptr, seeds, d=D, tol=tol, precision=prec)
    xb = x.cpu().numpy()
    for b in range(24):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.limit(g, D, v, tol=1e-14)
        assert stats[b]["residual_l1"] < tol
        assert _l1(xb[b], xs) <= stats[b]["err_bound_l1"] + eps, b


@pytest.mark.parametrize("sched,wlog,threads", [("mean", 8, 1024), ("op", 12, 512),
                                                ("op2", 13, 1024)])
def test_batch_launch_shapes(di, c1, sched, wlog, threads):
    """Batches at other schedules, window sizes and workgroup sizes: every
    vector within its bound of the exact PPR vector."""
    g = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 6, 100, seed=13)
    tune = di.make_tune(sched, 0.5, wlog, threads=threads)
    x, stats = di.solve_batch(G, ptr, seeds, d=D, tol=1e-11, precision="fp64", tune=tune)
    xb = x.cpu().numpy()
    for b in range(6):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.limit(g, D, v, tol=1e-14)
        assert stats[b]["residual_l1"] < 1e-11
        assert _l1(xb[b], xs) <= stats[b]["err_bound_l1"] + 1e-12, b


def test_batch_equals_solo(di, c1):
    g = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 8, 100, seed=12)
    x, stats = di.solve_batch(G, ptr, seeds, d=D, tol=1e-12, precision="fp64")
    for b in range(8):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs, ss = di.solve(G, v=v, d=D, tol=1e-12, precision="fp64")
        assert _l1(x[b].cpu().numpy(), xs.cpu().numpy()) <= \
            stats[b]["err_bound_l1"] + ss["err_bound_l1"] + 1e-12


def test_weighted_seeds_and_single_vector_batch(di, c1):
    g = c1
    G = di.Graph(g)
    rng = np.random.default_rng(3)
    seeds = np.sort(rng.choice(g.n, size=30, replace=False)).astype(np.int32)
    w = rng.random(30)
    w /= w.sum()
    ptr = np.array([0, 30], dtype=np.int64)
    x, stats = di.solve_batch(G, ptr, seeds, seed_w=w, d=D, tol=1e-12, precision="fp64")
    v = np.zeros(g.n)
    v[seeds] = w
    xs = oracle.limit(g, D, v, tol=1e-14)
    assert _l1(x[0].cpu().numpy(), xs) <= stats[0]["err_bound_l1"] + 1e-12


def test_unnormalised_result_is_linear_in_v(di, c1):
    """Y = (1-d)(I-dP)^{-1}V is linear in V: the batch of {a}, {b}, {a,b}."""
    g = c1
    G = di.Graph(g)
    a_, b_ = 17, 4242
    ptr = np.array([0, 1, 2, 4], dtype=np.int64)
    seeds = np.array([a_, b_, a_, b_], dtype=np.int32)
    x, st = di.solve_batch(G, ptr, seeds, d=D, tol=1e-13, precision="fp64", normalize=False)
    y = x.cpu().numpy()
    bound = sum(s["err_bound_l1"] for s in st)
    assert _l1(y[2], 0.5 * (y[0] + y[1])) <= bound + 1e-13


@pytest.mark.parametrize("ptr,seeds,w", [
    ([0, 0], [], None),                         # empty set
    ([0, 2], [1, 10 ** 9], None),               # out of range
    ([0, 2], [5, 5], None),                     # repeated
    ([0, 2], [1, 2], [0.5, 0.6]),               # weights do not sum to 1
    ([0, 2], [1, 2], [1.5, -0.5]),              # negative weight
])
def test_batch_rejects_invalid_seed_sets(di, c1, ptr, seeds, w):
    G = di.Graph(c1)
    with pytest.raises(di.DiError) as e:
        di.solve_batch(G, np.array(ptr), np.array(seeds, dtype=np.int32),
                       None if w is None else np.array(w), d=D, tol=1e-6)
    assert e.value.status == di.EINVAL


def test_batch_256_vectors_on_1m_graph(di):
    """The batched workload: 256 seed sets (1-100 nodes, log-uniform) on the
    10^6-node graph, fp32 fluid, stop at 1e-6; three sampled vectors against
    the oracle's MAT-ITER solution, all vectors against their stop rule."""
    g = wl.recipe("powerlaw-1m")
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 256, 100, seed=4)
    x, stats = di.solve_batch(G, ptr, seeds, d=D, tol=1e-6, precision="fp32")
    assert all(s["residual_l1"] < 1e-6 for s in stats)
    assert all(abs(s["mass_drift"]) < 1e-5 for s in stats)
    for b in [0, 101, 255]:
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        xs = oracle.power(g, D, 1e-11, v)["x"]
        assert _l1(x[b].cpu().numpy(), xs) <= stats[b]["err_bound_l1"] + 1e-6, b


@pytest.mark.parametrize("normalize", [True, False])
def test_batch_topk_is_the_top_of_the_full_result(di, c1, normalize):
    """di_solve_batch_topk returns, per vector, the k largest entries of what
    di_solve_batch returns in full (the same device arithmetic), largest first."""
    g = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 10, 100, seed=14)
    x, _ = di.solve_batch(G, ptr, seeds, d=D, tol=1e-11, precision="fp64", normalize=normalize)
    ids, vals, st = di.solve_batch_topk(G, ptr, seeds, k=50, d=D, tol=1e-11, precision="fp64",
                                        normalize=normalize)
    xb = x.cpu().numpy()
    assert ids.shape == (10, 50) and vals.shape == (10, 50)
    for b in range(10):
        assert st[b]["residual_l1"] < 1e-11
        assert np.all(np.diff(vals[b]) <= 0)
        np.testing.assert_allclose(vals[b], np.sort(xb[b])[::-1][:50], rtol=1e-13, atol=0)
        np.testing.assert_allclose(xb[b][ids[b]], vals[b], rtol=1e-13, atol=0)
        assert len(set(ids[b].tolist())) == 50


def test_batch_with_host_output(di, c1):
    """x as a host array: the library copies each group back; same result as
    the device output."""
    g = c1
    G = di.Graph(g)
    ptr, seeds = wl.ppr_seed_sets(g.n, 5, 100, seed=15)
    xh, sh = di.solve_batch(G, ptr, seeds, d=D, tol=1e-11, precision="fp64", host=True)
    xd, sd = di.solve_batch(G, ptr, seeds, d=D, tol=1e-11, precision="fp64")
    assert isinstance(xh, np.ndarray) and xh.shape == (5, g.n)
    for b in range(5):
        assert abs(sh[b]["rounds"] - sd[b]["rounds"]) <= 1
        assert _l1(xh[b], xd[b].cpu().numpy()) <= 1e-13


def test_batch_topk_pads_short_vectors(di):
    """A seed on a dangling leaf of an out-star keeps all its fluid: one
    non-zero entry, the rest of the k slots padded with -1 / 0."""
    g = wl.out_star(10)
    G = di.Graph(g)
    ptr = np.array([0, 1, 2], np.int64)
    seeds = np.array([3, 0], np.int32)
    ids, vals, _ = di.solve_batch_topk(G, ptr, seeds, k=20, d=D, tol=1e-13, precision="fp64")
    assert ids[0, 0] == 3 and abs(vals[0, 0] - 1.0) < 1e-15
    assert np.all(ids[0, 1:] == -1) and np.all(vals[0, 1:] == 0.0)
    # seed on the centre: the centre and its 10 leaves, then padding
    assert np.all(ids[1, :11] >= 0) and np.all(ids[1, 11:] == -1)
    xs = oracle.dense_exact(g, D, wl.seed_vector(g.n, [0]))[1]
    np.testing.assert_allclose(vals[1, :11], xs[ids[1, :11]], rtol=0, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_topk_with_many_ties(di, prec):
    """An out-star whose hub has the highest id and 12,000 dangling leaves,
    seeded at the hub: the leaves tie exactly (x_l = d/(k(1+d))), more than
    the device keeps per vector in one pass.  The hub (x_c = 1/(1+d)) must come
    first, then the lowest leaf ids; a second vector seeded at leaf 5 keeps all
    its fluid there."""
    k = 12000
    g = wl.from_edges(k + 1, [k] * k, list(range(k)))
    G = di.Graph(g)
    ptr = np.array([0, 1, 2], np.int64)
    seeds = np.array([k, 5], np.int32)
    tol = 1e-12 if prec == "fp64" else 1e-7
    ids, vals, _ = di.solve_batch_topk(G, ptr, seeds, k=100, d=D, tol=tol, precision=prec)
    assert ids[0, 0] == k
    assert abs(vals[0, 0] - 1.0 / (1.0 + D)) < (1e-12 if prec == "fp64" else 1e-6)
    assert ids[0, 1:].tolist() == list(range(99))
    np.testing.assert_allclose(vals[0, 1:], D / (k * (1.0 + D)), rtol=1e-6)
    assert ids[1, 0] == 5 and abs(vals[1, 0] - 1.0) < 1e-15 and np.all(ids[1, 1:] == -1)


@pytest.mark.parametrize("k", [0, 1025])
def test_batch_topk_rejects_bad_k(di, c1, k):
    G = di.Graph(c1)
    with pytest.raises(di.DiError) as e:
        di.solve_batch_topk(G, np.array([0, 1], np.int64), np.array([5], np.int32), k=k)
    assert e.value.status == di.EINVAL
