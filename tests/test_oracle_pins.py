"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check here is independent of the oracle's own code path: hand-derived
closed forms, a library eigensolver on the completed matrix, identities the
paper proves (Theorems 1 and 2, the Lemma of Section 3.1, the power series of
Section 2.2) evaluated with scipy.sparse matrices built here from the edge
list, and brute force on tiny graphs.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as wl

D = 0.85
ORDERS = ["per", "rand", "max", "sweep", "op", "op2"]


def P_sparse(g):
    """Column-stochastic P (zero dangling columns) built from the edge list."""
    src, dst = g.edges()
    deg = g.outdeg
    return sp.csr_matrix((1.0 / deg[src], (dst, src)), shape=(g.n, g.n))


def all_solvers(g, d, v=None, tol=1e-14):
    """Normalised results of every oracle route."""
    runs = {"power": oracle.power(g, d, tol, v, max_iter=100_000),
            "sets_c1": oracle.diter_sets(g, d, tol, c=1.0, v=v, max_rounds=100_000),
            "sets_jacobi": oracle.diter_sets(g, d, tol, c=0.0, v=v, max_rounds=100_000)}
    for o in ORDERS:
        runs[o] = oracle.diter(g, d, tol, order=o, v=v, seed=7, max_picks=2_000_000)
    for name, r in runs.items():
        assert r["converged"], name
    out = {name: r["x"] for name, r in runs.items()}
    out["dense"] = oracle.dense_exact(g, d, v)[1]
    return out


# ------------------------------------------------------------ closed forms

def test_transition_matrix_by_hand():
    # 0->1, 0->2, 0->2 (repeated), 1->1 (self-loop), 2 dangling
    g = wl.from_edges(3, [0, 0, 0, 1], [1, 2, 2, 1])
    P = oracle.transition_dense(g)
    expect = np.array([[0, 0, 0], [1 / 3, 1, 0], [2 / 3, 0, 0]])
    np.testing.assert_allclose(P, expect, atol=0)


def test_sparse_transition_by_hand_and_against_dense():
    """The sparse P used by the update and replay helpers: the same hand-worked
    matrix (repeated link, self-loop, dangling column), and equal to the dense
    one on random graphs with repeats and self-loops."""
    g = wl.from_edges(3, [0, 0, 0, 1], [1, 2, 2, 1])
    expect = np.array([[0, 0, 0], [1 / 3, 1, 0], [2 / 3, 0, 0]])
    np.testing.assert_allclose(oracle.transition_sparse(g).toarray(), expect, atol=0)
    for seed in (1, 2, 3):
        g = wl.random_small(120, 700, seed=seed)
        np.testing.assert_allclose(oracle.transition_sparse(g).toarray(),
                                   oracle.transition_dense(g), rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [1, 2, 7, 50])
def test_cycle_uniform(n):
    g = wl.cycle(n) if n > 1 else wl.from_edges(1, [0], [0])
    for name, x in all_solvers(g, D).items():
        np.testing.assert_allclose(x, np.full(n, 1.0 / n), atol=1e-13, err_msg=name)


@pytest.mark.parametrize("k", [1, 5, 17])
def test_in_star(k):
    # leaves -> dangling centre: x_c = (1+dk)/(k+1+dk), x_l = 1/(k+1+dk)
    g = wl.in_star(k)
    xc, xl = (1 + D * k) / (k + 1 + D * k), 1 / (k + 1 + D * k)
    expect = np.array([xc] + [xl] * k)
    for name, x in all_solvers(g, D).items():
        np.testing.assert_allclose(x, expect, atol=1e-13, err_msg=name)


@pytest.mark.parametrize("k", [1, 5, 17])
def test_out_star(k):
    # centre -> dangling leaves: x_c = 1/(k+1+d), x_l = (1+d/k)/(k+1+d)
    g = wl.out_star(k)
    expect = np.array([1 / (k + 1 + D)] + [(1 + D / k) / (k + 1 + D)] * k)
    for name, x in all_solvers(g, D).items():
        np.testing.assert_allclose(x, expect, atol=1e-13, err_msg=name)


@pytest.mark.parametrize("k", [2, 9])
def test_bi_star(k):
    # no dangling node: Y sums to one, Y_c = (1+dk)/(N(1+d)), Y_l = (1-d)/N + d Y_c/k
    g = wl.bi_star(k)
    n = k + 1
    yc = (1 + D * k) / (n * (1 + D))
    expect = np.array([yc] + [(1 - D) / n + D * yc / k] * k)
    Y, _ = oracle.dense_exact(g, D)
    np.testing.assert_allclose(Y, expect, atol=1e-15)
    for name, x in all_solvers(g, D).items():
        np.testing.assert_allclose(x, expect, atol=1e-13, err_msg=name)


def test_d_zero_gives_v():
    g = wl.random_small(30, 90, seed=3)
    v = np.random.default_rng(1).random(30)
    v /= v.sum()
    for name, x in all_solvers(g, 0.0, v).items():
        np.testing.assert_allclose(x, v, atol=1e-15, err_msg=name)


def test_all_dangling_gives_v():
    g = wl.from_edges(6, [], [])
    v = np.array([0.1, 0.2, 0.3, 0.15, 0.05, 0.2])
    for name, x in all_solvers(g, D, v).items():
        np.testing.assert_allclose(x, v, atol=1e-15, err_msg=name)


@pytest.mark.parametrize("n", [5, 12])
def test_ppr_on_cycle(n):
    # V = e_0 on a directed n-cycle: Y_k = (1-d) d^k / (1 - d^n)
    g = wl.cycle(n)
    v = np.zeros(n)
    v[0] = 1.0
    Y = (1 - D) * D ** np.arange(n) / (1 - D ** n)
    Yd, _ = oracle.dense_exact(g, D, v)
    np.testing.assert_allclose(Yd, Y, atol=1e-15)
    for name, x in all_solvers(g, D, v).items():
        np.testing.assert_allclose(x, Y / Y.sum(), atol=1e-13, err_msg=name)


# ----------------------------------------------- definitions cross-checked

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_renormalised_limit_is_completed_pagerank(seed):
    """Section 3.3: H_inf / ||H_inf||_1 equals the PageRank of the matrix completed
    with V on its dangling columns (independent route: eigenvector of A)."""
    g = wl.random_small(40, 120, seed=seed, p_dangling=0.3)
    v = np.random.default_rng(seed).random(40)
    v /= v.sum()
    x = oracle.dense_exact(g, D, v)[1]
    np.testing.assert_allclose(x, oracle.completed_pagerank(g, D, v), atol=1e-13)


def test_sparse_and_dense_exact_agree():
    g = wl.random_small(700, 4000, seed=5)
    np.testing.assert_allclose(oracle.sparse_exact(g, D)[1], oracle.dense_exact(g, D)[1],
                               atol=1e-14)


# -------------------------------------------------- theorems of Section 3

def _partial(g, order, picks, v=None, d=D):
    return oracle.diter(g, d, 1e-300, order=order, v=v, seed=11, max_picks=picks)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("picks", [1, 7, 60, 400])
def test_theorem1_invariant(order, picks):
    """Theorem 1: H_n + F_n = F_0 + d P H_n, componentwise, for any sequence.
    Also: the running R of ALGO-REF with the dangling rule (Section 3.3) equals
    the remaining fluid ||F_n||_1."""
    g = wl.random_small(50, 160, seed=picks, p_dangling=0.25)
    r = _partial(g, order, picks)
    assert r["stats"]["running_r"] == pytest.approx(r["F"].sum(), rel=1e-12)
    F0 = (1 - D) * np.full(g.n, 1.0 / g.n)
    lhs = r["H"] + r["F"]
    rhs = F0 + D * (P_sparse(g) @ r["H"])
    np.testing.assert_allclose(lhs, rhs, atol=1e-16, rtol=1e-13)


@pytest.mark.parametrize("picks", [3, 40, 300])
def test_theorem2_equality_without_dangling(picks):
    """Theorem 2: ||S_inf - H_n||_1 = ||F_n||_1/(1-d) when no column of P is zero."""
    g = wl.random_small(45, 200, seed=picks, p_dangling=0.0)
    assert g.n_dangling == 0
    Y, _ = oracle.dense_exact(g, D)
    for order in ORDERS:
        r = _partial(g, order, picks)
        err = np.abs(Y - r["H"]).sum()
        assert err == pytest.approx(np.abs(r["F"]).sum() / (1 - D), rel=1e-12), order


@pytest.mark.parametrize("picks", [3, 40, 300])
def test_theorem2_bounds_with_dangling(picks):
    """With dangling nodes ||F||/(1-d) only bounds ||Y - H||_1 (Section 3.3), and
    Y - (H+F) = dP(I-dP)^{-1}F >= 0 is bounded by d||F||_1/(1-d)."""
    g = wl.random_small(45, 150, seed=picks, p_dangling=0.3)
    Y, _ = oracle.dense_exact(g, D)
    for order in ORDERS:
        r = _partial(g, order, picks)
        nf = np.abs(r["F"]).sum()
        assert np.abs(Y - r["H"]).sum() <= nf / (1 - D) * (1 + 1e-12) + 1e-16
        gap = Y - (r["H"] + r["F"])
        assert gap.min() >= -1e-15
        assert gap.sum() <= D * nf / (1 - D) * (1 + 1e-12) + 1e-16


def test_history_increases_to_limit():
    """Section 3.1: H_n increases componentwise and stays below X = H_inf."""
    g = wl.random_small(60, 240, seed=9)
    Y, _ = oracle.dense_exact(g, D)
    prev = np.zeros(g.n)
    for picks in [1, 5, 20, 80, 320, 1280, 5120]:
        H = _partial(g, "rand", picks)["H"]
        assert np.all(H >= prev - 1e-17)
        assert np.all(H <= Y + 1e-15)
        prev = H


@pytest.mark.parametrize("order", ["max", "op", "op2"])
def test_lemma_contraction_for_argmax(order):
    """Lemma of Section 3.1: with i_n = argmax F, ||F_n|| <= ||F_{n-1}||(1-(1-d)/N).
    (Checked for MAX; OP/OP2 need not satisfy it, so they are only checked for
    monotone decrease.)"""
    g = wl.random_small(35, 120, seed=4)
    r = oracle.diter(g, D, 1e-300, order=order, max_picks=500, trace_len=500)
    tr = np.concatenate([[1 - D], r["trace"]])
    ratio = tr[1:] / tr[:-1]
    if order == "max":
        assert np.all(ratio <= 1 - (1 - D) / g.n + 1e-12)
    else:
        assert np.all(ratio <= 1 + 1e-12)


# Six nodes, worked by hand: out-links 0->{1,2,3}, 1->{0}, 2->{0,1}, 3 dangling,
# 4->{0,1,2,3}, 5->{0}; so #out = (3,1,2,0,4,1) and #in = (4,3,2,2,0,0).
# V = (.30,.20,.10,.08,.22,.10), F_0 = (1-d)V.  Scores of F_0 / (1-d):
#   MAX  F_i:                          .30 .20 .10 .08 .22 .10 -> node 0
#   OP2  F_i/(#out_i+1):               .075 .10 .033 .08 .044 .05 -> node 1
#   OP   F_i/((#in_i+1)(#out_i+1)):    .015 .025 .011 .027 .044 .05 -> node 5
# Second picks (d = .85), after the first node's d*F is pushed to its children:
#   MAX: node 0 sends .045 -> +.01275 to 1,2,3; F = (0,.04275,.02775,.02475,.033,.015) -> 1
#   OP2: node 1 sends .03 -> +.0255 to 0; scores (.017625,-,.005,.012,.0066,.0075) -> 0
#   OP:  node 5 sends .015 -> +.01275 to 0; scores (.0028875,.00375,.00167,.004,.0066,-) -> 4
# A slip in either score (a sum for OP's product, #in for OP2's #out, a
# dropped +1) moves the first pick to node 4 or 3.
_SCORE_G = ([0, 0, 0, 1, 2, 2, 4, 4, 4, 4, 5], [1, 2, 3, 0, 0, 1, 0, 1, 2, 3, 0])
_SCORE_V = np.array([0.30, 0.20, 0.10, 0.08, 0.22, 0.10])


@pytest.mark.parametrize("order,first,second,h2", [
    ("max", 0, 1, 0.15 * 0.20 + D * 0.15 * 0.30 / 3),
    ("op2", 1, 0, 0.15 * 0.30 + D * 0.15 * 0.20),
    ("op", 5, 4, 0.15 * 0.22),
])
def test_argmax_scores_by_hand(order, first, second, h2):
    """Section 4.3: ALGO-OP takes argmax F_i/((#in_i+1)(#out_i+1)), ALGO-OP2
    argmax F_i/(#out_i+1), ALGO-MAX argmax F_i (Section 4).  The first two picks
    of the oracle on the hand-worked graph above, and the fluid each moved."""
    g = wl.from_edges(6, *_SCORE_G)
    np.testing.assert_array_equal(g.outdeg, [3, 1, 2, 0, 4, 1])
    one = oracle.diter(g, D, 1e-300, order=order, v=_SCORE_V, max_picks=1)
    assert np.flatnonzero(one["H"]).tolist() == [first]
    assert one["H"][first] == pytest.approx((1 - D) * _SCORE_V[first], rel=1e-15)
    two = oracle.diter(g, D, 1e-300, order=order, v=_SCORE_V, max_picks=2)
    assert sorted(np.flatnonzero(two["H"]).tolist()) == sorted([first, second])
    assert two["H"][second] == pytest.approx(h2, rel=1e-14)


def test_jacobi_sets_equal_power_series():
    """All-nodes set steps from F_0 give H_n = S_{n-1} = (1-d) sum_{k<n} d^k P^k V
    (Section 2.2), which is also MAT-ITER's X_n from X_0 = 0."""
    g = wl.random_small(80, 300, seed=12)
    P = P_sparse(g)
    v = np.full(g.n, 1.0 / g.n)
    S, term = np.zeros(g.n), (1 - D) * v
    for n in range(1, 25):
        S = S + term
        term = D * (P @ term)
        H = oracle.diter_sets(g, D, 1e-300, c=0.0, max_rounds=n)["H"]
        X = oracle.power(g, D, 1e-300, max_iter=n)["X"]
        np.testing.assert_allclose(H, S, rtol=1e-13, atol=1e-18)
        np.testing.assert_allclose(X, S, rtol=1e-13, atol=1e-18)


def test_set_step_by_hand():
    # 0->1, 0->2, 1->2, 2 dangling; take {0, 2} with theta between b and min(a, c)
    g = wl.from_edges(3, [0, 0, 1], [1, 2, 2])
    a, b, c = 0.5, 0.1, 0.3
    F, H, taken, st = oracle.set_step(g, D, 0.3, [a, b, c], [1.0, 2.0, 3.0])
    np.testing.assert_array_equal(taken, [True, False, True])  # F_i >= theta is inclusive
    np.testing.assert_allclose(F, [0.0, b + D * a / 2, D * a / 2], rtol=1e-15)
    np.testing.assert_allclose(H, [1.0 + a, 2.0, 3.0 + c], rtol=1e-15)
    assert st["edges"] == 2 and st["picks"] == 2


def test_set_step_keeps_theorem1():
    g = wl.random_small(200, 900, seed=21)
    F, H = oracle.init_state(g.n, D)
    F0 = F.copy()
    rng = np.random.default_rng(0)
    for _ in range(30):
        theta = rng.uniform(0, 2) * F.sum() / g.n
        F, H, _, _ = oracle.set_step(g, D, theta, F, H)
    np.testing.assert_allclose(H + F, F0 + D * (P_sparse(g) @ H), rtol=1e-13, atol=1e-18)


def test_apply_set_by_hand_and_against_the_threshold_step():
    """apply_set (numpy) on the hand-worked example, and on random states equal
    to the C set step when given the threshold set."""
    g = wl.from_edges(3, [0, 0, 1], [1, 2, 2])
    a, b, c = 0.5, 0.1, 0.3
    F, H = oracle.apply_set(g, D, [True, False, True], [a, b, c], [1.0, 2.0, 3.0])
    np.testing.assert_allclose(F, [0.0, b + D * a / 2, D * a / 2], rtol=1e-15)
    np.testing.assert_allclose(H, [1.0 + a, 2.0, 3.0 + c], rtol=1e-15)
    g = wl.random_small(300, 1500, seed=23)
    rng = np.random.default_rng(3)
    F0 = rng.uniform(0, 1, g.n) * (rng.uniform(size=g.n) < 0.7)
    H0 = rng.uniform(0, 1, g.n)
    theta = 0.5 * F0.mean()
    Fc, Hc, taken, _ = oracle.set_step(g, D, theta, F0, H0)
    Fa, Ha = oracle.apply_set(g, D, taken, F0, H0)
    np.testing.assert_array_equal(Ha, Hc)
    np.testing.assert_allclose(Fa, Fc, rtol=1e-14, atol=1e-17)


def test_apply_set_keeps_theorem1_and_reaches_the_limit():
    """Any sequence of sets keeps H + F = F_0 + dPH (Theorem 1); sets that keep
    taking the nodes with fluid reach the exact limit (Theorem 2)."""
    g = wl.random_small(200, 900, seed=24)
    F, H = oracle.init_state(g.n, D)
    F0 = F.copy()
    rng = np.random.default_rng(5)
    for _ in range(40):
        F, H = oracle.apply_set(g, D, rng.uniform(size=g.n) < 0.4, F, H)
        np.testing.assert_allclose(H + F, F0 + D * (P_sparse(g) @ H), rtol=1e-13, atol=1e-18)
    for _ in range(400):
        F, H = oracle.apply_set(g, D, F > 0, F, H)
    assert F.sum() < 1e-14
    np.testing.assert_allclose((H + F) / (H + F).sum(), oracle.dense_exact(g, D)[1],
                               rtol=0, atol=1e-13)


# --------------------------------------------------- stop rule and orders

@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_order_independence_within_bound(tol):
    """Every sequence converges to the same limit (Sections 1, 3.2); at residual
    ||F||_1 < tol each normalised result is within 2d tol/((1-d)||H+F||_1) of x*."""
    g = wl.random_small(300, 1500, seed=2, p_dangling=0.2)
    xs = oracle.dense_exact(g, D)[1]
    for order in ORDERS:
        r = oracle.diter(g, D, tol, order=order, seed=3)
        assert r["converged"]
        nf = r["F"].sum()
        assert nf < tol
        bound = 2 * D * nf / ((1 - D) * (r["H"] + r["F"]).sum())
        assert np.abs(r["x"] - xs).sum() <= bound * (1 + 1e-9) + 1e-15, order
    for c in [0.0, 0.5, 1.0, 3.0]:
        r = oracle.diter_sets(g, D, tol, c=c)
        bound = 2 * D * r["F"].sum() / ((1 - D) * (r["H"] + r["F"]).sum())
        assert np.abs(r["x"] - xs).sum() <= bound * (1 + 1e-9) + 1e-15, c


def test_power_stop_rule_bound():
    """With X_0 = 0, X_n - X_{n-1} is the Jacobi fluid, so the MAT-ITER result at
    ||X_n - X_{n-1}||_1 < tol carries the same d tol/(1-d) bound (before
    normalisation) as the D-iteration."""
    g = wl.random_small(300, 1500, seed=8)
    Y, _ = oracle.dense_exact(g, D)
    for tol in [1e-3, 1e-6, 1e-9]:
        r = oracle.power(g, D, tol)
        assert r["converged"] and r["stats"]["residual"] < tol
        assert np.abs(Y - r["X"]).sum() <= D * r["stats"]["residual"] / (1 - D) * (1 + 1e-9)


def test_medium_graph_all_routes():
    """10k-node power-law graph: sparse LU, MAT-ITER and the threshold D-iteration."""
    g = wl.recipe("pagerank-10k")
    xs = oracle.sparse_exact(g, D)[1]
    np.testing.assert_allclose(oracle.power(g, D, 1e-13)["x"], xs, atol=1e-12)
    r = oracle.diter_sets(g, D, 1e-12, c=1.0)
    assert np.abs(r["x"] - xs).sum() < 1e-10
    r = oracle.diter(g, D, 1e-12, order="sweep")
    assert np.abs(r["x"] - xs).sum() < 1e-10


def test_threshold_variant_uses_fewer_elementary_steps():
    """Section 4.2's qualitative claim on a power-law graph: threshold rounds reach
    the same residual with fewer elementary steps than MAT-ITER."""
    g = wl.recipe("pagerank-10k")
    p = oracle.power(g, D, 1e-8)
    s = oracle.diter_sets(g, D, 1e-8, c=1.0)
    assert s["stats"]["edges"] < p["stats"]["edges"]


# ------------------------------------------------- graph updates (Section 3.2)

def _update_pair(seed):
    g0 = wl.random_small(40, 160, seed=seed, p_dangling=0.15)
    return g0, wl.modify_graph(g0, 0.25, seed=seed + 100)


def test_update_injection_gives_theorem1_for_the_new_graph():
    """After F' = F + d(P'-P)H, H + F' = F_0 + dP'H componentwise (the
    restart condition of the updating equation)."""
    g0, g1 = _update_pair(1)
    r = oracle.diter(g0, D, 1e-3, order="per")
    F1 = oracle.inject_update(g0, g1, D, r["F"], r["H"])
    P1 = oracle.transition_dense(g1)
    assert np.abs(r["H"] + F1 - ((1 - D) / g1.n + D * P1 @ r["H"])).max() < 1e-14


def test_update_equation_theorem3():
    """H'_inf - H_inf = (I - dP')^{-1} d (P' - P) H_inf, with both limits from
    dense solves of their definitions."""
    g0, g1 = _update_pair(3)
    Y0, Y1 = oracle.dense_exact(g0, D)[0], oracle.dense_exact(g1, D)[0]
    inj = oracle.inject_update(g0, g1, D, np.zeros(g0.n), Y0)
    Z = np.linalg.solve(np.eye(g1.n) - D * oracle.transition_dense(g1), inj)
    np.testing.assert_allclose(Z, Y1 - Y0, atol=1e-13)


def test_restart_after_update_reaches_the_new_limit_theorem4():
    """Continuing the D-iteration on P' from the injected state converges to
    the solution for P' (Theorem 4), although the injected fluid has both signs."""
    g0, g1 = _update_pair(2)
    r = oracle.diter(g0, D, 1e-4, order="per")
    F1 = oracle.inject_update(g0, g1, D, r["F"], r["H"])
    assert (F1 < 0).any() and (F1 > 0).any()
    r1 = oracle.diter(g1, D, 1e-14, order="per", state=(F1, r["H"]))
    assert r1["converged"]
    np.testing.assert_allclose(r1["x"], oracle.dense_exact(g1, D)[1], atol=1e-12)


def test_signed_set_steps_keep_theorem1_and_converge():
    g0, g1 = _update_pair(4)
    r = oracle.diter(g0, D, 1e-3, order="per")
    F, H = oracle.inject_update(g0, g1, D, r["F"], r["H"]), r["H"].copy()
    P1 = oracle.transition_dense(g1)
    for _ in range(400):
        nf = np.abs(F).sum()
        if nf < 1e-13:
            break
        F, H, S = oracle.set_step_signed(g1, D, nf / g1.n, F, H)
        assert S.any()
        assert np.abs(H + F - ((1 - D) / g1.n + D * P1 @ H)).max() < 1e-14
    assert np.abs(F).sum() < 1e-13
    np.testing.assert_allclose((H + F) / (H + F).sum(), oracle.dense_exact(g1, D)[1], atol=1e-12)


def test_modify_graph_changes_only_the_chosen_rows():
    g0 = wl.random_small(200, 1000, seed=9, p_dangling=0.1)
    g1 = wl.modify_graph(g0, 0.1, seed=10)
    d0, d1 = np.diff(g0.row_ptr), np.diff(g1.row_ptr)
    same = [i for i in range(g0.n) if d0[i] == d1[i] and np.array_equal(
        g0.col_idx[g0.row_ptr[i]:g0.row_ptr[i + 1]], g1.col_idx[g1.row_ptr[i]:g1.row_ptr[i + 1]])]
    assert 170 <= len(same) < 200
    for i in sorted(set(range(g1.n)) - set(same)):  # new rows: no self-links, no repeats
        row = g1.col_idx[g1.row_ptr[i]:g1.row_ptr[i + 1]]
        assert len(set(row.tolist())) == len(row) and i not in row


# ------------------------------------------------------------ weighted P

def test_weighted_closed_form_two_nodes():
    """Node 0 keeps 0.7 of its pushes on itself and sends 0.3 to node 1, which
    is dangling: Y0 = (1-d)v0/(1-0.7d), Y1 = (1-d)v1 + 0.3 d Y0."""
    g = wl.from_edges(2, [0, 0], [0, 1])
    w = np.array([0.7, 0.3])  # rows sorted by destination: 0 -> 0, 0 -> 1
    v = np.array([0.25, 0.75])
    Y, _ = oracle.dense_exact_weighted(g, w, D, v)
    y0 = (1 - D) * 0.25 / (1 - 0.7 * D)
    np.testing.assert_allclose(Y, [y0, (1 - D) * 0.75 + 0.3 * D * y0], rtol=1e-14)


def test_weighted_with_uniform_weights_is_the_unweighted_limit():
    g = wl.random_small(60, 300, seed=12, p_dangling=0.2)
    w = 1.0 / np.repeat(np.diff(g.row_ptr), np.diff(g.row_ptr))
    np.testing.assert_allclose(oracle.dense_exact_weighted(g, w, D)[1], oracle.dense_exact(g, D)[1],
                               atol=1e-14)


def test_weighted_set_steps_reach_the_weighted_limit():
    g = wl.random_small(50, 250, seed=13, p_dangling=0.2)
    w = wl.random_weights(g, seed=14)
    F, H = oracle.init_state(g.n, D)
    for _ in range(2000):
        nf = np.abs(F).sum()
        if nf < 1e-14:
            break
        F, H, _ = oracle.set_step_weighted(g, w, D, nf / g.n, F, H)
    np.testing.assert_allclose((H + F) / (H + F).sum(), oracle.dense_exact_weighted(g, w, D)[1],
                               atol=1e-12)


def test_openmp_mat_iter_is_the_sequential_mat_iter():
    """The oracle's OpenMP MAT-ITER (pull over in-links, used for the CPU
    baseline and the large references) takes the same products as the
    sequential push MAT-ITER: same count, iterates equal to rounding, and the
    exact limit at a tight stop -- also with repeated links, self-loops and a
    personalisation vector."""
    g = wl.random_small(500, 4000, seed=11)
    v = np.random.default_rng(2).random(g.n)
    v /= v.sum()
    for vv in (None, v):
        a = oracle.power(g, 0.85, 1e-12, v=vv)
        b = oracle.power_omp(g, 0.85, 1e-12, v=vv)
        assert a["stats"]["rounds"] == b["stats"]["rounds"]
        assert np.abs(a["X"] - b["X"]).max() < 1e-15
        assert b["threads"] >= 1
    y = oracle.power_omp(g, 0.85, 1e-15, v=v)["x"]
    assert np.abs(y - oracle.dense_exact(g, 0.85, v)[1]).sum() < 1e-13
