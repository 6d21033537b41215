"""Replay of the paper's simulation experiments on the CPU oracle: its graph
generator at the six scenarios of Section 4.1 (checked against the dangling
counts its tables print), and its qualitative result -- every D-iteration
order (PER, RAND, MAX, the threshold sweep, OP) reaches the target error with
fewer elementary steps (out-links used) than MAT-ITER (L per product).  The
paper's figures are not available, so no curve is matched point by point."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl

D = 0.85
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_scenarios.json")))


@pytest.mark.parametrize("name", list(wl.PAPER_SCENARIOS))
def test_generator_matches_the_papers_tables(name):
    ref = GOLDEN["scenarios"][name]
    assert wl.PAPER_SCENARIOS[name] == (ref["N"], ref["alpha"], ref["L"])
    g = wl.paper_scenario(name)
    assert g.n == ref["N"] and g.m == ref["L"]
    assert abs(g.n_dangling - ref["D"]) <= max(0.03 * ref["D"], 20), (g.n_dangling, ref["D"])
    src, dst = g.edges()
    assert not np.any(src == dst)
    assert len(np.unique(src.astype(np.int64) * g.n + dst)) == g.m


@pytest.mark.parametrize("name", list(wl.PAPER_SCENARIOS))
def test_diteration_orders_need_fewer_elementary_steps_than_mat_iter(name):
    g = wl.paper_scenario(name)
    tol = 1e-8
    p = oracle.power(g, D, tol)
    assert p["converged"]
    mat_iter_steps = p["stats"]["rounds"] * g.m
    xs = oracle.limit(g, D, tol=1e-14)
    for order in ["per", "rand", "max", "sweep", "op"]:
        r = oracle.diter(g, D, tol, order=order)
        assert r["converged"]
        assert r["stats"]["edges"] < mat_iter_steps, (order, r["stats"]["edges"], mat_iter_steps)
        # same accuracy: both within their bounds of the limit
        assert np.abs(r["x"] - xs).sum() <= 2 * D * tol / ((1 - D) * (r["H"] + r["F"]).sum()) + 1e-12
