"""The C ABI used from C alone: examples/pagerank_edges (built with the
library) reads an edge list, solves with host buffers through di_solve and
di_power_solve, and prints the largest entries; they must match the oracle's
exact PageRank within the reported bounds.  The CPU test only checks that
the program is built and reports its usage without touching a device."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1202_6158_amd", "examples", "pagerank_edges")


def test_example_is_built_and_prints_usage():
    assert os.path.exists(EXE), "build() compiles examples/pagerank_edges.c"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


@pytest.mark.gpu
def test_example_matches_the_oracle(tmp_path):
    g = wl.recipe("pagerank-10k")
    src, dst = g.edges()
    path = tmp_path / "edges.txt"
    np.savetxt(path, np.stack([src, dst], axis=1), fmt="%d")
    # n = the largest id in the list + 1; the oracle graph is built from the same list
    r = subprocess.run([EXE, str(path), "0.85", "1e-12", "20"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [ln.split() for ln in r.stdout.splitlines()]
    rec = {ln[0]: ln for ln in lines if ln[0] != "top"}
    n = int(rec["n"][1])
    xs = oracle.dense_exact(wl.from_edges(n, src, dst), 0.85)[1] if n <= 2000 else \
        oracle.sparse_exact(wl.from_edges(n, src, dst), 0.85)[1]
    assert float(rec["diter"][6]) < 1e-12  # residual
    bound_d, bound_p = float(rec["diter"][8]), float(rec["power"][6])
    tops = [ln for ln in lines if ln[0] == "top"]
    assert len(tops) == 20
    ids = np.array([int(t[2]) for t in tops])
    xd = np.array([float(t[3]) for t in tops])
    xp = np.array([float(t[4]) for t in tops])
    assert np.all(np.diff(xd) <= 0)
    assert np.all(np.abs(xd - xs[ids]) <= bound_d + 1e-12)
    assert np.all(np.abs(xp - xs[ids]) <= bound_p + 1e-12)
    assert float(rec["l1"][1]) <= bound_d + bound_p + 1e-12
