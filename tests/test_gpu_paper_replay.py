"""The paper's six simulation scenarios (Section 4.1) on the GPU: the threshold
D-iteration matches the exact limit within its bound and diffuses fewer links
than the GPU power iteration uses (L per product) at the same stop rule --
the paper's qualitative result, on the kernels of this library."""
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


@pytest.mark.parametrize("name", list(wl.PAPER_SCENARIOS))
def test_paper_scenario_on_gpu(di, name):
    g = wl.paper_scenario(name)
    G = di.Graph(g)
    x, st = di.solve(G, d=D, tol=1e-10, precision="fp64")
    xp, sp = di.power_solve(G, d=D, tol=1e-10, precision="fp64")
    xs = oracle.limit(g, D, tol=1e-14)
    assert float(np.abs(x.cpu().numpy() - xs).sum()) <= st["err_bound_l1"] + 1e-12
    assert float(np.abs(xp.cpu().numpy() - xs).sum()) <= sp["err_bound_l1"] + 1e-12
    assert st["edges_diffused"] < sp["rounds"] * g.m
