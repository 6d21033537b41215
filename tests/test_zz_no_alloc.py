"""GPU tests of di_power_solve_noalloc, the power iteration on the library's
fixed device scratch: called through the C ABI and compared with
di_power_solve on the same graphs -- two calls in a row, the second on a
smaller graph -- in both precisions, plus its size limit and argument checks."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
D = 0.85
EPS = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def di():
    import torch
    from paper_1202_6158_amd import di as _di
    torch.cuda.set_device(0)
    return _di


def _pair(di, G, prec, tol, v=None):
    """The same solve by both entry points; returns (x_noalloc, st, x_ref, st_ref)."""
    import torch
    out = torch.full((G.n,), float("nan"), dtype=torch.float64, device="cuda")
    x, st = di.power_solve_noalloc(G, out, v=v, d=D, tol=tol, precision=prec)
    assert x is out
    xr, sr = di.power_solve(G, v=v, d=D, tol=tol, precision=prec)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, xr.cpu().numpy(), sr


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_calls_match_power_solve(di, prec):
    """A call on the 10^6-node benchmark graph (close to the scratch limit in
    fp64), then one on the 10^4-node graph with a personalisation vector: each
    equal to di_power_solve's result within the precision's tolerance, with
    the same number of products, and within its bound of the exact limit."""
    import torch
    tol = 1e-10 if prec == "fp64" else 1e-8
    big = wl.recipe("powerlaw-1m")
    Gb = di.Graph(big)
    xa, sa, xb, sb = _pair(di, Gb, prec, tol)
    assert np.isfinite(xa).all()
    assert sa["rounds"] == sb["rounds"]
    assert sa["residual_l1"] < tol
    assert float(np.abs(xa - xb).sum()) <= EPS[prec]
    del Gb
    small = wl.recipe("pagerank-10k")
    Gs = di.Graph(small)
    rng = np.random.default_rng(5)
    vh = rng.random(small.n)
    vh /= vh.sum()
    v = torch.tensor(vh, dtype=torch.float64, device="cuda")
    xa, sa, xb, sb = _pair(di, Gs, prec, tol, v=v)
    assert sa["rounds"] == sb["rounds"]
    assert float(np.abs(xa - xb).sum()) <= EPS[prec]
    # and against the oracle's exact limit for this V
    xs = oracle.sparse_exact(small, D, v=vh)[1]
    assert float(np.abs(xa - xs).sum()) <= sa["err_bound_l1"] + EPS[prec]


def test_size_limit_and_arguments(di):
    import torch
    n = 1_100_000  # above the fp64 limit of the scratch, below the fp32 one
    G = di.Graph(wl.cycle(n))
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(di.DiError) as e:
        di.power_solve_noalloc(G, out, precision="fp64")
    assert e.value.status == di.EINVAL
    x, st = di.power_solve_noalloc(G, out, d=D, tol=1e-8, precision="fp32")
    assert float(np.abs(x.cpu().numpy() - 1.0 / n).sum()) <= st["err_bound_l1"] + 1e-6
    # host pointers (no DI_DEVICE_PTRS) are refused by the library itself
    small = di.Graph(wl.cycle(8))
    xh = np.zeros(8)
    o = di.make_opts(D, 1e-8, "fp64", True, 0, None, 0)
    st = di.Stats()
    rc = di._lib.di_power_solve_noalloc(small.handle, None, ctypes.byref(o),
                                        ctypes.c_void_p(xh.ctypes.data), ctypes.byref(st), None)
    assert rc == di.EINVAL
    o = di.make_opts(D, 1e-8, "fp64", True, 0, None, di.DEVICE_PTRS | di.TIMING)
    xd = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = di._lib.di_power_solve_noalloc(small.handle, None, ctypes.byref(o), di._ptr(xd),
                                        ctypes.byref(st), None)
    assert rc == di.EINVAL
