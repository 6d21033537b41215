"""The Python binding rejects tensors that do not match what the C ABI will
read or write (dtype against the precision, element count, device,
contiguity) with a ValueError, before any library call -- so these checks run
without a GPU, on a stand-in graph object that would fail if it were ever
passed to the library."""
import types

import numpy as np
import pytest
import torch

from paper_1202_6158_amd import di

N = 16
G = types.SimpleNamespace(n=N, handle=None)  # never reaches the library


def _cpu(dtype, n=N):
    return torch.zeros(n, dtype=dtype)


def _fake_cuda(dtype, n=N, contiguous=True):
    """A CPU tensor that claims to be on a CUDA device (enough for checks that
    stop before any device use)."""
    t = torch.zeros(n * (2 if not contiguous else 1), dtype=dtype)
    if not contiguous:
        t = t[::2]

    class T(torch.Tensor):
        @property
        def is_cuda(self):
            return True
    return t.as_subclass(T)


def test_state_dtype_must_match_precision():
    with pytest.raises(ValueError, match="state F"):
        di.solve(G, precision="fp32", state=(_fake_cuda(torch.float64), _fake_cuda(torch.float64)))
    with pytest.raises(ValueError, match="state F"):
        di.solve(G, precision="fp64", state=(_fake_cuda(torch.float32), _fake_cuda(torch.float64)))
    with pytest.raises(ValueError, match="state H"):
        di.solve(G, precision="fp32", state=(_fake_cuda(torch.float32), _fake_cuda(torch.float32)))


def test_state_size_device_and_layout():
    with pytest.raises(ValueError, match="elements"):
        di.solve(G, precision="fp32", state=(_fake_cuda(torch.float32, N - 1),
                                             _fake_cuda(torch.float64)))
    with pytest.raises(ValueError, match="CUDA"):
        di.solve(G, precision="fp32", state=(_cpu(torch.float32), _cpu(torch.float64)))
    with pytest.raises(ValueError, match="contiguous"):
        di.solve(G, precision="fp32", state=(_fake_cuda(torch.float32, contiguous=False),
                                             _fake_cuda(torch.float64)))


def test_out_tensors_checked():
    with pytest.raises(ValueError, match="out"):
        di.solve(G, out=_fake_cuda(torch.float32))
    with pytest.raises(ValueError, match="out"):
        di.power_solve(G, out=_fake_cuda(torch.float64, N + 1))
    with pytest.raises(ValueError, match="out"):
        di.solve(G, out=np.zeros(N, dtype=np.float32), host=True)
    with pytest.raises(ValueError, match="out"):
        di.solve_batch(G, [0, 1, 2], [0, 1], out=_fake_cuda(torch.float64, N))
    with pytest.raises(ValueError, match="out"):
        di.solve_batch(G, [0, 1, 2], [0, 1], out=np.zeros(N, dtype=np.float64), host=True)


def test_vectors_and_rounds_checked():
    with pytest.raises(ValueError, match="v"):
        di.solve(G, v=np.ones(N - 1) / (N - 1), host=True)
    with pytest.raises(ValueError, match="F"):
        di.diffuse_round(G, _fake_cuda(torch.float32, N - 2), _fake_cuda(torch.float64), 0.0)
    with pytest.raises(ValueError, match="H"):
        di.diffuse_round(G, _fake_cuda(torch.float32), _fake_cuda(torch.float32), 0.0)
    with pytest.raises(ValueError, match="F"):
        di.diffuse_round(G, _fake_cuda(torch.int32), _fake_cuda(torch.float64), 0.0)
    other = types.SimpleNamespace(n=N + 1, handle=None)
    with pytest.raises(ValueError, match="same number"):
        di.inject_update(G, other, _fake_cuda(torch.float32), _fake_cuda(torch.float64))
    with pytest.raises(ValueError, match="H"):
        di.inject_update(G, G, _fake_cuda(torch.float32), _fake_cuda(torch.float64, N - 1))
    with pytest.raises(ValueError, match="precision"):
        di.solve(G, precision="bf16")
