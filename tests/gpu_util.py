"""Helpers shared by the GPU parity tests (test infrastructure)."""

import numpy as np
import pytest

from paper_1609_04809_amd import workloads as W

EPS64 = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev_full(dim, n, x_int, dtype="float64"):
    """Interior vector -> device tensor in the (n+1)^dim node layout."""
    torch = torch_cuda()
    npdt = np.float64 if dtype == "float64" else np.float32
    full = W.interior_to_full(dim, n, np.asarray(x_int).astype(npdt), dtype=npdt)
    return torch.from_numpy(full).to("cuda")


def host_int(dim, n, t):
    """Device node tensor -> interior numpy vector (float64)."""
    return W.full_to_interior(dim, n, t.detach().cpu().numpy()).astype(np.float64)


def host_full(t):
    return t.detach().cpu().numpy().astype(np.float64)


def assert_scaled_close(got, want, scale, eps, c=64.0, what=""):
    """|got - want| <= c * eps * scale elementwise (a floating-point error
    bound for sums of a few dozen terms whose magnitudes add up to scale)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    err = np.abs(got - want)
    bound = c * eps * scale + 1e-300
    ratio = err / bound
    worst = int(np.argmax(ratio))
    assert ratio[worst] <= 1.0, (
        f"{what}: |err| {err[worst]:.3e} > bound {bound[worst]:.3e} at {worst} "
        f"(got {got[worst]!r}, want {want[worst]!r})")


def boundary_is_zero(dim, n, t):
    a = host_full(t).reshape((n + 1,) * dim)
    inner = np.zeros_like(a, dtype=bool)
    inner[(slice(1, n),) * dim] = True
    return not np.any(a[~inner])
