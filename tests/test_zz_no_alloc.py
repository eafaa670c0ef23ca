"""mg_solve_noalloc (the solve that allocates no device memory) against the
context-based mg_setup + mg_solve on the same inputs, through the C ABI:
two calls in a row, the second on a smaller problem, and a variable-kappa
and a 3D case.  Bar: the same cycle count, bitwise the same iterate (the
two run the same cycles), histories equal to rounding (1e-12 relative).
"""

import numpy as np
import pytest

from paper_1609_04809_amd import workloads as W
from tests.gpu_util import dev_full, host_full, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, levels, smoother, kappa, cycle, sigma, tol
    (2, 64, 5, "jacobi", False, "V", 0.0, 1e-10),   # the 2D 64^2 Jacobi workload's shape
    (2, 32, 4, "rbgs", True, "V", 0.0, 1e-8),       # smaller, second in a row
    (3, 16, 4, "rbgs", False, "W", 0.0, 1e-8),
    (3, 8, 3, "rbgs", True, "F", 0.0, 1e-8),
    (3, 8, 3, "rbgs", False, "V", 50.0, 1e-8),
]


def _reference(dim, n, levels, sm, kappa_d, cycle, sigma, bd, tol):
    from paper_1609_04809_amd.mg import Solver
    with Solver(dim, n, levels, kappa=kappa_d, smoother=sm, cycle=cycle, sigma=sigma) as S:
        return S.solve(bd, tol)


def test_noalloc_matches_context_solve_on_consecutive_calls():
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import solve_noalloc
    for q, (dim, n, levels, sm, kap, cycle, sigma, tol) in enumerate(CASES):
        print(f"[noalloc] case {q}: dim {dim} n {n} levels {levels} {sm} kappa {kap}",
              flush=True)
        kappa = W.kappa_lognormal(dim, n, 40 + q) if kap else None
        kd = None if kappa is None else torch.from_numpy(kappa).to("cuda")
        bd = dev_full(dim, n, W.rhs_uniform(dim, n, 50 + q))
        u_ref, k_ref, h_ref, st_ref = _reference(dim, n, levels, sm, kd, cycle, sigma, bd, tol)
        u = torch.full_like(bd, 7.0)       # every node is written
        u, k, hist, st = solve_noalloc(dim, n, levels, bd, tol, u=u, kappa=kd, smoother=sm,
                                       cycle=cycle, sigma=sigma)
        torch.cuda.synchronize()
        assert st == st_ref == "ok" and k == k_ref, (st, st_ref, k, k_ref)
        np.testing.assert_allclose(hist, h_ref, rtol=1e-12, atol=0)
        assert np.array_equal(host_full(u), host_full(u_ref))


def test_noalloc_edge_cases():
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import MgError, solve_noalloc
    dim, n, levels = 2, 64, 5
    bd = dev_full(dim, n, W.rhs_uniform(dim, n, 3))
    u, k, hist, st = solve_noalloc(dim, n, levels, bd, 1e-300, max_iter=3)
    assert st == "maxit" and k == 3 and len(hist) == 4
    z = torch.zeros_like(bd)
    u, k, hist, st = solve_noalloc(dim, n, levels, z, 1e-8)
    assert st == "ok" and k == 0 and hist == [1.0] and not torch.any(u)
    bn = bd.clone()
    bn[5 + 65 * 6] = float("nan")
    with pytest.raises(MgError) as e:
        solve_noalloc(dim, n, levels, bn, 1e-8)
    assert e.value.status == 7
    with pytest.raises(MgError) as e:                 # too large for one workgroup
        solve_noalloc(2, 128, 6, dev_full(2, 128, W.rhs_uniform(2, 128, 0)), 1e-8)
    assert e.value.status == 1
