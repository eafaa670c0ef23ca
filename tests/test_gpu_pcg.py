"""Parity of multigrid-preconditioned conjugate gradients (MG_FLAG_PCG) with
the CPU oracle's solve_pcg.

Bar for FP64: the same number of CG iterations (+-1), residual histories
within 1e-6 relative (+1e-14 absolute), and after the same number of
iterations ||u_gpu - u_oracle|| <= 1e-8 ||u_oracle||.  With the FP32
preconditioning cycle: the oracle's iteration count +-1, the true residual
of the returned u (recomputed by the oracle) <= tol, and the distance to
the oracle's FP64 CG solution <= 1e-6 relative.
"""

import numpy as np
import pytest

import oracle as O
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import dev_full, host_full, host_int, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, levels, smoother, op, kappa, tol
    (2, 64, 5, "jacobi", "stencil", False, 1e-10),     # whole cycle inside one workgroup
    (2, 128, 6, "rbgs", "stencil", True, 1e-8),
    (3, 32, 5, "rbgs", "stencil", False, 1e-8),
    (3, 32, 5, "rbgs", "csr", False, 1e-8),
    (3, 48, 5, "rbgs", "stencil", True, 1e-8),
    (3, 48, 5, "rbgs", "csr", True, 1e-8),
    (3, 64, 6, "jacobi", "stencil", True, 1e-8),
]


def _ids(c):
    return f"{c[0]}d-n{c[1]}-{c[3]}-{c[4]}-{'kap' if c[5] else 'poi'}"


def _solver(dim, n, levels, kappa, op, sm, prec, flags=0):
    from paper_1609_04809_amd.mg import FLAG_PCG, Solver
    return Solver(dim, n, levels, kappa=kappa, op=op, smoother=sm, precision=prec,
                  flags=FLAG_PCG | flags)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_fp64_pcg_matches_oracle(case):
    torch_cuda()
    dim, n, levels, sm, op, kap, tol = case
    kappa = W.kappa_lognormal(dim, n, 31) if kap else None
    b = W.rhs_uniform(dim, n, 4)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother=sm)
    u_or, k_or, hist_or, st_or = O.solve_pcg(H, b, tol)
    assert st_or == "ok"
    _, k_st, _, _ = O.solve(H, b, tol)
    assert k_or <= k_st
    bd = dev_full(dim, n, b)
    with _solver(dim, n, levels, kappa, op, sm, "fp64") as S:
        u, k, hist, st = S.solve(bd, tol)
        assert st == "ok" and abs(k - k_or) <= 1, (k, k_or)
        kk = min(k, k_or)
        np.testing.assert_allclose(hist[1:kk + 1], hist_or[1:kk + 1], rtol=1e-6, atol=1e-14)
        if k != k_or:
            u_or, _, _, _ = O.solve_pcg(H, b, 1e-300, max_iter=k)
        ug = host_int(dim, n, u)
        assert np.linalg.norm(ug - u_or) <= 1e-8 * np.linalg.norm(u_or)
        rho = np.linalg.norm(b - H.A[0] @ ug) / np.linalg.norm(b)
        assert rho <= tol * (1 + 1e-5)
        assert not np.any(host_full(u).reshape((n + 1,) * dim)[(0,) * dim])
        # deterministic run to run, and a second solve starts clean
        u2, k2, hist2, _ = S.solve(bd, tol)
        assert k2 == k and hist2 == hist
        assert np.array_equal(host_full(u2), host_full(u))


@pytest.mark.parametrize("case", [c for c in CASES if c[3] == "rbgs"], ids=_ids)
def test_fp32_cycle_pcg_matches_oracle(case):
    torch_cuda()
    dim, n, levels, sm, op, kap, tol = case
    kappa = W.kappa_lognormal(dim, n, 31) if kap else None
    b = W.rhs_uniform(dim, n, 4)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother=sm, fp32=True)
    u32, k32, _, st32 = O.solve_pcg(H, b, tol, fp32=True)
    u64, _, _, _ = O.solve_pcg(H, b, tol)
    assert st32 == "ok"
    with _solver(dim, n, levels, kappa, op, sm, "fp32_ir") as S:
        u, k, hist, st = S.solve(dev_full(dim, n, b), tol)
    assert st == "ok" and abs(k - k32) <= 1, (k, k32)
    ug = host_int(dim, n, u)
    rho = np.linalg.norm(b - H.A[0] @ ug) / np.linalg.norm(b)
    assert rho <= tol * (1 + 1e-5), rho
    assert np.linalg.norm(ug - u64) <= 1e-6 * np.linalg.norm(u64)


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_pcg_graph_and_eager_agree_bitwise(prec):
    torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_NO_GRAPH
    dim, n = 3, 32
    kappa = W.kappa_lognormal(dim, n, 2)
    bd = dev_full(dim, n, W.rhs_uniform(dim, n, 9))
    outs = []
    for flags in (0, FLAG_NO_GRAPH):
        with _solver(dim, n, 5, kappa, "stencil", "rbgs", prec, flags) as S:
            u, k, hist, st = S.solve(bd, 1e-8)
            assert st == "ok"
            outs.append((k, hist, host_full(u)))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2])


def test_pcg_zero_rhs_and_nonfinite():
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import MgError
    dim, n = 3, 16
    with _solver(dim, n, 4, None, "stencil", "rbgs", "fp64") as S:
        bd = torch.zeros((n + 1) ** 3, dtype=torch.float64, device="cuda")
        u, k, hist, st = S.solve(bd, 1e-8)
        assert st == "ok" and k == 0 and not torch.any(u != 0)
        b = W.rhs_uniform(dim, n, 1)
        b[100] = np.nan
        with pytest.raises(MgError):
            S.solve(dev_full(dim, n, b), 1e-8)


def test_full_size_variable_kappa_pcg_meets_tolerance():
    """192^3 variable kappa with the FP32 preconditioning cycle: the oracle's
    cell-by-cell operator recomputes the residual of the returned u, and CG
    needs fewer iterations than the plain cycle iteration."""
    torch_cuda()
    from paper_1609_04809_amd.mg import Solver
    w = W.WORKLOADS["kappa3d_192_rbgs_ir"]
    b, kappa = W.workload_inputs(w)
    bd = dev_full(w.dim, w.n, b)
    with _solver(w.dim, w.n, w.levels, kappa, "stencil", "rbgs", "fp32_ir") as S:
        u, k, hist, st = S.solve(bd, w.tol)
    assert st == "ok"
    with Solver(w.dim, w.n, w.levels, kappa=kappa, precision="fp32_ir") as S:
        _, k_st, _, _ = S.solve(bd, w.tol)
    assert k < k_st, (k, k_st)
    Au = O.apply_matfree(w.dim, w.n, kappa, host_full(u).reshape((w.n + 1,) * w.dim))
    r = b - O.to_interior(w.dim, w.n, Au)
    rho = np.linalg.norm(r) / np.linalg.norm(b)
    assert rho <= w.tol * (1 + 1e-5), rho
