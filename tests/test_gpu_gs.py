"""GPU parity of the multicolour (2^d-colour) Gauss-Seidel smoother with the
CPU oracle: single colour steps element by element, whole solves (cycle
counts +-1, solutions within 1e-8 relative after equal counts), the
FP32-inner form, CG with the symmetric Gauss-Seidel cycle, and the coarse
levels cycled in one workgroup against level-by-level launches (bitwise).
"""

import numpy as np
import pytest

import oracle as O
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import (EPS32, EPS64, assert_scaled_close, boundary_is_zero, dev_full,
                            host_full, host_int, torch_cuda)

pytestmark = pytest.mark.gpu

STEP_CASES = [
    # dim, n, levels, kappa, op, sigma
    (3, 40, 3, False, "stencil", 0.0),
    (3, 40, 3, True, "stencil", 0.0),
    (3, 40, 3, False, "stencil", 200.0),
    (3, 40, 3, True, "csr", 0.0),
    (2, 96, 4, True, "stencil", 0.0),
    (2, 96, 4, False, "csr", 0.0),
]


def _cid(c):
    return (f"{c[0]}d-n{c[1]}-{'kap' if c[3] else 'poi'}-{c[4]}"
            + (f"-sigma{c[5]:g}" if c[5] else ""))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", STEP_CASES, ids=_cid)
def test_gs_colour_steps_match_oracle(case, prec):
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import STEP_GS0, Solver
    dim, n, levels, kap, op, sigma = case
    kappa = W.kappa_lognormal(dim, n, 13) if kap else None
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother="gs", fp32=True, sigma=sigma)
    tdt = "float64" if prec == "fp64" else "float32"
    eps = EPS64 if prec == "fp64" else EPS32
    rng = np.random.default_rng(17)
    with Solver(dim, n, levels, kappa=kappa, op=op, smoother="gs", precision="fp32_ir",
                sigma=sigma) as S:
        for l in (0, 1):
            nl = H.nl[l]
            A = H.A[l] if prec == "fp64" else H.A32[l].astype(np.float64)
            d = H.diag[l] if prec == "fp64" else H.diag32[l].astype(np.float64)
            N = (nl - 1) ** dim
            rnd = lambda v: v if prec == "fp64" else v.astype(np.float32).astype(np.float64)
            x, b = rnd(rng.uniform(-1, 1, N)), rnd(rng.uniform(-1, 1, N))
            xd, bd = dev_full(dim, nl, x, tdt), dev_full(dim, nl, b, tdt)
            out = torch.empty_like(xd)
            scale = abs(x) + (abs(A) @ abs(x) + abs(b)) / d
            for c in range(2 ** dim):
                S.smooth(l, STEP_GS0 + c, xd, bd, out)
                sel = H.colours[l] == c
                want = O.mg.gs_colour_step(A, d, x, b, sel)
                got = host_int(dim, nl, out)
                assert_scaled_close(got, want, scale, eps, what=f"gs colour {c} l{l}")
                np.testing.assert_array_equal(got[~sel], x[~sel])
                assert boundary_is_zero(dim, nl, out)


SOLVE_CASES = [
    # dim, n, levels, op, kappa, prec, method
    (3, 64, 6, "stencil", False, "fp64", "cycle"),
    (3, 32, 5, "csr", False, "fp64", "cycle"),
    (3, 48, 5, "stencil", True, "fp64", "cycle"),
    (2, 128, 6, "stencil", False, "fp64", "cycle"),
    (3, 64, 6, "stencil", False, "fp32_ir", "cycle"),
    (3, 32, 5, "csr", True, "fp64", "pcg"),
]


@pytest.mark.parametrize("case", SOLVE_CASES,
                         ids=lambda c: f"{c[0]}d-n{c[1]}-{c[3]}-{'kap' if c[4] else 'poi'}-{c[5]}-{c[6]}")
def test_gs_solve_matches_oracle(case):
    torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_PCG, Solver
    dim, n, levels, op, kap, prec, method = case
    kappa = W.kappa_lognormal(dim, n, 19) if kap else None
    b = W.rhs_ones_load(dim, n) if kap else W.rhs_uniform(dim, n, 23)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother="gs", fp32=prec == "fp32_ir")
    if method == "pcg":
        u_or, k_or, hist_or, st_or = O.solve_pcg(H, b, 1e-8)
    elif prec == "fp32_ir":
        u_or, k_or, hist_or, st_or = O.solve_ir(H, b, 1e-8)
    else:
        u_or, k_or, hist_or, st_or = O.solve(H, b, 1e-8)
    assert st_or == "ok"
    with Solver(dim, n, levels, kappa=kappa, op=op, smoother="gs", precision=prec,
                flags=FLAG_PCG if method == "pcg" else 0) as S:
        u, k, hist, st = S.solve(dev_full(dim, n, b), 1e-8)
        assert st == "ok" and abs(k - k_or) <= 1, (k, k_or)
        kk = min(k, k_or)
        np.testing.assert_allclose(hist[1:kk + 1], hist_or[1:kk + 1], rtol=1e-6, atol=1e-14)
        ug = host_int(dim, n, u)
        rho = np.linalg.norm(b - H.A[0] @ ug) / np.linalg.norm(b)
        assert rho <= 1e-8 * (1 + 1e-6)
        if k == k_or and prec == "fp64":
            assert np.linalg.norm(ug - u_or) <= 1e-8 * np.linalg.norm(u_or)


@pytest.mark.parametrize("dim,n,levels,kap,prec", [
    (3, 64, 6, False, "fp64"),
    (3, 32, 5, True, "fp32_ir"),
    (2, 128, 6, False, "fp64"),
])
def test_gs_tail_and_grid_levels_agree_bitwise(dim, n, levels, kap, prec):
    torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_NO_TAIL, Solver
    kappa = W.kappa_lognormal(dim, n, 29) if kap else None
    b = dev_full(dim, n, W.rhs_uniform(dim, n, 31))
    outs = []
    for flags in (0, FLAG_NO_TAIL):
        with Solver(dim, n, levels, kappa=kappa, smoother="gs", precision=prec,
                    flags=flags) as S:
            u, k, hist, st = S.solve(b, 1e-8)
            assert st == "ok"
            outs.append((k, hist, host_full(u)))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2])


def test_gs_refusals():
    torch = torch_cuda()
    from paper_1609_04809_amd import mg
    with mg.Solver(3, 16, 3, op="csr") as S:     # rows blocked red-black
        x = torch.zeros(17 ** 3, dtype=torch.float64, device="cuda")
        with pytest.raises(mg.MgError):
            S.smooth(0, mg.STEP_GS0, x, x.clone(), torch.empty_like(x))
    srv = mg.Server(1 << 30, 4)
    try:
        with pytest.raises(mg.MgError):
            srv.submit(3, 16, 3, np.ones(17 ** 3), 1e-8, smoother="gs")
    finally:
        srv.close()
