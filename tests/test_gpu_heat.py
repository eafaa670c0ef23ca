"""GPU parity of the mass-shifted operator K + sigma M, warm-started solves,
the Crank-Nicolson right-hand side and the Crank-Nicolson time loop of the
heat-equation model problem (Sec. 6.2) with the CPU oracle.

Bars: right-hand sides element by element within 64 eps of the sum of the
magnitudes of their terms; solves as in the Poisson tests (cycle counts
+-1, solutions within 1e-8 relative after equal cycle counts); the time
loop within 1e-9 of the oracle's nodal values (both solve every step to a
1e-10 relative residual); fused/unfused and tail/grid paths bitwise.
"""

import numpy as np
import pytest

import oracle as O
from oracle import heat as OH
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import (EPS64, assert_scaled_close, boundary_is_zero, dev_full, host_full,
                            host_int, torch_cuda)

pytestmark = pytest.mark.gpu

SOLVE_CASES = [
    # dim, n, levels, op, kappa, sigma, prec, flags
    (3, 64, 6, "stencil", False, 200.0, "fp64", 0),
    (3, 48, 5, "stencil", False, 200.0, "fp32_ir", 0),
    (3, 32, 5, "csr", False, 200.0, "fp64", 0),
    (3, 32, 5, "csr", True, 50.0, "fp64", 0),
    (2, 128, 6, "stencil", False, 200.0, "fp64", 0),
    (3, 64, 6, "stencil", False, 200.0, "fp64", "pcg"),
]


def _sid(c):
    return f"{c[0]}d-n{c[1]}-{c[3]}-{'kap' if c[4] else 'poi'}-s{c[5]:g}-{c[6]}-{c[7]}"


def _flags(f):
    from paper_1609_04809_amd.mg import FLAG_PCG
    return FLAG_PCG if f == "pcg" else int(f)


@pytest.mark.parametrize("case", SOLVE_CASES, ids=_sid)
def test_shifted_solve_matches_oracle(case):
    torch_cuda()
    from paper_1609_04809_amd.mg import Solver
    dim, n, levels, op, kap, sigma, prec, fl = case
    kappa = W.kappa_lognormal(dim, n, 31) if kap else None
    b = W.rhs_uniform(dim, n, 32)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, sigma=sigma, fp32=prec == "fp32_ir")
    if fl == "pcg":
        u_or, k_or, hist_or, st_or = O.solve_pcg(H, b, 1e-9)
    elif prec == "fp32_ir":
        u_or, k_or, hist_or, st_or = O.solve_ir(H, b, 1e-9)
    else:
        u_or, k_or, hist_or, st_or = O.solve(H, b, 1e-9)
    assert st_or == "ok"
    with Solver(dim, n, levels, kappa=kappa, op=op, precision=prec, sigma=sigma,
                flags=_flags(fl)) as S:
        u, k, hist, st = S.solve(dev_full(dim, n, b), 1e-9)
        assert st == "ok" and abs(k - k_or) <= 1, (k, k_or)
        kk = min(k, k_or)
        np.testing.assert_allclose(hist[1:kk + 1], hist_or[1:kk + 1], rtol=1e-5, atol=1e-14)
        ug = host_int(dim, n, u)
        rho = np.linalg.norm(b - H.A[0] @ ug) / np.linalg.norm(b)
        assert rho <= 1e-9 * (1 + 1e-6) and abs(rho - hist[k]) <= 1e-6 * rho + 1e-14
        if k == k_or and prec == "fp64":
            assert np.linalg.norm(ug - u_or) <= 1e-8 * np.linalg.norm(u_or)


@pytest.mark.parametrize("dim,n,levels,prec,op,fl", [
    (3, 64, 6, "fp64", "stencil", 0),
    (3, 48, 5, "fp32_ir", "stencil", 0),
    (3, 32, 5, "fp64", "csr", 0),
    (2, 128, 6, "fp64", "stencil", 0),
    (3, 64, 6, "fp64", "stencil", "pcg"),
])
def test_warm_start_matches_oracle(dim, n, levels, prec, op, fl):
    """From a perturbed solution: hist[0] is the initial relative residual,
    the cycle count matches the oracle's warm-started solve, and a start
    that already meets the tolerance returns after zero cycles unchanged."""
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_WARM, Solver
    sigma = 200.0
    b = W.rhs_uniform(dim, n, 41)
    H = O.build_hierarchy(dim, n, levels, sigma=sigma, fp32=prec == "fp32_ir")
    u_star = O.dst_solve(dim, n, b, sigma)
    u0 = u_star + 1e-5 * np.abs(u_star).max() * np.random.default_rng(42).uniform(-1, 1, u_star.size)
    solver = O.solve_pcg if fl == "pcg" else (O.solve_ir if prec == "fp32_ir" else O.solve)
    _, k_or, hist_or, _ = solver(H, b, 1e-10, u0=u0)
    flags = FLAG_WARM | _flags(fl)
    with Solver(dim, n, levels, op=op, precision=prec, sigma=sigma, flags=flags) as S:
        ud = dev_full(dim, n, u0)
        # boundary entries of the start are ignored and come back as 0
        full = ud.view(*((n + 1,) * dim))
        full[(0,) * dim] = 7.0
        u, k, hist, st = S.solve(dev_full(dim, n, b), 1e-10, u=ud)
        assert st == "ok" and abs(k - k_or) <= 1, (k, k_or)
        assert hist[0] == pytest.approx(hist_or[0], rel=1e-9)
        assert boundary_is_zero(dim, n, u)
        ug = host_int(dim, n, u)
        assert np.linalg.norm(ug - u_star) <= 1e-8 * np.linalg.norm(u_star)
        # already converged: zero cycles, u untouched
        before = host_full(u)
        u2, k2, hist2, st2 = S.solve(dev_full(dim, n, b), 1e-6, u=u)
        assert st2 == "ok" and k2 == 0 and len(hist2) == 1 and hist2[0] <= 1e-6
        assert np.array_equal(host_full(u2), before)
        # b = 0: u = 0 after zero cycles
        u3, k3, _, st3 = S.solve(torch.zeros_like(u), 1e-8, u=u)
        assert st3 == "ok" and k3 == 0 and not np.any(host_full(u3))


def test_warm_start_from_zero_equals_cold_start_bitwise():
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_NO_FUSE, FLAG_WARM, Solver
    dim, n, levels = 3, 64, 6
    b = dev_full(dim, n, W.rhs_uniform(dim, n, 43))
    for fl in (0, FLAG_NO_FUSE):
        with Solver(dim, n, levels, sigma=200.0, flags=fl) as S:
            u, k, hist, _ = S.solve(b, 1e-9)
        with Solver(dim, n, levels, sigma=200.0, flags=fl | FLAG_WARM) as S:
            uw, kw, histw, _ = S.solve(b, 1e-9, u=torch.zeros_like(b))
        assert k == kw and hist == histw
        assert np.array_equal(host_full(u), host_full(uw))


def _cn_inputs(dim, n, seed):
    rng = np.random.default_rng(seed)
    N = (n + 1) ** dim
    # u with junk on the boundary (ignored), g0/g1 with junk inside
    # (ignored), F with junk on the boundary (ignored), a guess
    u, g0, g1, F, guess = (rng.uniform(-1, 1, N) for _ in range(5))
    return u, g0, g1, F, guess


@pytest.mark.parametrize("dim,n,levels,op", [(3, 80, 5, "stencil"), (3, 40, 3, "csr"),
                                             (3, 9, 1, "stencil"), (2, 160, 6, "stencil"),
                                             (2, 5, 1, "stencil")])
def test_cn_rhs_matches_oracle(dim, n, levels, op):
    """The plane-marching path with its boundary pass (3D n >= 32: ragged
    tiles, 79 = 64 + 15 and 39 = 32 + 7 unknowns per row), the node kernel
    (a grid where every block touches the boundary, 2D); absent data; the
    extrapolated guess; the load vector M f."""
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import Solver
    sigma = 200.0
    u, g0, g1, F, guess = _cn_inputs(dim, n, 51)
    c0, c1, cf = 0.93, 0.91, 57.3
    KM = O.assemble_full(dim, n)
    K, M = KM
    ui = W.full_to_interior(dim, n, u)
    Fi = W.full_to_interior(dim, n, F)
    want = OH.cn_rhs(dim, n, sigma, ui, g0, c0, g1, c1, Fi, cf, KM)
    # error scale: the terms' magnitudes
    bm = np.ones((n + 1,) * dim, dtype=bool)
    bm[(slice(1, n),) * dim] = False
    bm = bm.ravel()
    ax0 = np.where(bm, abs(c0 * g0), abs(u))
    ax1 = np.where(bm, abs(c1 * g1), 0.0)
    absB = abs(sigma * M) + abs(K)
    # (the boundary pass adds and removes u's boundary values: count them)
    scale_full = absB @ (ax0 + np.where(bm, abs(u), 0.0)) + absB @ ax1
    scale = W.full_to_interior(dim, n, scale_full) + abs(cf * Fi)
    with Solver(dim, n, levels, op=op, sigma=sigma) as S:
        td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
        gd = td(guess)
        b = S.cn_rhs(td(u), td(g0), c0, td(g1), c1, td(F), cf, guess=gd)
        assert_scaled_close(host_int(dim, n, b), want, scale, EPS64, what="cn_rhs")
        assert boundary_is_zero(dim, n, b)
        np.testing.assert_array_equal(host_int(dim, n, gd),
                                      2.0 * ui - W.full_to_interior(dim, n, guess))
        b2 = S.cn_rhs(td(u))
        want2 = OH.cn_rhs(dim, n, sigma, ui, None, 0, None, 0, None, 0, KM)
        assert_scaled_close(host_int(dim, n, b2), want2, scale, EPS64, what="cn_rhs no data")
        # load vector of nodal values
        f = np.random.default_rng(52).uniform(-1, 1, (n + 1) ** dim)
        Fd = S.mass(td(f))
        assert_scaled_close(host_int(dim, n, Fd), OH.load_vector(dim, n, f, KM),
                            W.full_to_interior(dim, n, abs(M) @ abs(f)), EPS64, what="mass")
        assert boundary_is_zero(dim, n, Fd)


@pytest.mark.parametrize("extrapolate", [False, True])
def test_cn_time_loop_matches_oracle(extrapolate):
    """Ten Crank-Nicolson steps of the model problem on 64^3 cells
    (warm-started V(3,3) solves to 1e-10, from u^n or from 2 u^n - u^{n-1})
    against the oracle's loop, and the error against the paper's exact
    solution."""
    torch_cuda()
    from paper_1609_04809_amd.heat import HeatRun
    w = W.HEAT_WORKLOADS["heat3d_64_cn"]
    s, u0 = W.heat_inputs(w)
    tol = 1e-10
    H = O.build_hierarchy(w.dim, w.n, w.levels, sigma=w.sigma, nu_pre=w.nu_pre,
                          nu_post=w.nu_post)
    u_or, its_or, _ = OH.run(H, w.dt, w.steps, u0, s, W.heat_gamma, s,
                             lambda t: W.heat_lambda(w.dim, t), tol, extrapolate=extrapolate)
    with HeatRun(w, tol=tol, extrapolate=extrapolate) as R:
        R.reset()
        its = R.run(w.steps)
        u = host_int(w.dim, w.n, R.u)
    assert all(abs(a - b) <= 1 for a, b in zip(its, its_or)), (its, its_or)
    assert np.abs(u - u_or).max() <= 1e-9 * np.abs(u_or).max()
    exact = W.heat_gamma(w.steps * w.dt) * u0
    assert np.abs(u - exact).max() <= 2e-4


def test_mass_shift_fused_and_tail_paths_agree_bitwise():
    """Head fusion, the prolongation fused into the first post-smoothing
    step and the one-workgroup tail give bitwise what separate launches
    give, for the face-coupled 3D operator."""
    torch_cuda()
    from paper_1609_04809_amd.mg import FLAG_NO_FUSE, FLAG_NO_TAIL, Solver
    dim, n, levels = 3, 64, 6
    b = dev_full(dim, n, W.rhs_uniform(dim, n, 61))
    outs = []
    for fl in (0, FLAG_NO_FUSE, FLAG_NO_TAIL, FLAG_NO_FUSE | FLAG_NO_TAIL):
        with Solver(dim, n, levels, sigma=200.0, nu_pre=3, nu_post=3, flags=fl) as S:
            u, k, hist, st = S.solve(b, 1e-10)
            assert st == "ok"
            outs.append((k, hist, host_full(u)))
    for a in range(1, 4):
        assert outs[a][0] == outs[0][0] and outs[a][1] == outs[0][1], a
        assert np.array_equal(outs[a][2], outs[0][2]), a


def test_full_size_cn_steps_on_sampled_nodes():
    """The 512^3 workload at its full size, as the benchmark runs it: two
    steps; the right-hand side on sampled unknowns against the oracle's
    per-row evaluation, and each step's relative residual recomputed on the
    host."""
    torch = torch_cuda()
    from paper_1609_04809_amd.heat import HeatRun
    w = W.HEAT_WORKLOADS["heat3d_512_cn"]
    n, dim = w.n, w.dim
    s, u0 = W.heat_inputs(w)
    rng = np.random.default_rng(71)
    nodes = rng.integers(1, n, size=(2000, 3))
    nodes[:8] = [[1, 1, 1], [n - 1, n - 1, n - 1], [1, n - 1, 5], [n - 1, 1, n - 1],
                 [2, 2, 2], [n // 2, n // 2, 1], [255, 256, 257], [64, 192, 511]]
    idx = nodes[:, 0] + (n + 1) * (nodes[:, 1] + (n + 1) * nodes[:, 2])
    sig = w.sigma
    with HeatRun(w, tol=w.tol, extrapolate=True) as R:
        R.reset()
        for step in range(3):
            t0, t1 = step * w.dt, (step + 1) * w.dt
            u_prev = host_full(R.u)
            R.step()
            b = host_full(R.b)
            # oracle rows: (sigma M - K) x0 - (sigma M + K) x1 + cf M f with
            # x0 = u_prev inside / gamma0 s on the boundary, x1 = gamma1 s
            x0 = u_prev.copy()
            bmask = np.ones((n + 1,) * 3, dtype=bool)
            bmask[1:n, 1:n, 1:n] = False
            bmask = bmask.ravel()
            x0[bmask] = W.heat_gamma(t0) * s[bmask]
            x1 = np.where(bmask, W.heat_gamma(t1) * s, 0.0)
            cf = W.heat_lambda(dim, t0) + W.heat_lambda(dim, t1)
            want = (_rows_full(dim, n, nodes, x0, sig, -1.0)
                    - _rows_full(dim, n, nodes, x1, sig, 1.0)
                    + cf * _rows_full(dim, n, nodes, s, 1.0, 0.0))
            got = b[idx]
            assert np.abs(got - want).max() <= 1e-11 * np.abs(b).max(), step
            rel = R.last_hist[-1]
            assert rel <= w.tol


def _rows_full(dim, n, nodes, x, alpha, beta):
    """(alpha M + beta K) x at interior nodes, boundary values included,
    cell by cell from the element matrices."""
    h = 1.0 / n
    Ke = O.element_matrix(dim, h)
    Me = O.element_mass(dim, h)
    E = alpha * Me + beta * Ke
    X = np.asarray(x).reshape((n + 1,) * dim)
    verts = [tuple((a >> d) & 1 for d in range(dim)) for a in range(2 ** dim)]
    out = np.zeros(len(nodes))
    for a, v in enumerate(verts):
        cell = nodes - np.array(v)
        for bb, ww in enumerate(verts):
            q = cell + np.array(ww)
            out += E[a, bb] * X[q[:, 2], q[:, 1], q[:, 0]]
    return out


def test_server_refuses_mass_shift_and_warm_start():
    torch_cuda()
    from paper_1609_04809_amd import mg
    srv = mg.Server(1 << 30, 4)
    try:
        b = np.ones(17 ** 3)
        for kw in (dict(sigma=1.0), dict(flags=mg.FLAG_WARM)):
            with pytest.raises(mg.MgError):
                srv.submit(3, 16, 3, b, 1e-8, **kw)
    finally:
        srv.close()
