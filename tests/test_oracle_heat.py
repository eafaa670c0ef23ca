"""Pins of the oracle's mass-shifted operator, warm-started solves and
Crank-Nicolson time loop (the heat-equation model problem of Sec. 6.2)
against facts fixed by the mathematics, not by the oracle itself.

What a plausible mistake would break:
* a wrong mass factor, index or tensor order: the quadrature element, the
  exact integrals of Q1 functions, the sine-basis eigenvalues;
* a wrong sign or a swapped time level in the right-hand side or the
  Dirichlet lifting: the exactly reproduced linear-in-time solution and
  the exact amplification of a sine mode;
* a wrong source scaling or initial state: second-order convergence to the
  paper's exact solution;
* warm-start bookkeeping: zero cycles from the solution, identical
  histories from a zero start.
"""

import itertools

import numpy as np
import pytest

import oracle as O
from oracle import heat as OH
from paper_1609_04809_amd import workloads as W


# ---------------------------------------------------------------- element

def _mass_by_quadrature(dim, h, q=3):
    """int phi_a phi_b over [0,h]^d by Gauss quadrature, basis evaluated
    point by point."""
    xi, wq = np.polynomial.legendre.leggauss(q)
    xi, wq = 0.5 * (xi + 1.0), 0.5 * wq
    verts = [tuple((a >> d) & 1 for d in range(dim)) for a in range(2 ** dim)]
    M = np.zeros((2 ** dim, 2 ** dim))
    for pt in itertools.product(range(q), repeat=dim):
        s = [xi[p] for p in pt]
        w = np.prod([wq[p] for p in pt]) * h ** dim
        phi = [np.prod([s[d] if v[d] else 1.0 - s[d] for d in range(dim)]) for v in verts]
        M += w * np.outer(phi, phi)
    return M


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("h", [1.0, 0.25])
def test_element_mass_matches_quadrature(dim, h):
    M = O.element_mass(dim, h)
    np.testing.assert_allclose(M, _mass_by_quadrature(dim, h), rtol=0, atol=1e-15)
    # the basis is a partition of unity: all entries sum to the cell volume
    assert M.sum() == pytest.approx(h ** dim, rel=1e-14)


# ---------------------------------------------------------------- global

def _nodal(dim, n, fn):
    c = np.arange(n + 1) / n
    grids = np.meshgrid(*[c] * dim, indexing="ij")      # [z, y, x] or [y, x]
    xyz = list(reversed(grids))
    return fn(*xyz).ravel()


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 4)])
def test_full_mass_and_stiffness_integrate_q1_functions(dim, n):
    # u, v in the Q1 space are represented exactly by their nodal values,
    # so u^T M v = int u v and u^T K u = int |grad u|^2
    K, M = O.assemble_full(dim, n)
    if dim == 2:
        u = _nodal(2, n, lambda x, y: 1.0 + x)
        v = _nodal(2, n, lambda x, y: x * y)
        exact_uv = 5.0 / 12.0                      # int (1+x) x y
        lin = _nodal(2, n, lambda x, y: x - 3.0 * y)
        exact_grad = 10.0
    else:
        u = _nodal(3, n, lambda x, y, z: 1.0 + x)
        v = _nodal(3, n, lambda x, y, z: y * z)
        exact_uv = 3.0 / 8.0                       # int (1+x) y z
        lin = _nodal(3, n, lambda x, y, z: x + 2.0 * y - 3.0 * z)
        exact_grad = 14.0
    assert u @ (M @ v) == pytest.approx(exact_uv, rel=1e-13)
    assert np.ones(u.size) @ (M @ np.ones(u.size)) == pytest.approx(1.0, rel=1e-13)
    assert lin @ (K @ lin) == pytest.approx(exact_grad, rel=1e-13)
    np.testing.assert_allclose(K @ np.ones(u.size), 0.0, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_shifted_operator_matches_sine_diagonalisation(dim, n):
    # K + sigma M on the unknowns against the DST-I route, which is built
    # from the 1D closed-form eigenvalues only
    sigma = 200.0
    b = np.random.default_rng(3).uniform(-1, 1, (n - 1) ** dim)
    A = O.assemble(dim, n, sigma=sigma)
    np.testing.assert_allclose(O.sparse_solve(A, b), O.dst_solve(dim, n, b, sigma),
                               rtol=1e-12, atol=1e-14)
    # the 3D face couplings come only from the mass term
    if dim == 3:
        Ad = A.toarray()
        h = 1.0 / n
        # unknowns 0 and 1 are the nodes (1,1,1) and (2,1,1): x-face neighbours
        assert Ad[0, 1] == pytest.approx(sigma * 2.0 * h ** 3 / 27.0, rel=1e-14)
        assert O.assemble(dim, n).toarray()[0, 1] == 0.0


@pytest.mark.parametrize("dim,n,kap", [(3, 8, None), (2, 16, "lognormal")])
def test_shifted_matfree_and_rows_match_assembly(dim, n, kap):
    sigma = 37.5
    kappa = W.kappa_lognormal(dim, n, 1) if kap else None
    A = O.assemble(dim, n, kappa, sigma=sigma)
    x = np.random.default_rng(4).uniform(-1, 1, (n + 1) ** dim)
    y = O.apply_matfree(dim, n, kappa, x.reshape((n + 1,) * dim), sigma=sigma)
    xi = O.to_interior(dim, n, x.reshape((n + 1,) * dim))
    np.testing.assert_allclose(O.to_interior(dim, n, y), A @ xi, rtol=1e-13, atol=1e-14)
    nodes = np.stack(O.interior_coords(dim, n), axis=1)[::5]
    np.testing.assert_allclose(O.apply_rows(dim, n, kappa, x, nodes, sigma=sigma),
                               (A @ xi)[::5], rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- warm start

def test_warm_start_from_solution_takes_zero_cycles():
    H = O.build_hierarchy(3, 8, 3, sigma=50.0)
    b = np.random.default_rng(5).uniform(-1, 1, 7 ** 3)
    u_star = O.sparse_solve(H.A[0], b)
    u, it, hist, st = O.solve(H, b, 1e-8, u0=u_star)
    assert st == "ok" and it == 0 and len(hist) == 1 and hist[0] < 1e-12
    np.testing.assert_array_equal(u, u_star)


def test_warm_start_from_zero_matches_cold_start():
    H = O.build_hierarchy(2, 16, 3, sigma=10.0)
    b = np.random.default_rng(6).uniform(-1, 1, 15 ** 2)
    cold = O.solve(H, b, 1e-9)
    warm = O.solve(H, b, 1e-9, u0=np.zeros_like(b))
    assert cold[1] == warm[1] and warm[2][0] == 1.0
    np.testing.assert_array_equal(cold[0], warm[0])
    np.testing.assert_array_equal(cold[2], warm[2])


def test_warm_start_reduces_cycles_and_reaches_same_limit():
    H = O.build_hierarchy(3, 16, 4, sigma=200.0, nu_pre=3, nu_post=3)
    b = np.random.default_rng(7).uniform(-1, 1, 15 ** 3)
    u_star = O.dst_solve(3, 16, b, 200.0)
    u0 = u_star + 1e-4 * np.random.default_rng(8).uniform(-1, 1, u_star.size)
    for solver in (O.solve, O.solve_pcg):
        cold = solver(H, b, 1e-10)
        warm = solver(H, b, 1e-10, u0=u0)
        assert warm[3] == "ok" and warm[1] < cold[1]
        assert warm[2][0] == pytest.approx(
            np.linalg.norm(b - H.A[0] @ u0) / np.linalg.norm(b), rel=1e-12)
        np.testing.assert_allclose(warm[0], u_star, rtol=0, atol=1e-9 * np.abs(u_star).max())


# ---------------------------------------------------------------- time loop

def test_cn_reproduces_linear_in_time_solution_exactly():
    # u = t * l(x) with l linear: the source is f = l (Laplace(l) = 0), the
    # Q1 space holds l exactly and Crank-Nicolson is exact for solutions
    # linear in t, so every step reproduces t_n l at the nodes -- any sign
    # or time-level mistake in the right-hand side or the lifting breaks it
    dim, n, dt, steps = 3, 8, 0.05, 4
    ell = _nodal(3, n, lambda x, y, z: x + 2.0 * y - z + 0.5)
    H = O.build_hierarchy(dim, n, 3, sigma=2.0 / dt)
    u, its, _ = OH.run(H, dt, steps, np.zeros((n - 1) ** 3), ell, lambda t: t, ell,
                       lambda t: 1.0, 1e-13)
    np.testing.assert_allclose(u, steps * dt * O.to_interior(dim, n, ell.reshape((n + 1,) * 3)),
                               rtol=0, atol=1e-11)


def test_cn_amplifies_a_sine_mode_by_the_closed_form_factor():
    # no source, zero Dirichlet data, u0 = the lowest sine mode: the mode is
    # a generalised eigenvector (K v = lam M v, lam = d k1 / m1), so each
    # step multiplies it by (sigma - lam) / (sigma + lam)
    dim, n, dt, steps = 2, 16, 0.01, 5
    h = 1.0 / n
    v = _nodal(2, n, lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))
    k1 = (2.0 / h) * (1.0 - np.cos(np.pi * h))
    m1 = (h / 3.0) * (2.0 + np.cos(np.pi * h))
    lam = dim * k1 / m1
    sigma = 2.0 / dt
    H = O.build_hierarchy(dim, n, 4, sigma=sigma)
    u0 = O.to_interior(dim, n, v.reshape((n + 1,) * 2))
    u, _, _ = OH.run(H, dt, steps, u0, None, lambda t: 0.0, None, lambda t: 0.0, 1e-13)
    np.testing.assert_allclose(u, ((sigma - lam) / (sigma + lam)) ** steps * u0,
                               rtol=0, atol=1e-11)


def test_cn_converges_to_the_papers_solution_at_second_order():
    # the model problem of Sec. 6.2 (solution exp(-0.1 t) sin(pi x)
    # cos(pi y) cos(pi z)), started from its nodal values: the nodal error
    # after a few steps falls by about 4 per halving of h
    dt, steps = 0.01, 3
    errs = []
    for n in (8, 16):
        w = W.HeatWorkload("t", 3, n, 3, dt, steps, 1e-12)
        s, u0 = W.heat_inputs(w)
        H = O.build_hierarchy(3, n, w.levels, sigma=w.sigma, nu_pre=3, nu_post=3)
        u, its, _ = OH.run(H, dt, steps, u0, s, W.heat_gamma, s,
                           lambda t: W.heat_lambda(3, t), w.tol)
        exact = W.heat_gamma(steps * dt) * u0
        errs.append(np.abs(u - exact).max())
    assert errs[1] < 5e-3
    assert 3.0 < errs[0] / errs[1] < 5.5


def test_heat_profile_is_the_stated_solution():
    # independent evaluation of sin(pi x) cos(pi y) cos(pi z) at one node
    n = 8
    s = W.heat_profile(3, n).reshape((n + 1,) * 3)
    i, j, k = 3, 5, 2
    assert s[k, j, i] == pytest.approx(
        np.sin(np.pi * i / n) * np.cos(np.pi * j / n) * np.cos(np.pi * k / n), rel=1e-15)
    assert W.heat_lambda(3, 0.0) == pytest.approx(3 * np.pi ** 2 - 0.1, rel=1e-15)


def test_load_vector_is_the_galerkin_integral_of_the_interpolated_source():
    # F = int f_h phi_i with f_h the Q1 (multilinear) interpolant of the
    # nodal source values: Gauss quadrature of f_h phi_i is exact, and a
    # lumped (diagonal) load would differ for rough nodal data
    from scipy.interpolate import RegularGridInterpolator
    dim, n = 3, 6
    f = np.random.default_rng(9).uniform(-1, 1, (n + 1) ** 3)
    c = np.arange(n + 1) / n
    interp = RegularGridInterpolator((c, c, c), f.reshape((n + 1,) * 3), method="linear")

    def fh(x, y, z):
        pts = np.stack([z.ravel(), y.ravel(), x.ravel()], axis=1)
        return interp(pts).reshape(x.shape)

    F = OH.load_vector(dim, n, f)
    np.testing.assert_allclose(F, O.assemble_load_quadrature(dim, n, fh, q=3),
                               rtol=1e-12, atol=1e-15)
    assert np.abs(F - O.to_interior(dim, n, f.reshape((n + 1,) * 3)) / n ** 3).max() > 1e-4
    # the right-hand side adds cf F to the operator terms
    b0 = OH.cn_rhs(dim, n, 40.0, np.zeros((n - 1) ** 3), None, 0.0, None, 0.0, None, 0.0)
    b1 = OH.cn_rhs(dim, n, 40.0, np.zeros((n - 1) ** 3), None, 0.0, None, 0.0, F, 2.5)
    assert not np.any(b0)
    np.testing.assert_array_equal(b1, 2.5 * F)


def test_extrapolated_start_takes_fewer_cycles_to_the_same_solution():
    # starting each solve from 2 u^n - u^{n-1} instead of u^n changes the
    # iteration, not its limit: both loops agree to the solve tolerance,
    # and the extrapolated start needs no more cycles
    dt, steps, n = 0.01, 4, 16
    w = W.HeatWorkload("t", 3, n, 3, dt, steps, 1e-10)
    s, u0 = W.heat_inputs(w)
    H = O.build_hierarchy(3, n, w.levels, sigma=w.sigma, nu_pre=3, nu_post=3)
    lam = lambda t: W.heat_lambda(3, t)
    ua, its_a, _ = OH.run(H, dt, steps, u0, s, W.heat_gamma, s, lam, w.tol)
    ub, its_b, hb = OH.run(H, dt, steps, u0, s, W.heat_gamma, s, lam, w.tol, extrapolate=True)
    assert sum(its_b) < sum(its_a) and its_b[0] == its_a[0]
    np.testing.assert_allclose(ub, ua, rtol=0, atol=1e-9 * np.abs(ua).max())
