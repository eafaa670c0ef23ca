"""Crank-Nicolson time stepping of the heat equation with Q1 elements (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The model problem of Sec. 6.2: u_t - Laplace(u) = f in (0, T] x (0,1)^3
with Dirichlet data, discretised by the standard Galerkin method in space
and the Crank-Nicolson scheme in time.  With the full-grid stiffness K and
mass M (boundary nodes included) and sigma = 2/dt, one step reads, on the
interior rows,

    (sigma M + K) u^{n+1} = (sigma M - K) u^n + M (f^n + f^{n+1}),

the Crank-Nicolson equation M (u^{n+1} - u^n)/dt + K (u^{n+1} + u^n)/2 =
(F^n + F^{n+1})/2 multiplied by 2/dt.  The load vectors are F = M f with f
the nodal values of the source (its Q1 interpolant); for a source
lambda(t) f(x) the load vector of f is formed once and scaled.  The
boundary values of u^n and u^{n+1} are the Dirichlet data at t_n and
t_{n+1}.  Moving the known boundary values of u^{n+1} to the right-hand
side leaves the interior system (K + sigma M)_II w = b of
:func:`oracle.mg.solve`.
"""

import numpy as np

from .q1 import assemble_full, to_full, to_interior
from .mg import solve, solve_ir, solve_pcg


def _boundary_mask(dim, n):
    m = np.ones((n + 1,) * dim, dtype=bool)
    m[tuple(slice(1, n) for _ in range(dim))] = False
    return m


def load_vector(dim, n, f, KM=None):
    """F = (M f)_I: the Galerkin load of the Q1 interpolant of the nodal
    values f (a full-grid array, boundary nodes included)."""
    _, M = KM if KM is not None else assemble_full(dim, n)
    return to_interior(dim, n, (M @ np.asarray(f, dtype=np.float64).ravel()).reshape(
        (n + 1,) * dim))


def cn_rhs(dim, n, sigma, u_int, g0, c0, g1, c1, F, cf, KM=None):
    """Right-hand side of one Crank-Nicolson step on the unknowns:

        b = [(sigma M - K) x0 - (sigma M + K) x1]_I + cf F

    x0: u_int on the interior nodes and c0 * g0 on the boundary nodes (the
    solution at t_n); x1: c1 * g1 on the boundary nodes and 0 inside (the
    Dirichlet data at t_{n+1}, moved to the right-hand side); F: a load
    vector on the unknowns (interior layout), scaled by cf (cf =
    lambda(t_n) + lambda(t_{n+1}) for a source lambda(t) f(x) with F the
    load of f).  g0, g1 are full-grid arrays (None: 0) of which only the
    boundary entries are used; F may be None.
    """
    K, M = KM if KM is not None else assemble_full(dim, n)
    shape = (n + 1,) * dim
    bm = _boundary_mask(dim, n)
    x0 = to_full(dim, n, u_int).astype(np.float64)
    x1 = np.zeros(shape)
    if g0 is not None:
        x0[bm] = c0 * np.asarray(g0, dtype=np.float64).reshape(shape)[bm]
    if g1 is not None:
        x1[bm] = c1 * np.asarray(g1, dtype=np.float64).reshape(shape)[bm]
    x0 = x0.ravel()
    x1 = x1.ravel()
    y = sigma * (M @ x0) - K @ x0 - (sigma * (M @ x1) + K @ x1)
    b = to_interior(dim, n, y.reshape(shape))
    if F is not None:
        b = b + cf * np.asarray(F, dtype=np.float64)
    return b


def run(H, dt, steps, u0_int, g, gamma, f, lam, tol, method="mg", max_iter=100,
        extrapolate=False):
    """Crank-Nicolson time loop with warm-started solves.

    H: hierarchy built with sigma = 2/dt.  Dirichlet data gamma(t) g(x) and
    source lambda(t) f(x) (g, f full-grid nodal arrays or None; gamma, lam
    callables).  u0_int: interior values at t = 0.  Each step forms the
    right-hand side with :func:`cn_rhs` (the load of f formed once) and
    solves from u^n, or with `extrapolate` from the linear extrapolation
    2 u^n - u^{n-1} (u^0 on the first step) -- method "mg": cycles, "ir":
    FP32-inner refinement, "pcg": preconditioned CG.  Returns (u_int at
    t = steps*dt, per-step cycle counts, per-step histories).
    """
    dim, n = H.dim, H.n
    sigma = H.sigma
    if abs(sigma - 2.0 / dt) > 1e-12 * sigma:
        raise ValueError("hierarchy sigma must be 2/dt")
    KM = assemble_full(dim, n)
    F = None if f is None else load_vector(dim, n, f, KM)
    u = np.asarray(u0_int, dtype=np.float64).copy()
    u_prev = None
    its, hists = [], []
    solver = {"mg": solve, "ir": solve_ir, "pcg": solve_pcg}[method]
    for s in range(steps):
        t0, t1 = s * dt, (s + 1) * dt
        b = cn_rhs(dim, n, sigma, u, g, gamma(t0), g, gamma(t1), F, lam(t0) + lam(t1), KM)
        start = 2.0 * u - u_prev if (extrapolate and u_prev is not None) else u
        u_new, it, hist, st = solver(H, b, tol, max_iter=max_iter, u0=start)
        if st != "ok":
            raise RuntimeError(f"step {s}: solve ended with {st}")
        its.append(it)
        hists.append(hist)
        u_prev, u = u, u_new
    return u, its, hists
