"""Seeded synthetic inputs for the Q1 multigrid workloads.

This module holds the input recipes only (random right-hand sides,
coefficients, request traces, the manufactured load of the 2D model
problem and the data of the heat-equation model problem); it contains none
of the solver's arithmetic.  Both the GPU path and
the CPU oracle are fed from here, so every comparison sees bit-identical
inputs.  All randomness is NumPy PCG64 ``default_rng(seed)`` on the host.

Layouts:
* "interior" vectors hold the (n-1)^d unknowns, x fastest;
* "full" arrays hold all (n+1)^d nodes, x fastest, boundary entries 0 --
  the layout the C library takes;
* cell arrays hold n^d values, x fastest.
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int
    levels: int
    smoother: str          # "jacobi" | "rbgs"
    op: str                # "stencil" | "csr"
    precision: str         # "fp64" | "fp32_ir"
    tol: float
    rhs: str               # "manufactured" | "uniform" | "ones"
    kappa: str             # "none" | "lognormal"
    omega: float = 2.0 / 3.0
    nu_pre: int = 2
    nu_post: int = 2
    seed: int = 0

    @property
    def dofs(self):
        """All nodes, boundary included: (n+1)^d."""
        return (self.n + 1) ** self.dim

    @property
    def unknowns(self):
        return (self.n - 1) ** self.dim


# The workloads of the benchmark.  Coarsest levels: 2D n_c = 4, 3D n_c = 2
# (or 3 for n = 192).  The variable-coefficient system is also solved in
# FP64 for comparison with its FP32-inner form.
WORKLOADS = {
    "poisson2d_64_jacobi": Workload(
        "poisson2d_64_jacobi", 2, 64, 5, "jacobi", "stencil", "fp64", 1e-10,
        "manufactured", "none"),
    "poisson3d_128_csr_rbgs": Workload(
        "poisson3d_128_csr_rbgs", 3, 128, 7, "rbgs", "csr", "fp64", 1e-8,
        "uniform", "none"),
    "poisson3d_256_rbgs_fp64": Workload(
        "poisson3d_256_rbgs_fp64", 3, 256, 8, "rbgs", "stencil", "fp64", 1e-8,
        "uniform", "none"),
    "poisson3d_256_rbgs_ir": Workload(
        "poisson3d_256_rbgs_ir", 3, 256, 8, "rbgs", "stencil", "fp32_ir", 1e-8,
        "uniform", "none"),
    "kappa3d_192_rbgs_ir": Workload(
        "kappa3d_192_rbgs_ir", 3, 192, 7, "rbgs", "stencil", "fp32_ir", 1e-8,
        "ones", "lognormal"),
    "kappa3d_192_rbgs_fp64": Workload(
        "kappa3d_192_rbgs_fp64", 3, 192, 7, "rbgs", "stencil", "fp64", 1e-8,
        "ones", "lognormal"),
}


def rhs_uniform(dim, n, seed):
    """Algebraic right-hand side b ~ U[-1, 1] at the interior nodes."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n - 1) ** dim)


def rhs_ones_load(dim, n):
    """Load vector of f = 1: b_i = int phi_i = h^d at every interior node."""
    return np.full((n - 1) ** dim, (1.0 / n) ** dim)


def rhs_manufactured(dim, n):
    """Exactly integrated load of f = d pi^2 prod_d sin(pi x_d).

    This is the right-hand side of the model problem whose solution is
    u = prod_d sin(pi x_d) with zero Dirichlet data.  The integral of
    sin(pi x) against the 1D hat function at x_i is
    h * 2 (1 - cos(pi h)) / (pi h)^2 * sin(pi x_i), and the d-dimensional
    integral is the product of the 1D ones.
    """
    h = 1.0 / n
    i = np.arange(1, n)
    one = h * 2.0 * (1.0 - np.cos(np.pi * h)) / (np.pi * h) ** 2 * np.sin(np.pi * i * h)
    out = np.ones(1)
    for _ in range(dim):
        out = np.multiply.outer(out, one)          # last axis = x (fastest)
    return dim * np.pi ** 2 * out.ravel()


def kappa_lognormal(dim, n, seed):
    """Cell coefficient kappa = exp(g), g ~ N(0, 1) i.i.d., n^d cells."""
    return np.exp(np.random.default_rng(seed).standard_normal(n ** dim))


def interior_to_full(dim, n, x_int, dtype=np.float64):
    """Embed an interior vector into the (n+1)^d layout (boundary 0)."""
    full = np.zeros((n + 1,) * dim, dtype=dtype)
    full[(slice(1, n),) * dim] = np.asarray(x_int).reshape((n - 1,) * dim)
    return full.ravel()


def full_to_interior(dim, n, x_full):
    """Inverse of :func:`interior_to_full`."""
    x = np.asarray(x_full).reshape((n + 1,) * dim)
    return x[(slice(1, n),) * dim].ravel().copy()


def workload_inputs(w):
    """(b_interior, kappa_cells_or_None) for a :class:`Workload`."""
    if w.rhs == "manufactured":
        b = rhs_manufactured(w.dim, w.n)
    elif w.rhs == "uniform":
        b = rhs_uniform(w.dim, w.n, w.seed)
    elif w.rhs == "ones":
        b = rhs_ones_load(w.dim, w.n)
    else:
        raise ValueError(w.rhs)
    kappa = kappa_lognormal(w.dim, w.n, w.seed) if w.kappa == "lognormal" else None
    return b, kappa


# --------------------------------------------------------------------------
# heat-equation model problem (Crank-Nicolson time loop)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class HeatWorkload:
    """u_t - Laplace(u) = f on (0,1)^dim with Dirichlet data, solution
    u = exp(-0.1 t) sin(pi x) cos(pi y) [cos(pi z)]; Crank-Nicolson steps
    of length dt, each a solve with K + (2/dt) M warm-started from the
    previous step."""
    name: str
    dim: int
    n: int
    levels: int
    dt: float
    steps: int
    tol: float
    smoother: str = "rbgs"
    nu_pre: int = 3
    nu_post: int = 3
    op: str = "stencil"
    precision: str = "fp64"

    @property
    def dofs(self):
        return (self.n + 1) ** self.dim

    @property
    def unknowns(self):
        return (self.n - 1) ** self.dim

    @property
    def sigma(self):
        return 2.0 / self.dt


# 512^3 cells: 135,005,697 nodes, the size of the paper's scaling run;
# T = 5 in 500 steps of 0.01; V(3,3) Gauss-Seidel.
HEAT_WORKLOADS = {
    "heat3d_512_cn": HeatWorkload("heat3d_512_cn", 3, 512, 9, 0.01, 500, 1e-8),
    "heat3d_64_cn": HeatWorkload("heat3d_64_cn", 3, 64, 6, 0.01, 10, 1e-8),
}


def heat_profile(dim, n):
    """s(x) = sin(pi x) cos(pi y) [cos(pi z)] at every node, full layout."""
    c = np.arange(n + 1) / n
    out = np.sin(np.pi * c)                           # x (fastest)
    for _ in range(dim - 1):
        out = np.multiply.outer(np.cos(np.pi * c), out)
    return out.ravel()


def heat_gamma(t):
    """Time factor of the solution and of the Dirichlet data."""
    return float(np.exp(-0.1 * t))


def heat_lambda(dim, t):
    """Time factor of the source: f = u_t - Laplace(u) = (dim pi^2 - 0.1)
    exp(-0.1 t) s(x)."""
    return float((dim * np.pi ** 2 - 0.1) * np.exp(-0.1 * t))


def heat_inputs(w):
    """(profile_full, u0_interior): the nodal profile s (Dirichlet data
    gamma(t) s on the boundary, source lambda(t) s) and the solution at
    t = 0 on the unknowns."""
    s = heat_profile(w.dim, w.n)
    return s, full_to_interior(w.dim, w.n, s)


# --------------------------------------------------------------------------
# serving trace
# --------------------------------------------------------------------------

SERVE_SIZES_2D = (64, 128, 256, 512, 1024)
SERVE_SIZES_3D = (32, 64, 128)


def serve_levels(dim, n):
    """Levels for a serving request: coarsest 4 cells in 2D, 2 in 3D."""
    coarsest = 4 if dim == 2 else 2
    lv = 1
    while (n >> (lv - 1)) > coarsest:
        lv += 1
    return lv


def serving_trace(num=2000, rate=200.0, seed=0, burst=False, kappa_frac=0.0):
    """Request trace: Poisson arrivals at ``rate`` per second.

    Each request is 2D or 3D with probability 1/2, with a mesh size drawn
    uniformly from the sizes of its dimension, and a seed for its
    U[-1, 1] right-hand side.  ``burst`` puts every arrival at t = 0.
    With ``kappa_frac`` > 0, that fraction of the 3D requests (drawn from
    a generator of their own, so the rest of the trace is unchanged) solve
    the variable-coefficient problem of the 192^3 workload, kappa = exp(g),
    g ~ N(0, 1) per cell from the request's seed.  (In 2D the rediscretised
    coarse operators of such coefficient fields make the cycle iteration
    diverge for some fields at n >= 512, in the CPU oracle as on the GPU.)
    Returns a list of dicts (t_arrival, dim, n, levels, seed, kappa).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, num)
    t = np.cumsum(gaps) - gaps[0]
    kap = np.random.default_rng(seed + 7919).random(num) < kappa_frac
    out = []
    for i in range(num):
        dim = 2 if rng.random() < 0.5 else 3
        sizes = SERVE_SIZES_2D if dim == 2 else SERVE_SIZES_3D
        n = int(sizes[rng.integers(len(sizes))])
        out.append(dict(id=i, t_arrival=0.0 if burst else float(t[i]),
                        dim=dim, n=n, levels=serve_levels(dim, n),
                        seed=int(1000 + i), kappa=bool(kap[i]) and dim == 3))
    return out
