"""Crank-Nicolson time loop of the heat-equation model problem on the GPU.

The model problem of Sec. 6.2 (u_t - Laplace(u) = f on the unit cube with
Dirichlet data, solution exp(-0.1 t) sin(pi x) cos(pi y) cos(pi z)), Q1 in
space and Crank-Nicolson in time: each step forms its right-hand side with
mg_cn_rhs and solves (K + (2/dt) M) u' = b with mg_solve warm-started from
the previous step (or from the linear extrapolation of the last two).  Both calls run on the library's kernels; this class only
holds the device arrays and passes the time factors of the data.
"""

import torch

from . import workloads as W
from .mg import FLAG_WARM, MgError, Solver


class HeatRun:
    """Device state of one time loop: u (the solution at the current step,
    unknowns only), b (the last right-hand side), the nodal profile s of the
    Dirichlet data and the load F = M s of the source profile (formed
    once).  With `extrapolate`, each solve starts from 2 u^n - u^{n-1}
    (formed by mg_cn_rhs in the buffer of u^{n-1}, which then receives
    u^{n+1}) instead of u^n."""

    def __init__(self, w, tol=None, precision=None, flags=0, max_iter=100, cycle="V",
                 extrapolate=False):
        self.w = w
        self.tol = w.tol if tol is None else tol
        self.extrapolate = extrapolate
        s, u0 = W.heat_inputs(w)
        self.s = torch.from_numpy(s).to("cuda")
        self.u0 = torch.from_numpy(W.interior_to_full(w.dim, w.n, u0)).to("cuda")
        self.u = torch.empty_like(self.u0)
        self.u_prev = torch.empty_like(self.u0) if extrapolate else None
        self.b = torch.empty_like(self.u0)
        self.S = Solver(w.dim, w.n, w.levels, op=w.op, smoother=w.smoother, nu_pre=w.nu_pre,
                        nu_post=w.nu_post, precision=precision or w.precision, sigma=w.sigma,
                        flags=flags | FLAG_WARM, max_iter=max_iter, cycle=cycle)
        self.F = self.S.mass(self.s)
        self.k = 0
        self.last_hist = None

    def reset(self):
        """Back to t = 0 (the solution's nodal values)."""
        self.u.copy_(self.u0)
        if self.extrapolate:
            self.u_prev.copy_(self.u0)     # the first step starts from u^0
        self.k = 0

    def step(self):
        """One Crank-Nicolson step; returns the cycles of its solve."""
        w = self.w
        t0, t1 = self.k * w.dt, (self.k + 1) * w.dt
        lam = W.heat_lambda(w.dim, t0) + W.heat_lambda(w.dim, t1)
        self.S.cn_rhs(self.u, self.s, W.heat_gamma(t0), self.s, W.heat_gamma(t1), self.F, lam,
                      b=self.b, guess=self.u_prev)
        target = self.u_prev if self.extrapolate else self.u
        _, it, hist, st = self.S.solve(self.b, self.tol, u=target)
        if st != "ok":
            raise MgError(5 if st == "maxit" else 6, f"step {self.k}: solve ended with {st}")
        if self.extrapolate:
            self.u, self.u_prev = self.u_prev, self.u
        self.last_hist = hist
        self.k += 1
        return it

    def run(self, steps):
        return [self.step() for _ in range(steps)]

    @property
    def t(self):
        return self.k * self.w.dt

    def close(self):
        self.S.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
