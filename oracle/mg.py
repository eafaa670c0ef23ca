"""Geometric multigrid V-cycle on the Q1 hierarchy (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):

* Gauss-Seidel, Eq. (1), is read with the division by the diagonal entry
  that the printed formula omits.
* "Red-black" Gauss-Seidel on Q1 couples nodes of the same colour (through
  the diagonal neighbours in 2D and the edge neighbours in 3D), so a
  parallel in-place half-sweep would be order dependent.  A half-sweep on
  colour c therefore updates every node of colour c simultaneously from the
  values at the start of the half-sweep.  Colour c = (sum of node
  coordinates) mod 2.  Pre-smoothing runs colour 0 then 1; post-smoothing
  runs 1 then 0, so that the cycle is symmetric.
* Multicolour Gauss-Seidel ("gs"): with the 2^d colours c = sum_d
  (x_d mod 2) 2^d no two nodes of one colour are coupled, so updating a
  colour's nodes one after the other or all at once gives the same values:
  a sweep over the colours in order is an exact Gauss-Seidel sweep in the
  colour-sorted ordering (Eq. (1) with the colour-wise numbering of
  Sec. 4.2.6).  Pre-smoothing runs colours 0..2^d-1, post-smoothing the
  reverse order (symmetric cycle).
* Damped Jacobi uses omega = 2/3 unless told otherwise.
* The coarsest level is solved exactly by a dense Cholesky factorisation
  (Algorithm 1 allows a direct solver there, Sec. 5.3).
* Coarse operators are rediscretised on every level (not Galerkin
  products); for variable kappa the coarse cell value is the geometric mean
  of its children.
* The outer iteration (Sec. 5.5.1) starts from u = 0 and stops after the
  first cycle whose relative residual ||b - A u||_2 / ||b||_2 over the
  unknowns is <= tol.  Started from a given u0 (a warm start, as in the
  time loop of Sec. 6.2), it first tests u0 itself and stops after zero
  cycles if u0 already meets the tolerance.
* With a mass shift sigma > 0 every level has the matrix K_l + sigma M_l
  (rediscretised, like K_l).
"""

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .q1 import assemble, interior_coords, kappa_hierarchy
from .transfer import prolongation


@dataclass
class Hierarchy:
    dim: int
    n: int
    levels: int
    smoother: str = "rbgs"          # "jacobi", "rbgs" or "gs" (2^d colours)
    cycle: str = "V"                # "V", "W" or "F"
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 2.0 / 3.0
    sigma: float = 0.0              # mass shift: A_l = K_l + sigma M_l
    A: list = field(default_factory=list)       # A[l], l = 0 finest
    diag: list = field(default_factory=list)
    P: list = field(default_factory=list)       # P[l]: level l+1 -> level l
    mask: list = field(default_factory=list)    # colour-0 boolean mask
    colours: list = field(default_factory=list) # 2^d-colour number per unknown
    coarse_factor: object = None
    nl: list = field(default_factory=list)
    # float32 copies for the iterative-refinement inner cycle
    A32: list = field(default_factory=list)
    diag32: list = field(default_factory=list)
    P32: list = field(default_factory=list)


def colour_mask(dim, n, colour):
    """Boolean mask over the unknowns: (sum of coordinates) mod 2 == colour."""
    s = sum(interior_coords(dim, n))
    return (s % 2) == colour


def colours(dim, n):
    """2^d-colour number of every unknown: sum_d (x_d mod 2) 2^d."""
    c = interior_coords(dim, n)
    out = np.zeros(c[0].size, dtype=np.int64)
    for d in range(dim):
        out += (c[d] % 2) << d
    return out


def build_hierarchy(dim, n, levels, kappa=None, smoother="rbgs", nu_pre=2,
                    nu_post=2, omega=2.0 / 3.0, fp32=False, cycle="V", sigma=0.0):
    """Assemble every level's operator and the transfers (Sec. 5.1)."""
    if levels < 1 or n % (1 << (levels - 1)) != 0 or (n >> (levels - 1)) < 2:
        raise ValueError("need n divisible by 2^(levels-1) and n_c >= 2")
    if cycle not in CYCLE_SCHEDULE:
        raise ValueError("cycle must be V, W or F")
    if not (np.isfinite(sigma) and sigma >= 0.0):
        raise ValueError("sigma must be finite and >= 0")
    H = Hierarchy(dim=dim, n=n, levels=levels, smoother=smoother, cycle=cycle,
                  nu_pre=nu_pre, nu_post=nu_post, omega=omega, sigma=sigma)
    kaps = kappa_hierarchy(dim, n, levels, kappa)
    for l in range(levels):
        nl = n >> l
        A = assemble(dim, nl, kaps[l], sigma)
        H.nl.append(nl)
        H.A.append(A)
        H.diag.append(A.diagonal().copy())
        H.mask.append(colour_mask(dim, nl, 0))
        H.colours.append(colours(dim, nl))
        if l < levels - 1:
            H.P.append(prolongation(dim, nl))
    Ac = H.A[-1].toarray()
    H.coarse_factor = sla.cho_factor(Ac, lower=True)
    if fp32:
        H.A32 = [A.astype(np.float32) for A in H.A]
        H.diag32 = [d.astype(np.float32) for d in H.diag]
        H.P32 = [P.astype(np.float32) for P in H.P]
    return H


# --------------------------------------------------------------------------
# smoothers (Eq. (1); Algorithm 1 steps "pre-smoothing" / "post-smoothing")
# --------------------------------------------------------------------------

def jacobi_sweep(A, diag, x, b, omega):
    """x + omega D^-1 (b - A x)."""
    r = b - A @ x
    return x + omega * (r / diag)


def rb_half_sweep(A, diag, x, b, mask):
    """Update the nodes selected by ``mask`` simultaneously from x."""
    r = b - A @ x
    return np.where(mask, x + r / diag, x)


def gs_colour_step(A, diag, x, b, sel):
    """Gauss-Seidel update of the unknowns selected by ``sel`` (one colour:
    no two of them coupled) from the current x."""
    r = b - A @ x
    return np.where(sel, x + r / diag, x)


def smooth(H, l, x, b, pre, fp32=False):
    A = H.A32[l] if fp32 else H.A[l]
    diag = H.diag32[l] if fp32 else H.diag[l]
    nu = H.nu_pre if pre else H.nu_post
    if H.smoother == "jacobi":
        om = np.float32(H.omega) if fp32 else H.omega
        for _ in range(nu):
            x = jacobi_sweep(A, diag, x, b, om)
        return x
    if H.smoother == "gs":
        nc = 2 ** H.dim
        order = range(nc) if pre else range(nc - 1, -1, -1)
        for _ in range(nu):
            for c in order:
                x = gs_colour_step(A, diag, x, b, H.colours[l] == c)
        return x
    red = H.mask[l]
    order = (red, ~red) if pre else (~red, red)
    for _ in range(nu):
        for m in order:
            x = rb_half_sweep(A, diag, x, b, m)
    return x


def coarse_solve(H, b, fp32=False):
    """Exact solve on the coarsest level with the FP64 Cholesky factor."""
    if fp32:
        return sla.cho_solve(H.coarse_factor, b.astype(np.float64)).astype(np.float32)
    return sla.cho_solve(H.coarse_factor, b)


# --------------------------------------------------------------------------
# V-cycle (Algorithm 1) and the outer iteration
# --------------------------------------------------------------------------

# Coarse-level cycles run from a level by each cycle kind, in order: the
# V-cycle solves the residual equation once, the W-cycle twice, the F-cycle
# by an F-cycle followed by a V-cycle.
CYCLE_SCHEDULE = {"V": ("V",), "W": ("W", "W"), "F": ("F", "V")}


def cycle(H, l, x, b, kind="V", fp32=False):
    """One multigrid cycle of the given kind on level l for A_l x = b,
    starting from x.

    Steps in the order of Algorithm 1: pre-smoothing, restriction of the
    residual, approximate solve of the coarse residual equation from a zero
    guess, prolongation of the correction added to x, post-smoothing.  The
    coarse equation is solved by the cycles of CYCLE_SCHEDULE[kind], each
    starting from the previous one's result (Algorithm 1 is the V-cycle; the
    paper mentions other cycle shapes, Sec. 5.3); directly above the
    coarsest level it is solved exactly, once, for every kind.
    """
    if l == H.levels - 1:
        return coarse_solve(H, b, fp32)
    A = H.A32[l] if fp32 else H.A[l]
    P = H.P32[l] if fp32 else H.P[l]
    x = smooth(H, l, x, b, pre=True, fp32=fp32)
    r = b - A @ x
    bc = P.T @ r
    e = np.zeros(bc.shape[0], dtype=bc.dtype)
    if l + 1 == H.levels - 1:
        e = coarse_solve(H, bc, fp32)
    else:
        for sub in CYCLE_SCHEDULE[kind]:
            e = cycle(H, l + 1, e, bc, sub, fp32)
    x = x + P @ e
    x = smooth(H, l, x, b, pre=False, fp32=fp32)
    return x


def vcycle(H, l, x, b, fp32=False):
    """One V-cycle (Algorithm 1) on level l for A_l x = b, starting from x."""
    return cycle(H, l, x, b, "V", fp32)


def _start(A, b, u0):
    """(u, r, nb, hist) at the start of a solve: u = 0 (hist[0] = 1) or the
    warm start u0 (hist[0] = ||b - A u0|| / ||b||)."""
    nb = np.linalg.norm(b)
    if u0 is None:
        return np.zeros_like(b), b.copy(), nb, [1.0]
    u = np.array(u0, dtype=np.float64)
    r = b - A @ u
    return u, r, nb, [np.linalg.norm(r) / nb if nb > 0.0 else 0.0]


def solve(H, b, tol, max_iter=100, u0=None, diverge=1e3):
    """Outer fixed-point iteration of V-cycles (Sec. 5.5.1) in FP64.

    Returns (u, iters, hist, status) with hist[0] the relative residual of
    the start (1 from u = 0) and hist[k] the relative residual after cycle
    k; status is "ok", "maxit" or "diverged".
    """
    b = np.asarray(b, dtype=np.float64)
    A = H.A[0]
    u, _, nb, hist = _start(A, b, u0)
    if nb == 0.0:
        return np.zeros_like(b), 0, [1.0], "ok"
    if u0 is not None and hist[0] <= tol:
        return u, 0, hist, "ok"
    for k in range(1, max_iter + 1):
        u = cycle(H, 0, u, b, H.cycle)
        rho = np.linalg.norm(b - A @ u) / nb
        hist.append(rho)
        if not np.isfinite(rho) or rho > diverge:
            return u, k, hist, "diverged"
        if rho <= tol:
            return u, k, hist, "ok"
    return u, max_iter, hist, "maxit"


def ir_scale(nb):
    """Scale of the float32 correction equations of iterative refinement:
    the power of two 2^e with ||b|| = m 2^e, 1/2 <= m < 1.  Dividing by a
    power of two is exact, so float32(r / s) = float32(r) / s and the float32
    cycle, homogeneous under such scalings, computes the correction of r as
    it would of float32(r) itself; s only keeps the float32 values near
    unit size whatever the scale of b."""
    return math.ldexp(1.0, math.frexp(float(nb))[1])


def solve_ir(H, b, tol, max_iter=100, diverge=1e3, u0=None):
    """FP32-inner / FP64-outer iterative refinement.

    FP64: r = b - A u; the correction equation is solved approximately by
    one float32 V-cycle (operators rounded from the FP64 assembly, coarse
    solve in FP64) applied to float32(r / s) from a zero guess, s =
    :func:`ir_scale` of ||b|| (fixed for the solve); then u += s *
    float64(c).  Starts and stops like :func:`solve`.
    """
    if not H.A32:
        raise ValueError("hierarchy built without fp32=True")
    b = np.asarray(b, dtype=np.float64)
    A = H.A[0]
    u, r, nb, hist = _start(A, b, u0)
    if nb == 0.0:
        return np.zeros_like(b), 0, [1.0], "ok"
    if u0 is not None and hist[0] <= tol:
        return u, 0, hist, "ok"
    s = ir_scale(nb)
    for k in range(1, max_iter + 1):
        r32 = (r / s).astype(np.float32)
        c32 = cycle(H, 0, np.zeros_like(r32), r32, H.cycle, fp32=True)
        u = u + s * c32.astype(np.float64)
        r = b - A @ u
        rho = np.linalg.norm(r) / nb
        hist.append(rho)
        if not np.isfinite(rho) or rho > diverge:
            return u, k, hist, "diverged"
        if rho <= tol:
            return u, k, hist, "ok"
    return u, max_iter, hist, "maxit"


def precondition(H, r, fp32=False):
    """The multigrid preconditioner: z = one cycle (H.cycle, V or W) from a
    zero guess on A z = r.  With fp32, the cycle runs in float32 on r / s
    and is scaled back: z = s * float64(cycle32(float32(r / s))), s =
    :func:`ir_scale` of ||r||.  The V- and W-cycles are symmetric (post-smoothing reverses
    the colour order of the pre-smoothing, nu_pre = nu_post), so in exact
    arithmetic z = B r with B symmetric positive definite; the F-cycle is
    not and is refused."""
    if H.cycle == "F":
        raise ValueError("CG needs a symmetric cycle (V or W)")
    if not fp32:
        return cycle(H, 0, np.zeros_like(r), r, H.cycle)
    nr = np.linalg.norm(r)
    if nr == 0.0:
        return np.zeros_like(r)
    s = ir_scale(nr)
    r32 = (r / s).astype(np.float32)
    return s * cycle(H, 0, np.zeros_like(r32), r32, H.cycle, fp32=True).astype(np.float64)


def solve_pcg(H, b, tol, max_iter=100, diverge=1e3, fp32=False, precond=None, u0=None):
    """Conjugate gradients on A u = b preconditioned by one V-cycle per
    iteration.  The paper names multigrid as a preconditioner for Krylov
    solvers (Sec. 1, with GMRES); A is symmetric positive definite and the
    V-cycle symmetric, so CG is the Krylov method used here.

    Steps per iteration k (u_0 = 0 or the warm start, r_0 = b - A u_0,
    z_0 = B r_0, p_0 = z_0):
      q = A p;  alpha = (r, z) / (p, q);  u += alpha p;  r' = r - alpha q;
      stop if ||r'|| / ||b|| <= tol;
      z' = B r';  beta = (z', r' - r) / (r, z);  p = z' + beta p.
    beta is the flexible (Polak-Ribiere) form: for a fixed SPD B it equals
    the classical (z', r') / (z, r) because (z', r) = 0, and it keeps the
    iteration robust when B is applied in float32.  The stopping test uses
    the recursively updated residual r'.

    precond: optional replacement for the V-cycle (a function r -> z), for
    the special cases that pin this routine.  Starts, stops and returns
    (u, iters, hist, status) like :func:`solve`.
    """
    b = np.asarray(b, dtype=np.float64)
    A = H.A[0]
    M = precond if precond is not None else (lambda v: precondition(H, v, fp32))
    u, r, nb, hist = _start(A, b, u0)
    if nb == 0.0:
        return np.zeros_like(b), 0, [1.0], "ok"
    if u0 is not None and hist[0] <= tol:
        return u, 0, hist, "ok"
    z = M(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, max_iter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        u = u + alpha * p
        r_new = r - alpha * q
        rho = np.linalg.norm(r_new) / nb
        hist.append(rho)
        if not np.isfinite(rho) or rho > diverge:
            return u, k, hist, "diverged"
        if rho <= tol:
            return u, k, hist, "ok"
        z = M(r_new)
        beta = (z @ r_new - z @ r) / rz
        rz = z @ r_new
        p = z + beta * p
        r = r_new
    return u, max_iter, hist, "maxit"
