"""Matrix-free form of the oracle's multigrid cycle, on full-grid arrays.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method and its readings are those of :mod:`oracle.mg`.  Only the storage
differs: no matrix is assembled, so the 256^3 and 192^3 systems fit (the
FP64 CSR matrix of 256^3 cells alone would take 5.4 GB).  Every vector is a
full-grid array of (n+1)^d nodes, x fastest, whose boundary entries are 0
(the eliminated Dirichlet nodes, Sec. 4.2.6).

* A x is the sum over cells of the element contributions (Sec. 2): for cell
  c with vertex values x_c (2^d of them), the cell adds kappa_c K_e x_c to
  the entries of its vertices.  The element matrix K_e is
  :func:`oracle.q1.element_matrix`; a library matrix product forms K_e x_c
  for all cells at once.
* The diagonal a_ii is the sum of kappa_c (K_e)_aa over the 2^d cells that
  hold node i as local vertex a.
* P (Sec. 5.4, read for nested Q1): a fine node whose coordinates have k odd
  entries takes the average of its 2^k coarse parents, weight 2^-k each;
  R = P^T collects the same weights the other way.
* Smoothers, the V/W/F cycle of Algorithm 1 (Sec. 5.3), the outer iteration
  (Sec. 5.5.1) and the FP32-inner / FP64-outer refinement follow
  :mod:`oracle.mg` step by step.  The coarsest matrix is built by applying
  A to unit vectors and factorised by dense Cholesky.

In FP32 mode the element matrix, the cell coefficients and every vector are
rounded to float32 and the inner cycle computes in float32; the coarsest
solve runs in FP64 on the up-cast right-hand side, as in :mod:`oracle.mg`.
"""

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .mg import CYCLE_SCHEDULE, ir_scale
from .q1 import element_matrix, kappa_hierarchy, local_vertices


def _vslice(v, n):
    """Slices of a full-grid array ([z, y, x] axes) selecting local vertex
    v = (v_x, v_y[, v_z]) of every cell."""
    return tuple(slice(vi, vi + n) for vi in reversed(v))


def _zero_boundary(a):
    for ax in range(a.ndim):
        idx = [slice(None)] * a.ndim
        idx[ax] = 0
        a[tuple(idx)] = 0
        idx[ax] = -1
        a[tuple(idx)] = 0


def colour_full(dim, n):
    """Red-black colour (sum of node coordinates mod 2) of every node."""
    c = np.zeros((n + 1,) * dim, dtype=np.int64)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n + 1
        c = c + np.arange(n + 1).reshape(shape)
    return c % 2


def interior_full(dim, n):
    m = np.zeros((n + 1,) * dim, dtype=bool)
    m[(slice(1, n),) * dim] = True
    return m


# --------------------------------------------------------------------------
# operator (Sec. 2): element by element, never assembled
# --------------------------------------------------------------------------

def apply(dim, n, kappa, x, Ke):
    """y = A x on the full grid.  kappa: n^d cell values (shape (n,)*d) or
    None; Ke: element matrix (its dtype sets the arithmetic).  Boundary
    values of x are taken as 0 and those of y are set to 0."""
    dt = Ke.dtype
    x = np.asarray(x, dtype=dt).reshape((n + 1,) * dim).copy()
    _zero_boundary(x)
    verts = local_vertices(dim)
    # X[b] holds, for every cell, the value of x at its local vertex b
    X = np.empty((len(verts),) + (n,) * dim, dtype=dt)
    for b, w in enumerate(verts):
        X[b] = x[_vslice(w, n)]
    Y = (Ke @ X.reshape(len(verts), -1)).reshape(X.shape)   # K_e x_c, every cell
    del X
    y = np.zeros_like(x)
    for a, v in enumerate(verts):
        if kappa is None:
            y[_vslice(v, n)] += Y[a]
        else:
            y[_vslice(v, n)] += kappa * Y[a]
    _zero_boundary(y)
    return y


def diagonal(dim, n, kappa, Ke):
    """a_ii on the full grid (1 on the boundary, where it is never used)."""
    dt = Ke.dtype
    ones = np.ones((n,) * dim, dtype=dt) if kappa is None else kappa
    d = np.zeros((n + 1,) * dim, dtype=dt)
    for a, v in enumerate(local_vertices(dim)):
        d[_vslice(v, n)] += ones * Ke[a, a]
    inner = interior_full(dim, n)
    d[~inner] = 1
    return d


# --------------------------------------------------------------------------
# transfers (Sec. 5.4)
# --------------------------------------------------------------------------

def _parity_pairs(dim, nc):
    """(weight, fine slices, coarse slices) for every fine parity p in
    {0,1}^d and every coarse parent offset q <= p.  A fine node 2I + p has
    the parents I + q, q_d in {0, p_d}, each with weight 2^-|p|."""
    out = []
    for p in itertools.product((0, 1), repeat=dim):          # p = (p_x, p_y[, p_z])
        w = 0.5 ** sum(p)
        qs = itertools.product(*[(0, 1) if pd else (0,) for pd in p])
        for q in qs:
            fs, cs = [], []
            for d in reversed(range(dim)):                    # array axes z, y, x
                if p[d] == 0:
                    fs.append(slice(0, 2 * nc + 1, 2))        # even fine nodes, I = 0..nc
                    cs.append(slice(0, nc + 1))
                else:
                    fs.append(slice(1, 2 * nc, 2))            # odd fine nodes, I = 0..nc-1
                    cs.append(slice(q[d], q[d] + nc))
            out.append((w, tuple(fs), tuple(cs)))
    return out


def prolong(dim, n_fine, e):
    """P e: coarse full grid ((n_fine/2)+1)^d -> fine full grid."""
    nc = n_fine // 2
    e = np.asarray(e).reshape((nc + 1,) * dim)
    out = np.zeros((n_fine + 1,) * dim, dtype=e.dtype)
    for w, fs, cs in _parity_pairs(dim, nc):
        out[fs] += e.dtype.type(w) * e[cs]
    _zero_boundary(out)
    return out


def restrict(dim, n_fine, r):
    """P^T r: fine full grid -> coarse full grid (no 2^-d scaling)."""
    nc = n_fine // 2
    r = np.asarray(r).reshape((n_fine + 1,) * dim)
    out = np.zeros((nc + 1,) * dim, dtype=r.dtype)
    for w, fs, cs in _parity_pairs(dim, nc):
        out[cs] += r.dtype.type(w) * r[fs]
    _zero_boundary(out)
    return out


# --------------------------------------------------------------------------
# hierarchy, smoothers, cycle
# --------------------------------------------------------------------------

@dataclass
class MFHierarchy:
    dim: int
    n: int
    levels: int
    smoother: str = "rbgs"
    cycle: str = "V"
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 2.0 / 3.0
    nl: list = field(default_factory=list)
    kappa: list = field(default_factory=list)     # per level: (n_l,)*d or None
    Ke: list = field(default_factory=list)        # element matrix per level (h_l)
    diag: list = field(default_factory=list)
    colour: list = field(default_factory=list)    # red-black colour per node
    inner: list = field(default_factory=list)     # interior-node mask
    coarse_factor: object = None
    coarse_n: int = 0
    fp32: bool = False
    kappa32: list = field(default_factory=list)
    Ke32: list = field(default_factory=list)
    diag32: list = field(default_factory=list)


def build(dim, n, levels, kappa=None, smoother="rbgs", nu_pre=2, nu_post=2,
          omega=2.0 / 3.0, fp32=False, cycle="V"):
    """Per-level coefficients (geometric-mean coarsening), element matrices,
    diagonals and colours, and the Cholesky factor of the coarsest matrix."""
    if levels < 1 or n % (1 << (levels - 1)) != 0 or (n >> (levels - 1)) < 2:
        raise ValueError("need n divisible by 2^(levels-1) and n_c >= 2")
    if smoother not in ("jacobi", "rbgs"):
        raise ValueError("smoother must be jacobi or rbgs")
    if cycle not in CYCLE_SCHEDULE:
        raise ValueError("cycle must be V, W or F")
    H = MFHierarchy(dim=dim, n=n, levels=levels, smoother=smoother, cycle=cycle,
                    nu_pre=nu_pre, nu_post=nu_post, omega=omega, fp32=fp32)
    kaps = kappa_hierarchy(dim, n, levels, kappa)
    for l in range(levels):
        nl = n >> l
        k = None if kaps[l] is None else kaps[l].reshape((nl,) * dim)
        Ke = element_matrix(dim, 1.0 / nl)
        H.nl.append(nl)
        H.kappa.append(k)
        H.Ke.append(Ke)
        H.diag.append(diagonal(dim, nl, k, Ke))
        H.colour.append(colour_full(dim, nl))
        H.inner.append(interior_full(dim, nl))
        if fp32:
            k32 = None if k is None else k.astype(np.float32)
            Ke32 = Ke.astype(np.float32)
            H.kappa32.append(k32)
            H.Ke32.append(Ke32)
            H.diag32.append(diagonal(dim, nl, k32, Ke32))
    nc = H.nl[-1]
    H.coarse_n = nc
    Ac = coarse_matrix(H)
    H.coarse_factor = sla.cho_factor(Ac, lower=True)
    return H


def coarse_matrix(H):
    """Dense matrix of the coarsest level on its unknowns, column j = A e_j."""
    dim, nc = H.dim, H.nl[-1]
    inner = H.inner[-1]
    idx = np.flatnonzero(inner.ravel())
    Ac = np.zeros((idx.size, idx.size))
    for j, p in enumerate(idx):
        e = np.zeros((nc + 1) ** dim)
        e[p] = 1.0
        Ac[:, j] = apply(dim, nc, H.kappa[-1], e, H.Ke[-1]).ravel()[idx]
    return Ac


def op(H, l, x, fp32=False):
    if fp32:
        return apply(H.dim, H.nl[l], H.kappa32[l], x, H.Ke32[l])
    return apply(H.dim, H.nl[l], H.kappa[l], x, H.Ke[l])


def smooth(H, l, x, b, pre, fp32=False):
    """nu Jacobi sweeps x + omega D^-1 (b - A x), or nu red-black sweeps, each
    two half-sweeps that update every node of one colour at once from the
    values at the start of the half-sweep (colour 0 first before the coarse
    correction, colour 1 first after it)."""
    diag = H.diag32[l] if fp32 else H.diag[l]
    inner = H.inner[l]
    nu = H.nu_pre if pre else H.nu_post
    if H.smoother == "jacobi":
        om = np.float32(H.omega) if fp32 else H.omega
        for _ in range(nu):
            r = b - op(H, l, x, fp32)
            x = np.where(inner, x + om * (r / diag), x)
        return x
    order = (0, 1) if pre else (1, 0)
    for _ in range(nu):
        for c in order:
            r = b - op(H, l, x, fp32)
            x = np.where(inner & (H.colour[l] == c), x + r / diag, x)
    return x


def coarse_solve(H, b, fp32=False):
    """Exact solve on the coarsest level (FP64 Cholesky factor)."""
    inner = H.inner[-1]
    rhs = b[inner].astype(np.float64)
    sol = sla.cho_solve(H.coarse_factor, rhs)
    out = np.zeros_like(b)
    out[inner] = sol.astype(b.dtype)
    return out


def cycle(H, l, x, b, kind="V", fp32=False):
    """One cycle of the given kind on level l (Algorithm 1's step order):
    pre-smoothing, restriction of the residual, coarse correction from a
    zero guess (exact directly above the coarsest level, otherwise the
    cycles of CYCLE_SCHEDULE[kind]), prolongation added to x,
    post-smoothing."""
    if l == H.levels - 1:
        return coarse_solve(H, b, fp32)
    x = smooth(H, l, x, b, pre=True, fp32=fp32)
    r = b - op(H, l, x, fp32)
    bc = restrict(H.dim, H.nl[l], r)
    e = np.zeros_like(bc)
    if l + 1 == H.levels - 1:
        e = coarse_solve(H, bc, fp32)
    else:
        for sub in CYCLE_SCHEDULE[kind]:
            e = cycle(H, l + 1, e, bc, sub, fp32)
    x = x + prolong(H.dim, H.nl[l], e)
    x = smooth(H, l, x, b, pre=False, fp32=fp32)
    return x


def norm(v):
    """Euclidean norm over the unknowns (boundary entries are 0)."""
    return float(np.linalg.norm(np.asarray(v, dtype=np.float64).ravel()))


# --------------------------------------------------------------------------
# outer iterations (Sec. 5.5.1)
# --------------------------------------------------------------------------

def iterate(H, b, fp32=False, max_iter=None):
    """Yield (k, u_k, rho_k) for k = 1, 2, ... from u_0 = 0.

    FP64: u_k = cycle(u_{k-1}, b).  FP32-inner (``fp32``): r = b - A u,
    c = float32 cycle from 0 on float32(r / s), u += s c, with s the power
    of two :func:`oracle.mg.ir_scale` of ||b||.
    rho_k = ||b - A u_k|| / ||b|| in FP64.  b is a full-grid FP64 array with
    zero boundary and a nonzero interior."""
    b = np.asarray(b, dtype=np.float64).reshape((H.n + 1,) * H.dim)
    nb = norm(b)
    u = np.zeros_like(b)
    r = b.copy()
    k = 0
    while max_iter is None or k < max_iter:
        k += 1
        if fp32:
            s = ir_scale(nb)
            r32 = (r / s).astype(np.float32)
            c = cycle(H, 0, np.zeros_like(r32), r32, H.cycle, fp32=True)
            u = u + s * c.astype(np.float64)
        else:
            u = cycle(H, 0, u, b, H.cycle)
        r = b - op(H, 0, u)
        yield k, u, norm(r) / nb


def solve(H, b, tol, max_iter=100, fp32=False, diverge=1e3):
    """Cycles from u = 0 until ||b - A u|| / ||b|| <= tol.  Returns
    (u, iters, hist, status) like :func:`oracle.mg.solve` (full-grid u)."""
    b = np.asarray(b, dtype=np.float64).reshape((H.n + 1,) * H.dim)
    if norm(b) == 0.0:
        return np.zeros_like(b), 0, [1.0], "ok"
    hist = [1.0]
    u = None
    for k, u, rho in iterate(H, b, fp32, max_iter):
        hist.append(rho)
        if not np.isfinite(rho) or rho > diverge:
            return u, k, hist, "diverged"
        if rho <= tol:
            return u, k, hist, "ok"
    return u, max_iter, hist, "maxit"
