"""Q1 finite elements on the uniform mesh of the unit square / cube (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions used throughout the oracle:

* A mesh of ``n`` cells per direction has mesh width h = 1/n and nodes
  x_i = i*h, i in {0..n}^d.  A "full-grid" array is a NumPy array of shape
  ``(n+1,)*d`` indexed ``[z, y, x]`` (3D) or ``[y, x]`` (2D), so that its
  C-order flattening has x fastest.  Cells are indexed the same way with shape
  ``(n,)*d``; cell c spans [c, c+1]^d in node coordinates.
* The unknowns are the interior nodes {1..n-1}^d, numbered lexicographically
  with x fastest.  Homogeneous Dirichlet boundary nodes are eliminated (their
  rows and columns are dropped); the paper keeps Dirichlet DOFs apart from the
  others in its DOF reordering (Sec. 4.2.6).
* A local vertex of a cell is v in {0,1}^d with local number
  a = v_x + 2 v_y + 4 v_z.

The system is the standard Galerkin discretisation assembled cell by cell
(Sec. 2): the stiffness matrix of -div(kappa grad u) with kappa constant on
each cell, plus sigma times the mass matrix when a shift sigma >= 0 is
given (the Crank-Nicolson step of the heat equation of Sec. 6.2, scaled by
2/dt, has the matrix K + (2/dt) M).
"""

import itertools

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# element level
# --------------------------------------------------------------------------

def element_factors(h):
    """1D Q1 element stiffness k and mass m on an interval of length h.

    With the two linear basis functions of [0, h]:
    k_ab = int phi_a' phi_b' = (1/h) [[1, -1], [-1, 1]],
    m_ab = int phi_a phi_b   = (h/6) [[2, 1], [1, 2]].
    """
    k = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m = np.array([[2.0, 1.0], [1.0, 2.0]]) * (h / 6.0)
    return k, m


def element_mass(dim, h):
    """Q1 element mass matrix on a cube of side h: the tensor product of
    the 1D mass factors, M_e[a, b] = prod_d m[v_d, w_d]."""
    _, m = element_factors(h)
    verts = local_vertices(dim)
    nv = len(verts)
    Me = np.zeros((nv, nv))
    for a, v in enumerate(verts):
        for b, w in enumerate(verts):
            p = 1.0
            for d in range(dim):
                p *= m[v[d], w[d]]
            Me[a, b] = p
    return Me


def local_vertices(dim):
    """Local vertices v (tuples (v_x, v_y[, v_z])) in local-number order."""
    # itertools.product varies the last entry fastest; reverse each tuple so
    # that v_x varies fastest and local number a = v_x + 2 v_y + 4 v_z.
    return [tuple(reversed(t)) for t in itertools.product((0, 1), repeat=dim)]


def element_matrix(dim, h):
    """Q1 element stiffness matrix for kappa = 1 on a cube of side h.

    The Q1 basis is the tensor product of 1D linear bases, so the gradient
    bilinear form splits into a sum over directions d of products of 1D
    factors: K_e = sum_d prod_e F_e, F_e = k if e == d else m.
    """
    k, m = element_factors(h)
    verts = local_vertices(dim)
    nv = len(verts)
    K = np.zeros((nv, nv))
    for a, v in enumerate(verts):
        for b, w in enumerate(verts):
            s = 0.0
            for d in range(dim):
                p = 1.0
                for e in range(dim):
                    f = k if e == d else m
                    p *= f[v[e], w[e]]
                s += p
            K[a, b] = s
    return K


# --------------------------------------------------------------------------
# numbering helpers
# --------------------------------------------------------------------------

def n_interior(dim, n):
    """Number of unknowns (n-1)^d."""
    return (n - 1) ** dim


def _vslice(v, n):
    """Slices of a full-grid array selecting vertex v of every cell.

    Array axes are ordered [z, y, x], v is (v_x, v_y[, v_z]).
    """
    return tuple(slice(vi, vi + n) for vi in reversed(v))


def _interior_map(dim, n):
    """Full-grid array of interior-unknown numbers (-1 on the boundary)."""
    imap = -np.ones((n + 1,) * dim, dtype=np.int64)
    inner = tuple(slice(1, n) for _ in range(dim))
    imap[inner] = np.arange(n_interior(dim, n)).reshape((n - 1,) * dim)
    return imap


def interior_coords(dim, n):
    """Integer coordinates (x, y[, z]) of the unknowns, in unknown order."""
    grids = np.meshgrid(*[np.arange(1, n)] * dim, indexing="ij")
    # grids[0] is the slowest axis (z in 3D); return x, y, z order
    return [g.ravel() for g in reversed(grids)]


def to_full(dim, n, x_int):
    """Embed an interior vector into a full-grid array (boundary = 0)."""
    full = np.zeros((n + 1,) * dim, dtype=np.asarray(x_int).dtype)
    inner = tuple(slice(1, n) for _ in range(dim))
    full[inner] = np.asarray(x_int).reshape((n - 1,) * dim)
    return full


def to_interior(dim, n, x_full):
    """Extract the interior vector from a full-grid array."""
    x_full = np.asarray(x_full).reshape((n + 1,) * dim)
    inner = tuple(slice(1, n) for _ in range(dim))
    return x_full[inner].ravel().copy()


def _cells(dim, n, kappa):
    if kappa is None:
        return np.ones((n,) * dim)
    kappa = np.asarray(kappa, dtype=np.float64).reshape((n,) * dim)
    return kappa


# --------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------

def assemble(dim, n, kappa=None, sigma=0.0):
    """Global matrix K + sigma M on the unknowns, assembled cell by cell.

    For every cell c and every pair of local vertices (a, b) whose nodes are
    both interior, kappa_c * K_e[a, b] + sigma * M_e[a, b] is added to
    A[node_a, node_b] (Sec. 2; the paper stores its matrices in CSR,
    Sec. 6.1).  ``kappa`` is an array of n^d cell values (x fastest) or None
    for kappa = 1; the mass term is not weighted by kappa.
    Returns a SciPy CSR matrix of shape (N_I, N_I).
    """
    h = 1.0 / n
    Ke = element_matrix(dim, h)
    Me = element_mass(dim, h)
    kap = _cells(dim, n, kappa)
    imap = _interior_map(dim, n)
    NI = n_interior(dim, n)
    verts = local_vertices(dim)
    rows, cols, vals = [], [], []
    for a, v in enumerate(verts):
        ia = imap[_vslice(v, n)]
        for b, w in enumerate(verts):
            # zero element entries (face pairs in 3D without a mass term)
            # are kept as explicit zeros: the structural pattern is every
            # pair of nodes sharing a cell, 3^d per interior row away from
            # the boundary
            ib = imap[_vslice(w, n)]
            mask = (ia >= 0) & (ib >= 0)
            rows.append(ia[mask].astype(np.int32))
            cols.append(ib[mask].astype(np.int32))
            vals.append(kap[mask] * Ke[a, b] + sigma * Me[a, b])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(NI, NI)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def assemble_full(dim, n):
    """Stiffness K and mass M (kappa = 1) over every node of the grid,
    boundary nodes included, assembled cell by cell; rows and columns are
    the full-grid node numbers (x fastest).  Used where Dirichlet data
    enters a right-hand side."""
    h = 1.0 / n
    Ke = element_matrix(dim, h)
    Me = element_mass(dim, h)
    N = (n + 1) ** dim
    num = np.arange(N).reshape((n + 1,) * dim)
    verts = local_vertices(dim)
    rows, cols, kv, mv = [], [], [], []
    for a, v in enumerate(verts):
        ia = num[_vslice(v, n)].ravel()
        for b, w in enumerate(verts):
            ib = num[_vslice(w, n)].ravel()
            rows.append(ia)
            cols.append(ib)
            kv.append(np.full(ia.size, Ke[a, b]))
            mv.append(np.full(ia.size, Me[a, b]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(kv), (rows, cols)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (rows, cols)), shape=(N, N)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def apply_matfree(dim, n, kappa, x_full, sigma=0.0):
    """y = A x on the full grid, cell by cell, without forming A.

    Same cell-by-cell definition as :func:`assemble` (with the mass shift
    sigma); boundary values of x are treated as 0 (eliminated) and boundary
    values of y are set to 0.
    """
    h = 1.0 / n
    Ke = element_matrix(dim, h)
    Me = element_mass(dim, h)
    kap = _cells(dim, n, kappa)
    x = np.array(x_full, dtype=np.float64).reshape((n + 1,) * dim)
    _zero_boundary(x)
    y = np.zeros_like(x)
    verts = local_vertices(dim)
    for a, v in enumerate(verts):
        acc = np.zeros((n,) * dim)
        accm = np.zeros((n,) * dim)
        for b, w in enumerate(verts):
            if Ke[a, b] != 0.0:
                acc += Ke[a, b] * x[_vslice(w, n)]
            if sigma != 0.0:
                accm += Me[a, b] * x[_vslice(w, n)]
        y[_vslice(v, n)] += kap * acc + sigma * accm
    _zero_boundary(y)
    return y


def apply_rows(dim, n, kappa, x_full, nodes, sigma=0.0):
    """(A x)_p for a list of interior nodes p, each computed on its own.

    ``nodes`` is an integer array of shape (S, dim) with columns (x, y[, z]).
    For node p and each of the 2^d cells containing it (p is local vertex a
    of that cell), the cell adds sum_w (kappa_c K_e[a, w] + sigma M_e[a, w])
    x[cell + w].  Boundary values of x are treated as 0.
    """
    h = 1.0 / n
    Ke = element_matrix(dim, h)
    Me = element_mass(dim, h)
    kap = _cells(dim, n, kappa)
    x = np.array(x_full, dtype=np.float64).reshape((n + 1,) * dim)
    _zero_boundary(x)
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, dim)
    verts = local_vertices(dim)
    out = np.zeros(nodes.shape[0])
    for a, v in enumerate(verts):
        cell = nodes - np.array(v)            # (S, dim) in (x, y, z) order
        kc = kap[tuple(cell[:, d] for d in reversed(range(dim)))]
        acc = np.zeros(nodes.shape[0])
        accm = np.zeros(nodes.shape[0])
        for b, w in enumerate(verts):
            q = cell + np.array(w)
            xv = x[tuple(q[:, d] for d in reversed(range(dim)))]
            acc += Ke[a, b] * xv
            accm += Me[a, b] * xv
        out += kc * acc + sigma * accm
    return out


def _zero_boundary(full):
    d = full.ndim
    for ax in range(d):
        idx = [slice(None)] * d
        idx[ax] = 0
        full[tuple(idx)] = 0.0
        idx[ax] = -1
        full[tuple(idx)] = 0.0


def assemble_load_quadrature(dim, n, f, q=6):
    """Load vector b_i = int f phi_i by tensor Gauss-Legendre quadrature.

    ``f`` maps coordinate arrays (x, y[, z]) to values.  q points per
    direction on every cell.  Returns the interior vector.
    """
    h = 1.0 / n
    xi, wq = np.polynomial.legendre.leggauss(q)
    xi = 0.5 * (xi + 1.0)           # points on (0, 1)
    wq = 0.5 * wq
    cell_lo = [np.arange(n) * h] * dim
    verts = local_vertices(dim)
    full = np.zeros((n + 1,) * dim)
    for qp in itertools.product(range(q), repeat=dim):
        # qp[d] is the point index in direction d (x, y, z)
        coords = np.meshgrid(*[cell_lo[d] + xi[qp[d]] * h
                               for d in reversed(range(dim))], indexing="ij")
        coords = list(reversed(coords))          # x, y, z
        fv = f(*coords) * np.prod([wq[qp[d]] for d in range(dim)]) * h ** dim
        for v in verts:
            phi = 1.0
            for d in range(dim):
                s = xi[qp[d]]
                phi *= s if v[d] else (1.0 - s)
            full[_vslice(v, n)] += fv * phi
    return to_interior(dim, n, full)


# --------------------------------------------------------------------------
# coefficient hierarchy
# --------------------------------------------------------------------------

def kappa_coarsen(dim, n, kappa):
    """Coarse-cell coefficient: geometric mean of its 2^d children.

    The coarse operators are rediscretised on every level; the coarse cell
    value is exp(mean(log kappa_child)).  ``kappa`` holds n^d fine cells,
    x fastest; returns (n/2)^d coarse cells.
    """
    nc = n // 2
    k = np.asarray(kappa, dtype=np.float64).reshape((nc, 2) * dim)
    g = np.log(k).mean(axis=tuple(range(1, 2 * dim, 2)))
    return np.exp(g).ravel()


def kappa_hierarchy(dim, n, levels, kappa):
    """[kappa_0 (finest), ..., kappa_{L-1}]; None entries for kappa = 1."""
    out = [None if kappa is None else np.asarray(kappa, dtype=np.float64).ravel()]
    nl = n
    for _ in range(1, levels):
        out.append(None if out[-1] is None else kappa_coarsen(dim, nl, out[-1]))
        nl //= 2
    return out
