"""Exact references for the Q1 system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

These give the limit of the multigrid iteration, u* = A^-1 b, by routes
that share nothing with the V-cycle, and are used to pin the oracle itself.
"""

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def dst_eigenvalues(dim, n, sigma=0.0):
    """Eigenvalues of the kappa = 1 Q1 matrix K + sigma M on the sine basis.

    The 1D Q1 stiffness and mass matrices on the unknowns are the
    tridiagonal (1/h) tri(-1, 2, -1) and (h/6) tri(1, 4, 1); both are
    diagonalised by the sine vectors sin(pi k i / n), k = 1..n-1, with
    eigenvalues k^(k) = (2/h)(1 - cos(pi k/n)) and
    m^(k) = (h/3)(2 + cos(pi k/n)).  The d-dimensional matrix is the sum
    over directions of Kronecker products (stiffness in one direction, mass
    in the others) and the mass matrix the Kronecker product of the 1D mass
    matrices, so the eigenvalue for mode (k_x, k_y[, k_z]) is
    sum_d k^(k_d) prod_{e != d} m^(k_e) + sigma prod_d m^(k_d).  Returned as
    a full array of shape (n-1,)*dim indexed [k_z, k_y, k_x].
    """
    h = 1.0 / n
    k = np.arange(1, n)
    c = np.cos(np.pi * k / n)
    kh = (2.0 / h) * (1.0 - c)
    mh = (h / 3.0) * (2.0 + c)
    lam = np.zeros((n - 1,) * dim)
    for d in range(dim):
        term = np.ones((n - 1,) * dim)
        for e in range(dim):
            v = kh if e == d else mh
            shape = [1] * dim
            shape[dim - 1 - e] = n - 1          # axis of direction e
            term = term * v.reshape(shape)
        lam += term
    if sigma != 0.0:
        mass = np.ones((n - 1,) * dim)
        for e in range(dim):
            shape = [1] * dim
            shape[dim - 1 - e] = n - 1
            mass = mass * mh.reshape(shape)
        lam += sigma * mass
    return lam


def dst_solve(dim, n, b_int, sigma=0.0):
    """u* = A^-1 b for kappa = 1 (A = K + sigma M) by DST-I
    diagonalisation, any size."""
    B = np.asarray(b_int, dtype=np.float64).reshape((n - 1,) * dim)
    Bh = sfft.dstn(B, type=1, norm="ortho")
    U = sfft.idstn(Bh / dst_eigenvalues(dim, n, sigma), type=1, norm="ortho")
    return U.ravel()


def dense_solve(A, b):
    """Dense Cholesky solve (tiny systems); raises if A is not SPD."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    c = sla.cho_factor(Ad, lower=True)
    return sla.cho_solve(c, b)


def sparse_solve(A, b):
    """Sparse LU solve (moderate systems)."""
    return spla.splu(A.tocsc()).solve(np.asarray(b, dtype=np.float64))


def manufactured_factor(dim, h):
    """alpha_d(h): discrete solution / nodal values for u = prod sin(pi x_d).

    With the exactly integrated load of f = d pi^2 prod sin(pi x_d), the
    load vector is a multiple of the lowest sine mode, so the discrete
    solution is alpha_d(h) times the nodal interpolant, with
    alpha_d(h) = [6 (1 - cos pi h) / ((pi h)^2 (2 + cos pi h))]^(d-1).
    """
    ph = np.pi * h
    return (6.0 * (1.0 - np.cos(ph)) / (ph * ph * (2.0 + np.cos(ph)))) ** (dim - 1)
