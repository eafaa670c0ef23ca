"""Grid transfer operators between nested Q1 spaces (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper uses general transfer operators for arbitrary finite element
spaces (Sec. 5.4).  For nested conforming Q1 spaces the coarse space is a
subspace of the fine one, and the canonical prolongation is the natural
injection: a coarse function, written in the fine nodal basis, has as fine
nodal values its multilinear interpolant.  A fine node whose coordinates
have k odd entries lies in the middle of a coarse edge/face/cell and takes
the average of its 2^k coarse neighbours (weight 2^-k each); coarse
boundary values are 0.  Restriction of a residual (a functional) is the
adjoint, R = P^T, with no extra scaling.
"""

import itertools

import numpy as np
import scipy.sparse as sp

from .q1 import interior_coords, n_interior


def prolongation(dim, n_fine):
    """Sparse P of shape (N_I(fine), N_I(coarse)) for n_fine cells per side."""
    if n_fine % 2:
        raise ValueError("n_fine must be even")
    nc = n_fine // 2
    fine = interior_coords(dim, n_fine)               # x, y[, z] arrays
    nf_rows = n_interior(dim, n_fine)
    rows, cols, vals = [], [], []
    # o[d] = 0: lower (or only) coarse parent in direction d; 1: upper parent
    for o in itertools.product((0, 1), repeat=dim):
        keep = np.ones(nf_rows, dtype=bool)
        weight = np.ones(nf_rows)
        parent = []
        for d in range(dim):
            i = fine[d]
            odd = (i % 2) == 1
            if o[d] == 0:
                I = i // 2                       # even: i/2 ; odd: (i-1)/2
                w = np.where(odd, 0.5, 1.0)
            else:
                I = i // 2 + 1                   # odd only: (i+1)/2
                w = np.where(odd, 0.5, 0.0)
                keep &= odd
            keep &= (I >= 1) & (I <= nc - 1)     # coarse boundary value is 0
            weight = weight * w
            parent.append(I)
        col = np.zeros(nf_rows, dtype=np.int64)
        stride = 1
        for d in range(dim):
            col += (parent[d] - 1) * stride
            stride *= nc - 1
        rows.append(np.nonzero(keep)[0])
        cols.append(col[keep])
        vals.append(weight[keep])
    P = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(nf_rows, n_interior(dim, nc)),
    ).tocsr()
    P.sum_duplicates()
    return P


def restriction(dim, n_fine):
    """R = P^T (weights 1, 1/2, 1/4, 1/8; each fine node's weights sum to 1)."""
    return prolongation(dim, n_fine).T.tocsr()
