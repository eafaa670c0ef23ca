"""FP64 CPU oracle for the Q1 geometric-multigrid V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package; only the
test suite, the smoke check and the benchmark's CPU-baseline leg use it.  It
shares no code with the GPU path.

What it computes, and where the paper defines it:

* the linear system A x = b from the standard Galerkin finite element method
  (Sec. 2 and Sec. 6.2), specialised to conforming Q1 elements on the unit
  square / cube with homogeneous Dirichlet data on nested uniform meshes
  (Sec. 5.1);
* the multigrid V-cycle of Algorithm 1 (Sec. 5.3): pre-smoothing, residual
  restriction, exact coarsest solve, prolongation plus correction,
  post-smoothing, with Jacobi or Gauss-Seidel smoothing (Eq. (1));
* canonical Q1 transfer operators: multilinear interpolation P and its
  adjoint R = P^T (Sec. 5.4, read for nested conforming Q1 spaces);
* the outer fixed-point iteration of cycles (Sec. 5.5.1);
* an FP32-inner / FP64-outer iterative-refinement wrapper of that iteration
  (float32 correction cycles on the residual scaled by a power of two);
* conjugate gradients preconditioned by one V-cycle per iteration
  (multigrid as a Krylov preconditioner, Sec. 1), in FP64 or with the
  cycle in FP32;
* the mass-shifted matrix K + sigma M, warm-started solves and the
  Crank-Nicolson time loop of the heat-equation model problem (Sec. 6.2;
  module ``oracle.heat``);
* independent exact references (dense Cholesky, DST-I diagonalisation,
  sparse LU) used only to pin the rest;
* the same cycle and outer iterations matrix-free on full-grid arrays
  (module ``oracle.matfree``: A applied cell by cell, never assembled), for
  the 256^3 and 192^3 systems whose assembled matrices do not fit.

Everything is plain NumPy/SciPy in float64 (float32 only inside the
iterative-refinement inner cycle, by definition of that mode).
"""

from .q1 import (
    element_factors,
    element_matrix,
    element_mass,
    n_interior,
    interior_coords,
    assemble,
    assemble_full,
    assemble_load_quadrature,
    apply_matfree,
    apply_rows,
    kappa_coarsen,
    kappa_hierarchy,
    to_full,
    to_interior,
)
from .transfer import prolongation, restriction
from .mg import (
    Hierarchy,
    build_hierarchy,
    cycle,
    CYCLE_SCHEDULE,
    jacobi_sweep,
    rb_half_sweep,
    smooth,
    vcycle,
    solve,
    solve_ir,
    solve_pcg,
    ir_scale,
    precondition,
    colour_mask,
)
from .exact import (
    dst_eigenvalues,
    dst_solve,
    dense_solve,
    sparse_solve,
    manufactured_factor,
)

__all__ = [
    "element_factors", "element_matrix", "element_mass", "n_interior",
    "interior_coords", "assemble", "assemble_full", "assemble_load_quadrature", "apply_matfree", "apply_rows",
    "kappa_coarsen", "kappa_hierarchy", "to_full", "to_interior",
    "prolongation", "restriction",
    "Hierarchy", "build_hierarchy", "jacobi_sweep", "rb_half_sweep", "smooth",
    "vcycle", "solve", "solve_ir", "ir_scale", "colour_mask",
    "dst_eigenvalues", "dst_solve", "dense_solve", "sparse_solve",
    "manufactured_factor",
]
