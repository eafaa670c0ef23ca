// Internal interfaces of the Q1 multigrid library: level geometry, operator
// descriptors and the host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

// Geometry of one level: n cells per direction, (n+1)^dim nodes, x fastest.
struct Geo {
  int dim;
  int n;      // cells per direction
  long sy;    // node stride in y  (= n+1)
  long sz;    // node stride in z  (= (n+1)^2, 0 in 2D)
  long nodes; // (n+1)^dim
};

inline Geo make_geo(int dim, int n) {
  Geo g;
  g.dim = dim;
  g.n = n;
  g.sy = n + 1;
  g.sz = dim == 3 ? (long)(n + 1) * (n + 1) : 0;
  g.nodes = dim == 3 ? (long)(n + 1) * (n + 1) * (n + 1) : (long)(n + 1) * (n + 1);
  return g;
}

// Largest coarsest system (unknowns) solved by the one-block Cholesky kernel.
constexpr int kCoarseMaxUnknowns = 4096;

enum OpKind { OP_CONST = 0, OP_KAPPA = 1 };

// Matrix-free Q1 operator of one level.
//  OP_CONST: kappa = 1, the assembled stencil weights
//     2D: wc = 8/3, w1 = -1/3 (x/y neighbours), w2 = -1/3 (diagonals)
//     3D: wc = 8h/3, w1 = -h/6 (edge neighbours), w2 = -h/12 (corners);
//         face neighbours have weight 0.
//  OP_KAPPA: kappa per cell; element matrix scale s = 1/6 (2D), h/12 (3D).
template <typename T>
struct StencilOp {
  int kind;
  const T* kappa;  // n^dim cells, x fastest
  T wc, w1, w2;
  T s;
};

// CSR operator of one level.  Rows are the unknowns, blocked by colour
// (colour 0 rows first); row r is node rowmap[r] of the full grid; column
// indices are full-grid node indices; the diagonal entry is stored first.
template <typename T>
struct CsrOp {
  const int* rowptr;
  const int* col;
  const T* val;
  const int* rowmap;
  int rows;
  int coff[3];  // colour c rows: [coff[c], coff[c+1])
};

// Smoothing step kinds (mg_apply_smooth "step" 0..2).
enum SmoothKind { SM_JACOBI = 0, SM_RB0 = 1, SM_RB1 = 2 };

// ---- grid kernels (kernels_grid.hip) -------------------------------------
template <typename T> void launch_fill(T* v, long count, T val, hipStream_t s);
template <typename T> void launch_copy(const T* a, T* b, long count, hipStream_t s);

// Number of per-block partial sums written by the norm-producing launches.
long grid_blocks(const Geo& g);

template <typename T>
void launch_residual(const Geo& g, const StencilOp<T>& op, const T* x,
                     const T* b, T* r, double* partials, hipStream_t s);
template <typename T>
void launch_smooth(const Geo& g, const StencilOp<T>& op, int kind,
                   const T* xin, const T* b, T* xout, T omega, hipStream_t s);
template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const T* r, T* bc,
                     hipStream_t s);
template <typename T>
void launch_resid_restrict(const Geo& gf, const Geo& gc, const StencilOp<T>& op,
                           const T* x, const T* b, T* bc, hipStream_t s);
template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const T* e, T* x,
                        hipStream_t s);
template <typename T>
void launch_coarse_solve(const Geo& gc, const double* L, int m, const T* bc,
                         T* xc, hipStream_t s);
template <typename T>
void launch_norm2_partial(const Geo& g, const T* v, double* partials,
                          hipStream_t s);
void launch_reduce_final(const double* partials, long count, double* out,
                         hipStream_t s);
void launch_scale_cast(const Geo& g, const double* r, const double* norm2,
                       float* b32, hipStream_t s);
void launch_ir_update(const Geo& g, double* u, const float* c,
                      const double* norm2, hipStream_t s);
void launch_kappa_coarsen(int dim, int nf, const double* kf, double* kc,
                          hipStream_t s);
void launch_cast_f32(const double* a, float* b, long count, hipStream_t s);
void launch_count_bad_kappa(const double* k, long count, int* bad_nonpos,
                            int* bad_nonfinite, hipStream_t s);

// ---- CSR kernels (kernels_csr.hip) ----------------------------------------
template <typename T>
void launch_csr_build(const Geo& g, const double* kappa, double s_elem, int rows,
                      const int* rowmap, const int* rowptr, int* col, T* val,
                      hipStream_t s);
template <typename T>
void launch_csr_residual(const Geo& g, const CsrOp<T>& A, const T* x,
                         const T* b, T* r, double* partials, hipStream_t s);
long csr_residual_blocks(int rows);
template <typename T>
void launch_csr_smooth(const Geo& g, const CsrOp<T>& A, int kind,
                       const T* xin, const T* b, T* xout, T omega,
                       hipStream_t s);

}  // namespace mg
