// Grid kernels of the Q1 multigrid V-cycle for gfx950: matrix-free operator
// application (residual, smoothers), grid transfers, coarsest solve, norms,
// the iterative-refinement helpers and the one-workgroup V-cycle on the
// coarse "tail" levels.
//
// Every node kernel is batched: blockIdx.z enumerates (request, z plane),
// and each request's buffers come from the launch's Batch.  A single solve
// is a batch of one, so a request computes bitwise the same alone and fused
// with others.
//
// Thread layout of the node kernels: a block of 64 x 4 threads covers 64
// consecutive x and 4 consecutive y of one z plane of interior nodes, so one
// wavefront (64 lanes) reads 64 consecutive values of a grid row.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "mg_internal.h"

namespace mg {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int TAIL_THREADS = 1024;

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

inline dim3 node_grid(const Geo& g, int count) {
  const long m = g.n - 1;  // interior nodes per direction
  return dim3(cdiv(m, BX), cdiv(m, BY), g.dim == 3 ? (unsigned)(m * count) : (unsigned)count);
}

// Sum of v over the 256 threads of a 64x4 block; result valid in thread
// (0,0).  Wave-level butterfly, then the four wave sums in a fixed order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double ws[BY];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (threadIdx.x == 0) ws[threadIdx.y] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0 && threadIdx.y == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  return t;
}

// Level geometry as seen by device code.
struct DGeo {
  int n;
  long sy, sz;
};

__device__ __forceinline__ DGeo dgeo(const Geo& g) { return DGeo{g.n, g.sy, g.sz}; }
__device__ __forceinline__ DGeo dgeo(int dim, int n) {
  return DGeo{n, (long)(n + 1), dim == 3 ? (long)(n + 1) * (n + 1) : 0L};
}

// ---------------------------------------------------------------------------
// Operator application at one interior node p = (i, j[, k]).
// at():   (A x)_p in ax and the diagonal entry a_pp in dg.
// diag(): a_pp only.
// ---------------------------------------------------------------------------
template <typename T, int DIM, int KIND>
struct Apply;

// 2D, kappa = 1: 8/3 centre, -1/3 for all eight neighbours.
template <typename T>
struct Apply<T, 2, OP_CONST> {
  __device__ static void at(const StencilParams<T>& op, const T*, const DGeo& g,
                            const T* __restrict__ x, long p, int, int, int, T& ax, T& dg) {
    const long sy = g.sy;
    T f = (x[p - 1] + x[p + 1]) + (x[p - sy] + x[p + sy]);
    T c = (x[p - 1 - sy] + x[p + 1 - sy]) + (x[p - 1 + sy] + x[p + 1 + sy]);
    ax = op.wc * x[p] + op.w1 * f + op.w2 * c;
    dg = op.wc;
  }
  __device__ static T diag(const StencilParams<T>& op, const T*, const DGeo&, int, int, int) {
    return op.wc;
  }
};

// 3D arithmetic; shared by every kernel that applies the 3D operator (the
// node kernels and the tail on a 3x3x3 neighbourhood v[dz+1][dy+1][dx+1],
// the plane-marching sweep kernel on per-plane windows), so that all of
// them round identically.  The operator is written as a sum of per-plane
// parts so that a kernel marching in z can form each part when its plane is
// at hand.
//
// kappa = 1: 8h/3 centre, -h/6 on the 12 edge neighbours, -h/12 on the
// 8 corners, 0 on the 6 face neighbours.  Parts of one plane, in a window
// w[dy+1][c] whose node column is c = u+1:
//   xe = x-edge pair of the centre row, ye = y-edge pair of the centre
//   column, q = the four corners (for the node's own plane: its in-plane
//   edge neighbours).
template <typename T, typename W>
__device__ __forceinline__ void plane_parts(const W& w, int u, T& xe, T& ye, T& q) {
  xe = w[1][u] + w[1][u + 2];
  ye = w[0][u + 1] + w[2][u + 1];
  q = (w[0][u] + w[0][u + 2]) + (w[2][u] + w[2][u + 2]);
}

// A x at a node from the parts: xc its value, g the corners of its own
// plane, (a0, b0, c0) / (a1, b1, c1) the parts of the planes below / above.
template <typename T>
__device__ __forceinline__ T stencil3_const_sum(const StencilParams<T>& op, T xc, T g, T a0, T a1,
                                                T b0, T b1, T c0, T c1) {
  const T e = (g + (a0 + a1)) + (b0 + b1);
  const T c = c0 + c1;
  return op.wc * xc + op.w1 * e + op.w2 * c;
}

template <typename T, typename V>
__device__ __forceinline__ T stencil3_const(const StencilParams<T>& op, const V& v) {
  T a0, b0, c0, a1, b1, c1, ea, eb, g;
  plane_parts<T>(v[0], 0, a0, b0, c0);
  plane_parts<T>(v[2], 0, a1, b1, c1);
  plane_parts<T>(v[1], 0, ea, eb, g);
  return stencil3_const_sum(op, v[1][1][1], g, a0, a1, b0, b1, c0, c1);
}

// K + sigma M (kappa = 1): every neighbour is coupled.  The same parts as
// for kappa = 1 plus the face neighbours: fo = the x- and y-faces of the
// node's own plane (the xe + ye parts of that plane), z0 / z1 = the centre
// values of the planes below / above.
template <typename T>
__device__ __forceinline__ T stencil3_mass_sum(const StencilParams<T>& op, T xc, T g, T fo, T a0,
                                               T a1, T b0, T b1, T c0, T c1, T z0, T z1) {
  const T e = (g + (a0 + a1)) + (b0 + b1);
  const T c = c0 + c1;
  const T f = fo + (z0 + z1);
  return op.wc * xc + op.wf * f + op.w1 * e + op.w2 * c;
}

template <typename T, typename V>
__device__ __forceinline__ T stencil3_mass(const StencilParams<T>& op, const V& v) {
  T a0, b0, c0, a1, b1, c1, fa, fb, g;
  plane_parts<T>(v[0], 0, a0, b0, c0);
  plane_parts<T>(v[2], 0, a1, b1, c1);
  plane_parts<T>(v[1], 0, fa, fb, g);
  return stencil3_mass_sum(op, v[1][1][1], g, fa + fb, a0, a1, b0, b1, c0, c1, v[0][1][1],
                           v[2][1][1]);
}

// kappa per cell: cell (c, b, a) of the eight around p (sides sx = 2a-1,
// sy = 2b-1, sz = 2c-1) with coefficient kappa_abc contributes
//   kappa_abc * h/12 * (4 x_p - x_{p+sx+sy} - x_{p+sx+sz} - x_{p+sy+sz}
//                       - x_{p+sx+sy+sz});
// face neighbours have element weight 0.  Summed by planes:
//   A x = h/12 (P - (Q + R)),  P = sum_cells kappa (4 x_p - x_{p+sx+sy}),
//   Q = sum over the 4 cells below of kappa (x_{p+sx+sz} + x_{p+sy+sz} +
//   x_{p+sx+sy+sz}), R = the same over the 4 cells above; diagonal
//   h/12 * 4 * sum_cells kappa.  A cell layer window kw[b][c] holds the
//   cells on the node's y sides b, x side c - u (node column u+1 of w).
template <typename T, typename KW, typename W>
__device__ __forceinline__ T kappa_side(const KW& kw, const W& w, int u) {
  T q = 0;
#pragma unroll
  for (int bb = 0; bb < 2; ++bb)
#pragma unroll
    for (int a = 0; a < 2; ++a)
      q += kw[bb][u + a] * ((w[1][u + 2 * a] + w[2 * bb][u + 1]) + w[2 * bb][u + 2 * a]);
  return q;
}

template <typename T, typename KW, typename W>
__device__ __forceinline__ void kappa_plane(const KW& kwlo, const KW& kwhi, const W& w, int u,
                                            T& P, T& ks) {
  const T xp = w[1][u + 1];
  P = 0;
  ks = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T kc = c ? kwhi[bb][u + a] : kwlo[bb][u + a];
        P += kc * (T(4) * xp - w[2 * bb][u + 2 * a]);
        ks += kc;
      }
}

template <typename T, typename KW>
__device__ __forceinline__ T kappa_cell_sum(const KW& kwlo, const KW& kwhi, int u) {
  T ks = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) ks += c ? kwhi[bb][u + a] : kwlo[bb][u + a];
  return ks;
}

template <typename T, typename V, typename K>
__device__ __forceinline__ T stencil3_kappa(const StencilParams<T>& op, const K& kk, const V& v,
                                            T& dg) {
  T P, ks;
  kappa_plane<T>(kk[0], kk[1], v[1], 0, P, ks);
  const T Q = kappa_side<T>(kk[0], v[0], 0);
  const T R = kappa_side<T>(kk[1], v[2], 0);
  dg = op.s * T(4) * ks;
  return op.s * (P - (Q + R));
}

template <typename T, typename K>
__device__ __forceinline__ T kappa_diag3(const StencilParams<T>& op, const K& kk) {
  return op.s * T(4) * kappa_cell_sum<T>(kk[0], kk[1], 0);
}

template <typename T>
__device__ __forceinline__ void gather27(const T* __restrict__ x, long p, long sy, long sz,
                                         T (&v)[3][3][3]) {
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) v[dz][dy][dx] = x[p + (dx - 1) + (dy - 1) * sy + (dz - 1) * sz];
}

template <typename T>
__device__ __forceinline__ void gather_cells3(const T* __restrict__ kp, long n, T (&kk)[2][2][2]) {
  const long cz = n * n;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) kk[c][b][a] = kp[a + n * b + cz * c];
}

template <typename T>
struct Apply<T, 3, OP_CONST> {
  __device__ static void at(const StencilParams<T>& op, const T*, const DGeo& g,
                            const T* __restrict__ x, long p, int, int, int, T& ax, T& dg) {
    T v[3][3][3];
    gather27(x, p, g.sy, g.sz, v);  // face entries are loaded but carry weight 0
    ax = stencil3_const(op, v);
    dg = op.wc;
  }
  __device__ static T diag(const StencilParams<T>& op, const T*, const DGeo&, int, int, int) {
    return op.wc;
  }
};

template <typename T>
struct Apply<T, 3, OP_MASS> {
  __device__ static void at(const StencilParams<T>& op, const T*, const DGeo& g,
                            const T* __restrict__ x, long p, int, int, int, T& ax, T& dg) {
    T v[3][3][3];
    gather27(x, p, g.sy, g.sz, v);
    ax = stencil3_mass(op, v);
    dg = op.wc;
  }
  __device__ static T diag(const StencilParams<T>& op, const T*, const DGeo&, int, int, int) {
    return op.wc;
  }
};

// 2D, kappa per cell.  Cell (a, b) of the four around p (a, b in {0,1}, on
// the side sx = 2a-1, sy = 2b-1) contributes
//   kappa_ab / 6 * (4 x_p - x_{p+sx} - x_{p+sy} - 2 x_{p+sx+sy}).
template <typename T>
struct Apply<T, 2, OP_KAPPA> {
  __device__ static void at(const StencilParams<T>& op, const T* __restrict__ kappa,
                            const DGeo& g, const T* __restrict__ x, long p, int i, int j, int,
                            T& ax, T& dg) {
    const long sy = g.sy;
    const long n = g.n;
    const T* kp = kappa + (i - 1) + n * (j - 1);
    const T xp = x[p];
    T acc = 0, ks = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T kc = kp[a + n * b];
        const long dx = a ? 1 : -1;
        const long dy = b ? sy : -sy;
        acc += kc * (T(4) * xp - x[p + dx] - x[p + dy] - T(2) * x[p + dx + dy]);
        ks += kc;
      }
    }
    ax = op.s * acc;
    dg = op.s * T(4) * ks;
  }
  __device__ static T diag(const StencilParams<T>& op, const T* __restrict__ kappa,
                           const DGeo& g, int i, int j, int) {
    const long n = g.n;
    const T* kp = kappa + (i - 1) + n * (j - 1);
    T ks = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) ks += kp[a + n * b];
    return op.s * T(4) * ks;
  }
};

// 3D, kappa per cell (stencil3_kappa).
template <typename T>
struct Apply<T, 3, OP_KAPPA> {
  __device__ static void at(const StencilParams<T>& op, const T* __restrict__ kappa,
                            const DGeo& g, const T* __restrict__ x, long p, int i, int j, int k,
                            T& ax, T& dg) {
    const long n = g.n;
    T kk[2][2][2];
    gather_cells3(kappa + (i - 1) + n * (j - 1) + n * n * (k - 1), n, kk);
    T v[3][3][3];
    gather27(x, p, g.sy, g.sz, v);
    ax = stencil3_kappa(op, kk, v, dg);
  }
  __device__ static T diag(const StencilParams<T>& op, const T* __restrict__ kappa,
                           const DGeo& g, int i, int j, int k) {
    const long n = g.n;
    T kk[2][2][2];
    gather_cells3(kappa + (i - 1) + n * (j - 1) + n * n * (k - 1), n, kk);
    return kappa_diag3(op, kk);
  }
};

// ---------------------------------------------------------------------------
// Per-node steps, shared by the grid kernels and the tail kernel so that
// both compute bitwise the same values.
// ---------------------------------------------------------------------------

// New value of unknown p for one smoothing step.  KS = SM_JACOBI: every
// unknown gets x + omega (b - A x)/a_pp; SM_RB0/SM_RB1: unknowns of that
// colour get x + (b - A x)/a_pp, the others keep x.  xin == nullptr: x = 0.
template <typename T, int DIM, int KIND>
__device__ __forceinline__ T smooth_node(const StencilParams<T>& op, const T* kappa,
                                         const DGeo& g, int ks, const T* __restrict__ xin,
                                         const T* __restrict__ b, T omega, long p, int i, int j,
                                         int k) {
  const bool upd = (ks == SM_JACOBI) || (((i + j + k) & 1) == (ks == SM_RB1 ? 1 : 0));
  if (xin == nullptr) {
    if (!upd) return T(0);
    const T dg = Apply<T, DIM, KIND>::diag(op, kappa, g, i, j, k);
    return ks == SM_JACOBI ? omega * (b[p] / dg) : b[p] / dg;
  }
  if (!upd) return xin[p];
  T ax, dg;
  Apply<T, DIM, KIND>::at(op, kappa, g, xin, p, i, j, k, ax, dg);
  const T q = (b[p] - ax) / dg;
  return ks == SM_JACOBI ? xin[p] + omega * q : xin[p] + q;
}

// Gauss-Seidel update of unknown p in place (multicolour Gauss-Seidel: the
// other unknowns of its colour are not coupled to it, so they may be
// updated at the same time): x_p + (b_p - (A x)_p) / a_pp.
template <typename T, int DIM, int KIND>
__device__ __forceinline__ T gs_node(const StencilParams<T>& op, const T* kappa, const DGeo& g,
                                     const T* x, const T* __restrict__ b, long p, int i, int j,
                                     int k) {
  T ax, dg;
  Apply<T, DIM, KIND>::at(op, kappa, g, x, p, i, j, k, ax, dg);
  const T q = (b[p] - ax) / dg;
  return x[p] + q;
}

template <typename T, int DIM, int KIND>
__device__ __forceinline__ T residual_node(const StencilParams<T>& op, const T* kappa,
                                           const DGeo& g, const T* __restrict__ x,
                                           const T* __restrict__ b, long p, int i, int j,
                                           int k) {
  T ax, dg;
  Apply<T, DIM, KIND>::at(op, kappa, g, x, p, i, j, k, ax, dg);
  return b[p] - ax;
}

// The 3D restriction as explicit fused multiply-adds (the same roundings
// in every kernel that restricts, whatever the compiler contracts): a row
// of three fine values around an even column, r0 + (rm + rp) / 2, and the
// weighted sum of three rows (then of three planes), m / 2 + c + p / 2.
template <typename T>
__device__ __forceinline__ T restrict_row(T rm, T r0, T rp) {
  return fma(T(0.5), rm + rp, r0);
}
template <typename T>
__device__ __forceinline__ T restrict_sum(T m, T c, T p) {
  return fma(T(0.5), p, fma(T(0.5), m, c));
}

// Coarse node (i, j[, k]) gathers the fine residual around fine node 2I
// with weights prod_d (o_d == 0 ? 1 : 1/2).  Only fine unknowns are read.
template <typename T, int DIM>
__device__ __forceinline__ T restrict_node(const DGeo& gf, const T* __restrict__ r, int i,
                                           int j, int k) {
  const long pf = 2 * i + 2 * j * gf.sy + 2L * k * gf.sz;
  const T h = T(0.5), q = T(0.25);
  if (DIM == 2) {
    const long sy = gf.sy;
    return r[pf] + h * ((r[pf - 1] + r[pf + 1]) + (r[pf - sy] + r[pf + sy])) +
           q * ((r[pf - 1 - sy] + r[pf + 1 - sy]) + (r[pf - 1 + sy] + r[pf + 1 + sy]));
  }
  const long sy = gf.sy, sz = gf.sz;
  T pl[3];
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {
    T row[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const long o = pf + (dy - 1) * sy + (dz - 1) * sz;
      row[dy] = restrict_row(r[o - 1], r[o], r[o + 1]);
    }
    pl[dz] = restrict_sum(row[0], row[1], row[2]);
  }
  return restrict_sum(pl[0], pl[1], pl[2]);
}

// Multilinear interpolant of the coarse correction at fine node (i, j[, k]):
// per direction an even coordinate has the single parent i/2 (weight 1), an
// odd one the parents (i-1)/2 and (i+1)/2 (weight 1/2 each).  Coarse
// boundary entries of e are read and must be 0.
template <typename T, int DIM>
__device__ __forceinline__ T prolong_node(const DGeo& gc, const T* __restrict__ e, int i, int j,
                                          int k) {
  const int i0 = i >> 1, i1 = (i + 1) >> 1;
  const int j0 = j >> 1, j1 = (j + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1);
  const T wj = (j & 1) ? T(0.5) : T(1);
  if (DIM == 2) {
    const long sy = gc.sy;
    T r0 = (i & 1) ? wi * (e[i0 + j0 * sy] + e[i1 + j0 * sy]) : e[i0 + j0 * sy];
    T r1 = (i & 1) ? wi * (e[i0 + j1 * sy] + e[i1 + j1 * sy]) : e[i0 + j1 * sy];
    return (j & 1) ? wj * (r0 + r1) : r0;
  }
  const long sy = gc.sy, sz = gc.sz;
  const int k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wk = (k & 1) ? T(0.5) : T(1);
  auto line = [&](int jj, int kk) -> T {
    const long o = jj * sy + kk * sz;
    return (i & 1) ? wi * (e[o + i0] + e[o + i1]) : e[o + i0];
  };
  auto plane = [&](int kk) -> T {
    return (j & 1) ? wj * (line(j0, kk) + line(j1, kk)) : line(j0, kk);
  };
  return (k & 1) ? wk * (plane(k0) + plane(k1)) : plane(k0);
}

// ---------------------------------------------------------------------------
// 3D sweep kernel for the large levels: a block of 64 x 4 threads owns a tile
// of 128 x 4 unknowns in (x, y) and marches over kz planes in z.  Per plane,
// the block stages the plane's (128+2) x (4+2) tile of x (and the cell layer
// of kappa) in LDS once; every thread copies its 4 x 3 window of the plane
// into registers, so it holds planes k-1, k, k+1 for its two unknowns
// (i, i+1) and reads 6 LDS vectors per plane instead of 2 x 20 global
// loads.  In a red-black half-sweep exactly one of the two unknowns has the
// colour being updated, and the whole wavefront agrees on which one.
//
// MODE: SM_JACOBI, SM_RB0, SM_RB1 (smoothing; ZERO: x = 0, not read),
// SW_RESID (r = b - A x with per-block partial sums of r^2 when NORM) or
// SW_HEAD_RB0 / SW_HEAD_JAC: the partial sums of (b - A x)^2 together with
// the red-black colour-0 (Jacobi) smoothing step of x, written to out.
// ---------------------------------------------------------------------------
constexpr int SW_RESID = 3;
constexpr int SW_HEAD_RB0 = 4;
constexpr int SW_HEAD_JAC = 5;
constexpr int SW_APPLY = 6;  // out = A x with partial sums of x.(A x)
// out = W x + omega F (F in the b slot; W the launch's operator weights);
// with Item::e != nullptr also e = 2 x - e at every unknown (node-local)
constexpr int SW_CN = 7;
constexpr int SW_TX = 128;  // unknowns per tile in x (2 per thread)
constexpr int SW_TY = 4;    // unknowns per tile in y (1 per thread row)
constexpr int SW_LX = SW_TX + 2, SW_LY = SW_TY + 2;

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// sweep3 launch shape: planes per block for a level with m unknowns per
// direction and elements of elem bytes (MG_SWEEP3_KZ overrides).  Long
// z-marches re-read fewer halo planes; short ones give the small levels
// enough workgroups to fill the chip.  Measured on MI355X: FP64 levels take
// 32 planes from 255 up (16 cost 2-3% on the 256^3 and 512^3 solves, 24
// leaves an unbalanced last chunk) and 24 at 191; FP32 levels 32 from 511,
// 16 at 255 and 12 at 191; every kind 4, 2 and 1 at 127, 63 and 31.
// (Builds with MG_TUNING_KNOBS defined read MG_SWEEP3_KZ, MG_SWEEP3_REMAP
// and MG_PROLONG_PZ from the environment to override the launch shapes,
// for sweeps of them; the library as built here does not.)
inline int sweep3_kz(int m, int elem) {
#ifdef MG_TUNING_KNOBS
  static const int forced = [] {
    const char* e = getenv("MG_SWEEP3_KZ");
    return e ? atoi(e) : 0;
  }();
  if (forced > 0) return forced;
#endif
  if (m >= 255) return elem == 8 || m >= 511 ? 32 : 16;
  if (m >= 191) return elem == 8 ? 24 : 12;
  return m >= 127 ? 4 : (m >= 63 ? 2 : 1);
}

// PRO (smoothing modes): the coarse correction e of the next coarser level
// (Item::e) is prolongated and added to x as x is staged, so the launch
// smooths x + P e -- the prolongation step fused into the first
// post-smoothing step, bitwise as k_prolong_add followed by the sweep.
// XL: layout of the iterate on a level with even n whose iterate is kept
// colour-split (the even-index nodes, which are the red ones, at p / 2 of
// one half, the odd ones at p / 2 of another; Item::a / Item::a2 are the
// halves read, Item::c the half written).  0: natural in and out.  1:
// natural in, split out -- the updated colour to Item::c, the other colour
// to Item::c2.  2: split in and out, only the updated colour written (a
// residual reads x split and writes r natural).  3: split in, natural out
// (both colours).  4: split in and out, both halves written (Item::c the
// updated colour's, Item::c2 the other's; with the fused prolongation,
// whose correction changes every node).  The arithmetic per node is the
// same in every layout.
// IRU (FP32 smoothing steps that write a natural iterate): the step is the
// last one of the FP32 correction cycle of iterative refinement, and instead
// of the correction c it writes u + s c (u: the FP64 iterate, Item::c; s =
// ir_scale(*Item::scal)), in the arithmetic of k_ir_update -- the
// refinement update fused into the step that produces c.  The step reads no
// u that other blocks write, so the update can be in place.
// CAST (FP64 residual, x and b natural): r = b - A x is not stored; the
// step writes float(r / s) (s = ir_scale(*Item::scal)) to the FP32 vector
// Item::c in the layout Item::lay, in the arithmetic of k_scale_cast -- the
// residual of iterative refinement written directly as the right-hand side
// of the next FP32 correction cycle.
template <typename T, int KIND, int MODE, bool ZERO, bool NORM, bool PRO = false, int XL = 0,
          bool IRU = false, bool CAST = false>
__global__ __launch_bounds__(256) void k_sweep3(Geo g, StencilParams<T> op, T omega, int kz,
                                                int nzc, int remap, Batch B) {
  using V2 = typename Vec2<T>::type;
  constexpr bool HEAD = MODE == SW_HEAD_RB0 || MODE == SW_HEAD_JAC;
  static_assert(XL == 0 || ((MODE == SM_RB0 || MODE == SM_RB1) && !NORM) ||
                    (MODE == SW_HEAD_RB0 && (XL == 1 || XL == 2)) ||
                    (MODE == SW_RESID && XL == 2),
                "split iterates are for red-black half-sweeps, heads and residuals");
  static_assert(!PRO || XL <= 1 || XL == 4, "the prolongation writes both colours");
  static_assert(XL != 4 || PRO, "both halves of a split iterate change only with a prolongation");
  static_assert(!(ZERO && (XL == 2 || XL == 3 || XL == 4)), "x = 0 is read in no layout");
  constexpr bool XIN = XL == 2 || XL == 3 || XL == 4;         // x read colour-split
  constexpr bool XOUT = XL == 1 || XL == 2 || XL == 4;        // updated unknowns written split
  constexpr bool XBOTH = XL == 1 || XL == 4;                  // the other colour to Item::c2
  static_assert(!IRU || (sizeof(T) == 4 && !ZERO && !PRO && (XL == 0 || XL == 3) &&
                         (MODE == SM_RB0 || MODE == SM_RB1 || MODE == SM_JACOBI)),
                "the refinement update follows a natural-output FP32 smoothing step");
  static_assert(!CAST || (sizeof(T) == 8 && MODE == SW_RESID && !ZERO && !PRO && XL == 0),
                "the scaled cast is written by an FP64 residual");
  __shared__ __align__(16) T sx[2][SW_LY][SW_LX];
  __shared__ T sk[2][SW_TY + 1][SW_TX + 1];
  const int n = g.n, m = n - 1;
  const long sy = g.sy, sz = g.sz;
  // tile (bx, by, bz): with `remap`, tiles that are neighbours in y and z
  // run on one XCD, so the halo rows they share are read once into its L2
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if (remap) {
    const int gxy = gridDim.x * gridDim.y;
    const int nb = gxy * gridDim.z;
    const int L = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
    bx = L % gridDim.x;
    by = (L / gridDim.x) % gridDim.y;
    bz = L / gxy;
  }
  const int item = bz / nzc, zc = bz % nzc;
  const Item& I = B.it[item];
  const T* __restrict__ x = (const T*)I.a;  // natural x, or its even half (XIN)
  const T* __restrict__ xodd = XIN ? (const T*)I.a2 : nullptr;
  const T* __restrict__ b = (const T*)I.b;
  T* __restrict__ out = (T*)I.c;  // natural, or the updated colour's half (XOUT)
  T* __restrict__ out2 = XBOTH ? (T*)I.c2 : nullptr;
  const T* __restrict__ kap = (const T*)I.kappa;
  const int i0 = 1 + bx * SW_TX, j0 = 1 + by * SW_TY, k0 = 1 + zc * kz;
  const int k1 = min(k0 + kz - 1, m);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int i = i0 + 2 * tx, j = j0 + ty;
  const bool row_ok = j <= m;
  const bool ok0 = row_ok && i <= m, ok1 = row_ok && i + 1 <= m;

  // A plane of x (columns i0-1 .. i0+128, rows j0-1 .. j0+4) is staged by
  // the block's threads, element e = tid + 256 q; a cell layer (cells
  // i0-1 .. i0+127, j0-1 .. j0+3) likewise.  Loads go to registers first
  // (prefetch) and are written to LDS one plane later (commit), so they are
  // in flight while the previous plane is computed.
  constexpr int NX = (SW_LX * SW_LY + 255) / 256;
  constexpr int NK = ((SW_TX + 1) * (SW_TY + 1) + 255) / 256;
  int xoff[NX];  // node offsets within a plane (grids have < 2^31 nodes)
  T xpf[NX];
  // A split iterate (XIN) is staged with the columns of each row sorted by
  // parity -- element c of a row takes column 2c (c < SW_LX / 2) or column
  // 2 (c - SW_LX / 2) + 1 -- so that neighbouring lanes read neighbouring
  // entries of one half.
  auto xcol = [&](int cc) {
    return XIN ? (cc < SW_LX / 2 ? 2 * cc : 2 * (cc - SW_LX / 2) + 1) : cc;
  };
#pragma unroll
  for (int q = 0; q < NX; ++q) {
    const int e = tid + 256 * q;
    const int r = e / SW_LX, c = xcol(e - r * SW_LX);
    const int gi = i0 - 1 + c, gj = j0 - 1 + r;
    xoff[q] = min(gi, n) + min(gj, n) * (int)sy;  // always inside the grid
  }
  // Loads sit behind no branch or select, so the compiler keeps a plane's
  // loads in flight across the computation of the previous plane instead of
  // waiting at each one: a staged position off the grid (x or y beyond n,
  // z beyond n, or past the tile) reads some node of the grid instead, and
  // only the stencils of unknowns beyond m, which are never written, see
  // such a value.  The same holds for b and the cell coefficients below.
  auto prefetch_x = [&](int z) {
    if constexpr (XIN) {
      const long zb = (long)min(z, n) * sz;
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        const long p = zb + xoff[q];
        xpf[q] = ((p & 1) ? xodd : x)[p >> 1];
      }
    } else {
      const T* __restrict__ xz = x + (long)min(z, n) * sz;
#pragma unroll
      for (int q = 0; q < NX; ++q) xpf[q] = xz[xoff[q]];
    }
  };
  // Coarse planes of e (PRO) for the tile and its halo: coarse columns
  // 64 bx .. 64 bx + 65, rows 2 by .. 2 by + 3, plane K in slot K % 3,
  // staged from registers one step after their loads.
  constexpr int CX = SW_TX / 2 + 2, CY = SW_TY / 2 + 2;
  constexpr int NCS = (CX * CY + 255) / 256;
  __shared__ T sc[PRO ? 3 : 1][CY][CX];
  const int nco = n >> 1;
  const long syc = nco + 1, szc = syc * syc;
  const T* __restrict__ ec = PRO ? (const T*)I.e : nullptr;
  int coff[NCS];
  T cpf[NCS];
  if (PRO) {
#pragma unroll
    for (int q = 0; q < NCS; ++q) {
      const int e = tid + 256 * q;
      const int r = e / CX, c = e - r * CX;
      coff[q] = min(64 * bx + c, nco) + min(2 * by + r, nco) * (int)syc;
    }
  }
  auto prefetch_c = [&](int K) {
    const T* __restrict__ ez = ec + (long)min(K, nco) * szc;
#pragma unroll
    for (int q = 0; q < NCS; ++q) cpf[q] = ez[coff[q]];
  };
  auto commit_c = [&](int K) {
    T* dst = &sc[PRO ? K % 3 : 0][0][0];
#pragma unroll
    for (int q = 0; q < NCS; ++q) {
      const int e = tid + 256 * q;
      if (e < CX * CY) dst[e] = cpf[q];
    }
  };
  // the multilinear interpolant of e at staged fine node (gi, gj, z), in the
  // arithmetic of prolong_node
  // The multilinear interpolant of e at the staged fine node of element q
  // in plane z, in the arithmetic of prolong_node: the in-plane (x, y)
  // interpolant of the coarse planes z/2 (even z), or (z-1)/2 and (z+1)/2
  // (odd z, weight 1/2).  FP32 (IPREG): a coarse plane K serves the fine
  // planes 2K-1, 2K and 2K+1, so each thread forms its in-plane interpolant
  // once, when the plane first enters (ip_plane), and keeps it and the one
  // before in registers (ipo, ipn), which takes the LDS reads and index
  // arithmetic of the staging from about 3.4 to about 1.1 per element and
  // plane.  FP64 recomputes it from LDS per plane: the registers of the
  // cache would cost a quarter of the FP64 kernel's occupancy.
  constexpr bool IPREG = PRO && sizeof(T) == 4;
  // FP64 (IPLDS): the same cache, in thread-private LDS slots instead of
  // registers (slot (K & 1) holds coarse plane K's interpolants)
  constexpr bool IPLDS = PRO && sizeof(T) == 8;
  __shared__ T ipl[IPLDS ? 2 : 1][IPLDS ? NX : 1][IPLDS ? 256 : 1];
  auto ip_elem = [&](int q, int ss) -> T {
    const int e = tid + 256 * q;
    const int r = e / SW_LX, c = xcol(e - r * SW_LX);
    const int gi = i0 - 1 + c, gj = j0 - 1 + r;
    const int a0 = (gi >> 1) - 64 * bx, a1 = ((gi + 1) >> 1) - 64 * bx;
    const int r0 = (gj >> 1) - 2 * by, r1 = ((gj + 1) >> 1) - 2 * by;
    const T wi = (gi & 1) ? T(0.5) : T(1), wj = (gj & 1) ? T(0.5) : T(1);
    auto line = [&](int rr) -> T {
      return (gi & 1) ? wi * (sc[ss][rr][a0] + sc[ss][rr][a1]) : sc[ss][rr][a0];
    };
    return (gj & 1) ? wj * (line(r0) + line(r1)) : line(r0);
  };
  T ipo[IPREG ? NX : 1], ipn[IPREG ? NX : 1];
  auto ip_plane = [&](int K) {
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      if constexpr (IPLDS)
        ipl[K & 1][q][tid] = ip_elem(q, K % 3);
      else
        ipn[q] = ip_elem(q, K % 3);
    }
  };
  auto pe = [&](int q, int z) -> T {
    if constexpr (IPREG) {
      return (z & 1) ? T(0.5) * (ipo[q] + ipn[q]) : ipn[q];
    } else if constexpr (IPLDS) {
      const int K = (z + 1) >> 1;  // the newer plane (z / 2 for even z)
      return (z & 1) ? T(0.5) * (ipl[(K - 1) & 1][q][tid] + ipl[K & 1][q][tid])
                     : ipl[K & 1][q][tid];
    } else {
      const int s0 = (z >> 1) % 3, s1 = ((z + 1) >> 1) % 3;
      return (z & 1) ? T(0.5) * (ip_elem(q, s0) + ip_elem(q, s1)) : ip_elem(q, s0);
    }
  };
  auto commit_x = [&](int s, int z) {
    T* dst = &sx[s][0][0];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = tid + 256 * q;
      if (e < SW_LX * SW_LY) {
        if (PRO) {
          const int r = e / SW_LX, c = xcol(e - r * SW_LX);
          dst[r * SW_LX + c] = xpf[q] + pe(q, z);
        } else if (XIN) {
          const int r = e / SW_LX;
          dst[r * SW_LX + xcol(e - r * SW_LX)] = xpf[q];
        } else {
          dst[e] = xpf[q];
        }
      }
    }
  };
  int koff[NK];
  T kpf[NK];
  if (KIND == OP_KAPPA) {
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      const int e = tid + 256 * q;
      const int r = e / (SW_TX + 1), c = e - r * (SW_TX + 1);
      const int cx = i0 - 1 + c, cy = j0 - 1 + r;
      koff[q] = min(cx, n - 1) + n * min(cy, n - 1);
    }
  }
  auto prefetch_k = [&](int cz) {
    const T* __restrict__ kz_ = kap + (long)n * n * min(cz, n - 1);
#pragma unroll
    for (int q = 0; q < NK; ++q) kpf[q] = kz_[koff[q]];
  };
  auto commit_k = [&](int s) {
    T* dst = &sk[s][0][0];
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      const int e = tid + 256 * q;
      if (e < (SW_TX + 1) * (SW_TY + 1)) dst[e] = kpf[q];
    }
  };
  // this thread's window of plane slot s: rows j-1..j+1, columns i-1..i+2
  auto window_x = [&](int s, T (&w)[3][4]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const V2* row = reinterpret_cast<const V2*>(&sx[s][ty + r][0]);
      const V2 a = row[tx], c = row[tx + 1];
      w[r][0] = a.x;
      w[r][1] = a.y;
      w[r][2] = c.x;
      w[r][3] = c.y;
    }
  };
  auto window_k = [&](int s, T (&w)[2][3]) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) w[r][c] = sk[s][ty + r][2 * tx + c];
  };

  // Planes are processed in order p = k0-1 .. k1+1; plane p and cell layer
  // p go to LDS slot p & 1.  At plane p each thread reads its window once
  // and reduces it to the sums the stencils need (the operator is a sum of
  // per-plane parts, see stencil3_const_sum / the kappa parts): the parts of
  // plane p for the unknowns of planes p-1 and p+1 (x/y edges and corners,
  // or the kappa Q/R sums) and for the unknown of plane p itself (in-plane
  // corners and centre, or P and the coefficient sum).  The unknowns of
  // plane p-1 are then complete and are written.  Only these sums are
  // carried between planes, not the windows, which keeps the register
  // count low.  In a red-black half-sweep a thread updates one of its two
  // unknowns per plane, alternately i and i+1, so one set of sums suffices.
  constexpr bool RB = MODE == SM_RB0 || MODE == SM_RB1;
  constexpr bool KAP = KIND == OP_KAPPA;
  constexpr bool MASS = KIND == OP_MASS;
  constexpr int NS = MASS ? 4 : 3;  // side parts carried per plane
  constexpr int NC = RB ? 1 : 2;    // unknowns computed per thread and plane
  const int colour = MODE == SM_RB1 ? 1 : 0;
  const long pb0 = min(i, n - 1) + min(j, n) * sy;  // clamped into the grid
  T bpf[2] = {T(0), T(0)};
  T* const ge = MODE == SW_CN ? (T*)const_cast<void*>(I.e) : nullptr;
  T gpf[2] = {T(0), T(0)};
  const long blay = CAST ? 0 : I.lay;  // b colour-split (see Item::lay) or natural
  // Red-black on a colour-split b: every unknown a half-sweep updates has
  // parity `colour`, so its b is element p / 2 of that colour's half.  A
  // lane clamped onto node (n, n, n) (parity 0) in a colour-1 sweep reads
  // the one padding element past the odd half; its value is not used.
  const int bsh = blay ? 1 : 0;
  const T* const bq = b + (blay && colour ? blay : 0);
  auto prefetch_b = [&](int k) {
    const long p = pb0 + (long)min(k, n) * sz;
#pragma unroll
    for (int u = 0; u < 2; ++u) bpf[u] = b[lay_idx(p + u, blay)];
    if (MODE == SW_CN && ge != nullptr) {
#pragma unroll
      for (int u = 0; u < 2; ++u) gpf[u] = ge[p + u];
    }
  };
  double* const uo = IRU ? (double*)I.c : nullptr;
  const double sr = IRU || CAST ? ir_scale(*I.scal) : 0.0;
  float* const co = CAST ? (float*)I.c : nullptr;
  auto put = [&](long p, T v) {
    if constexpr (IRU)
      uo[p] = uo[p] + sr * (double)v;
    else if constexpr (CAST)
      co[lay_idx(p, I.lay)] = (float)((double)v / sr);
    else
      out[p] = v;
  };
  auto store = [&](int k, int u, T v) { put(i + u + j * sy + (long)k * sz, v); };
  // red-black: an updated unknown, and one of the other colour (its old
  // value, or 0 from x = 0), in the layout XL writes
  auto store_upd = [&](int k, int u, T v) {
    const long p = i + u + j * sy + (long)k * sz;
    if (XOUT)
      out[p >> 1] = v;
    else
      put(p, v);
  };
  auto store_oth = [&](int k, int u, T v) {
    const long p = i + u + j * sy + (long)k * sz;
    if (XBOTH)
      out2[p >> 1] = v;
    else if (!XOUT)
      put(p, v);
  };
  double sq = 0.0;
  T kwp[2][3];  // cell window of layer p-1
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) kwp[r][c] = T(0);

  if (ZERO) {
    // x = 0: an updated unknown gets (omega) b / a_pp, the others 0
    if (KAP) {
      prefetch_k(k0 - 1);
      commit_k((k0 - 1) & 1);
      prefetch_k(k0);
      __syncthreads();
      window_k((k0 - 1) & 1, kwp);
    }
    // b of the unknowns set at plane k -- for red-black only the updated
    // one's (u = (colour + i + j + k) & 1) -- loaded one plane ahead; no
    // barrier without cell layers (nothing else goes through LDS)
    T bnx[2] = {T(0), T(0)};
    auto load_b = [&](int k) {
      const long p = pb0 + (long)min(k, n) * sz;
      if (MODE == SM_JACOBI) {
#pragma unroll
        for (int u = 0; u < 2; ++u) bnx[u] = b[lay_idx(p + u, blay)];
      } else {
        bnx[0] = b[lay_idx(p + ((colour + i + j + k) & 1), blay)];
      }
    };
    load_b(k0);
    for (int k = k0; k <= k1; ++k) {
      const T bc0 = bnx[0], bc1 = bnx[1];
      load_b(k + 1);
      T kwc[2][3];
      if (KAP) {
        commit_k(k & 1);
        prefetch_k(k + 1);
        __syncthreads();
        window_k(k & 1, kwc);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool ok = u == 0 ? ok0 : ok1;
        const bool upd = MODE == SM_JACOBI || (((i + u + j + k) & 1) == colour);
        if (!ok) continue;
        const T bv = MODE == SM_JACOBI && u == 1 ? bc1 : bc0;
        T dg = op.wc;
        if (KAP) dg = op.s * T(4) * kappa_cell_sum<T>(kwp, kwc, u);
        if (MODE == SM_JACOBI)
          store(k, u, omega * (bv / dg));
        else if (upd)
          store_upd(k, u, bv / dg);
        else
          store_oth(k, u, T(0));
      }
      if (KAP) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) kwp[r][c] = kwc[r][c];
      }
    }
    return;
  }

  // sums carried per computed unknown q (see above):
  //   s2 / s1: side parts of planes p-2 / p-1 for the unknowns two / one
  //            plane(s) up: {x-edges, y-edges, corners} (kappa: {Q, -, -};
  //            with the mass term also the centre value, a face neighbour)
  //   g1, x1, k1s, f1: plane-(p-1) parts of its own unknown: in-plane
  //            corners (kappa: P), centre value, coefficient sum (kappa),
  //            in-plane faces (mass term)
  T s2[NC][NS], s1[NC][NS], g1[NC], x1[NC], k1s[NC], f1[NC];
  T xo1 = T(0);  // red-black: old value of the other unknown at plane p-1
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    g1[q] = x1[q] = k1s[q] = f1[q] = T(0);
#pragma unroll
    for (int t = 0; t < NS; ++t) s2[q][t] = s1[q][t] = T(0);
  }
  prefetch_x(k0 - 1);
  if (KAP) prefetch_k(k0 - 1);
  // PRO: coarse planes c0 .. c0+2 cover the fine planes committed before
  // the first odd step stages the next one; an odd step q stages coarse
  // plane (q+3)/2 (needed from fine plane q+2 on) into the slot of plane
  // (q-3)/2, whose last fine plane q-2 was committed two steps before
  const int c0 = (k0 - 1) >> 1;
  if (PRO) {
#pragma unroll
    for (int K = c0; K <= c0 + 2; ++K) {
      prefetch_c(K);
      commit_c(K);
    }
    prefetch_c(c0 + 3);
    __syncthreads();
    if (IPREG || IPLDS) ip_plane((k0 - 1) >> 1);
  }
  for (int p = k0 - 1; p <= k1 + 1; ++p) {
    if (PRO && (p & 1) && ((p + 3) >> 1) > c0 + 2) {
      commit_c((p + 3) >> 1);
      prefetch_c(((p + 3) >> 1) + 1);
    }
    if (IPLDS && (p & 1)) ip_plane((p + 1) >> 1);  // (the slot of (p-3)/2)
    if (IPREG && (p & 1)) {
      // fine plane p (odd) interpolates from coarse planes (p-1)/2, kept,
      // and (p+1)/2, new (staged at least one step earlier)
#pragma unroll
      for (int q = 0; q < NX; ++q) ipo[q] = ipn[q];
      ip_plane((p + 1) >> 1);
    }
    commit_x(p & 1, p);
    prefetch_x(p + 1);
    if (KAP) {
      commit_k(p & 1);
      prefetch_k(p + 1);
    }
    const T bcur[2] = {bpf[0], bpf[1]};  // b of plane p-1 (red-black: [0], its updated unknown)
    const T gcur[2] = {gpf[0], gpf[1]};  // SW_CN: the guess at plane p-1
    if (!RB && MODE != SW_APPLY) prefetch_b(p);
    __syncthreads();
    T w[3][4];
    window_x(p & 1, w);
    T kwc[2][3];
    if (KAP) window_k(p & 1, kwc);
    // red-black: column updated at plane p (the unknowns at p-1, p+1 use
    // the other one); the same for a whole wavefront (one row j), so the
    // branch below does not diverge, and inside it every window index is a
    // constant (runtime indices into register arrays become select chains)
    T sn[NC][NS], gn[NC], xn[NC], kn[NC], fn[NC], xon;
    const int k = p - 1;
    auto step = [&](auto upc) {
      constexpr int up = decltype(upc)::value;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int cs = RB ? 1 - up : q;  // column of the unknowns at p-1 and p+1
        const int cc = RB ? up : q;      // column of the unknown at p
        if (KAP) {
          sn[q][0] = kappa_side<T>(kwc, w, cs);  // Q of the unknown at p+1 (layer p)
          sn[q][1] = kappa_side<T>(kwp, w, cs);  // R of the unknown at p-1 (layer p-1)
          sn[q][2] = T(0);
          kappa_plane<T>(kwp, kwc, w, cc, gn[q], kn[q]);
          fn[q] = T(0);
        } else {
          plane_parts<T>(w, cs, sn[q][0], sn[q][1], sn[q][2]);
          if constexpr (MASS) sn[q][3] = w[1][cs + 1];
          T ea, eb;
          plane_parts<T>(w, cc, ea, eb, gn[q]);
          fn[q] = MASS ? ea + eb : T(0);
          kn[q] = T(0);
        }
        xn[q] = w[1][cc + 1];
      }
      xon = w[1][(1 - up) + 1];
      if (k < k0) return;
      // complete the unknowns of plane k
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int u = RB ? 1 - up : q;
        const bool ok = u == 0 ? ok0 : ok1;
        if (!ok) continue;
        T ax, dg;
        if (KAP) {
          ax = op.s * (g1[q] - (s2[q][0] + sn[q][1]));
          dg = op.s * T(4) * k1s[q];
        } else if constexpr (MASS) {
          ax = stencil3_mass_sum(op, x1[q], g1[q], f1[q], s2[q][0], sn[q][0], s2[q][1],
                                 sn[q][1], s2[q][2], sn[q][2], s2[q][3], sn[q][3]);
          dg = op.wc;
        } else {
          ax = stencil3_const_sum(op, x1[q], g1[q], s2[q][0], sn[q][0], s2[q][1], sn[q][1],
                                  s2[q][2], sn[q][2]);
          dg = op.wc;
        }
        const T res = (RB ? bcur[0] : bcur[u]) - ax;
        if (MODE == SW_CN) {
          store(k, u, ax + omega * bcur[u]);
          if (ge != nullptr) ge[i + u + j * sy + (long)k * sz] = T(2) * x1[q] - gcur[u];
        } else if (MODE == SW_APPLY) {
          store(k, u, ax);
          sq += (double)x1[q] * (double)ax;
        } else if (MODE == SW_RESID) {
          store(k, u, res);
          sq += (double)res * (double)res;
        } else if (HEAD) {
          sq += (double)res * (double)res;
          const T d = res / dg;
          const bool c0 = ((i + u + j + k) & 1) == 0;
          if (MODE == SW_HEAD_JAC)
            store(k, u, x1[q] + omega * d);
          else if (c0)
            store_upd(k, u, x1[q] + d);
          else
            store_oth(k, u, x1[q]);
        } else {
          const T d = res / dg;
          if (RB)
            store_upd(k, u, x1[q] + d);
          else
            store(k, u, x1[q] + omega * d);
        }
      }
      if (RB && (up == 0 ? ok0 : ok1)) store_oth(k, up, xo1);  // the other unknown keeps its value
    };
    // red-black: b of the unknown updated at plane p, for the next plane
    auto prefetch_b1 = [&](int up) {
      bpf[0] = bq[(pb0 + (long)min(p, n) * sz + up) >> bsh];
    };
    if (!RB || ((colour + 1 + j + p) & 1) == 0) {  // i is odd
      if (RB) prefetch_b1(0);
      step(std::integral_constant<int, 0>{});
    } else {
      prefetch_b1(1);
      step(std::integral_constant<int, 1>{});
    }
    // shift
#pragma unroll
    for (int q = 0; q < NC; ++q) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        s2[q][t] = s1[q][t];
        s1[q][t] = sn[q][t];
      }
      g1[q] = gn[q];
      x1[q] = xn[q];
      k1s[q] = kn[q];
      f1[q] = fn[q];
    }
    xo1 = xon;
    if (KAP) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) kwp[r][c] = kwc[r][c];
    }
  }
  if ((MODE == SW_RESID && NORM) || HEAD || MODE == SW_APPLY) {
    const double t = block_sum(sq);
    if (tid == 0)
      I.partials[bx + (long)gridDim.x * (by + (long)gridDim.y * zc)] = t;
  }
}

// ---------------------------------------------------------------------------
// Residual and restriction in one pass on the 3D levels k_sweep3 runs (the
// constant-coefficient and mass-shifted kinds): the coarse right-hand side
// b_c = R (b - A x), R = P^T, without storing r.  A block computes r on the
// k_sweep3 tile (128 x 4 unknowns, two per thread and plane, with the same
// plane parts and sums, so r is bitwise that of the k_sweep3 residual) and
// on one more row, the next tile's first, with a fifth wave: coarse row J
// reads fine rows 2J-1 .. 2J+1, and the rows j0 .. j0+4 (j0 odd) hold those
// of the tile's coarse rows (j0+1)/2 and (j0+3)/2.  In x a lane forms the
// row sum of coarse column (i+1)/2 from its two unknowns and its right
// neighbour's first (a lane shift); the last lane's coarse column needs the
// next tile's first column, so the three fine columns of that coarse column
// are written to Item::e, packed as edge_idx gives, and k_restrict_xcols
// restricts it afterwards.  In z a block marches the fine planes
// 2K0-1 .. 2K1+1 of its coarse planes K0 .. K1 (plane 2K1+1 is also the next
// chunk's first): plane 2K-1 opens coarse plane K, 2K adds to it and 2K+1
// completes it, with the sums of restrict_node in its order, so b_c is
// bitwise that of the separate residual and restriction launches.
//   Item: a = x (XIN: its even half, a2 the odd half), b = b (layout lay),
//   c = b_c (colour-split when flag), e = the fine residual vector.
// ---------------------------------------------------------------------------
// Packed fine columns 2I-1, 2I, 2I+1 (c = 0, 1, 2) of the coarse column
// I = 64 (col + 1) at fine row j, plane k: consecutive rows are adjacent.
__device__ __forceinline__ long edge_idx(int n, int col, int k, int j, int c) {
  return (((long)col * (n + 1) + k) * (n + 1) + j) * 3 + c;
}

constexpr int RR_TY = SW_TY + 1;  // fine rows computed per tile
constexpr int RR_LY = RR_TY + 2;  // staged rows of x
constexpr int RR_THREADS = 64 * RR_TY;

template <typename T, int KIND, bool XIN>
__global__ __launch_bounds__(RR_THREADS) void k_resid_restrict3(Geo g, StencilParams<T> op,
                                                                int kzc, int nzc, int remap,
                                                                Batch B) {
  static_assert(KIND != OP_KAPPA, "the per-cell operator has its own parts");
  constexpr bool MASS = KIND == OP_MASS;
  constexpr int NS = MASS ? 4 : 3;
  __shared__ __align__(16) T sx[2][RR_LY][SW_LX];
  __shared__ T srow[RR_TY][64];
  const int n = g.n, m = n - 1, nco = n >> 1, mc = nco - 1;
  const long sy = g.sy, sz = g.sz;
  const long syc = nco + 1, szc = syc * syc;
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if (remap) {
    const int gxy = gridDim.x * gridDim.y;
    const int nb = gxy * gridDim.z;
    const int L = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
    bx = L % gridDim.x;
    by = (L / gridDim.x) % gridDim.y;
    bz = L / gxy;
  }
  const int item = bz / nzc, zc = bz % nzc;
  const Item& I = B.it[item];
  const T* __restrict__ x = (const T*)I.a;
  const T* __restrict__ xodd = XIN ? (const T*)I.a2 : nullptr;
  const T* __restrict__ b = (const T*)I.b;
  T* __restrict__ bc = (T*)I.c;
  T* __restrict__ rv = (T*)const_cast<void*>(I.e);
  const long blay = I.lay;
  const long clay = I.flag ? (syc * szc + 1) / 2 : 0;
  const int i0 = 1 + bx * SW_TX, j0 = 1 + by * SW_TY;
  const int K0 = 1 + zc * kzc, K1 = min(K0 + kzc - 1, mc);
  const int k0 = 2 * K0 - 1, k1 = 2 * K1 + 1;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int i = i0 + 2 * tx, j = j0 + ty;
  const bool row_ok = j <= m;
  const bool ok0 = row_ok && i <= m, ok1 = row_ok && i + 1 <= m;

  // x planes staged as in k_sweep3 (columns i0-1 .. i0+128, rows
  // j0-1 .. j0+5), element e = tid + RR_THREADS q
  constexpr int NX = (SW_LX * RR_LY + RR_THREADS - 1) / RR_THREADS;
  int xoff[NX];
  // FP64: x planes two ahead (planes p+1 and p+2 in flight, slot = plane &
  // 1; 2% faster 256^3 FP64 solves with two blocks per CU); FP32 one ahead
  // (two ahead was 1% slower there)
  constexpr bool PF2 = sizeof(T) == 8;
  T xpf[PF2 ? 2 : 1][NX];
  auto xcol = [&](int cc) {
    return XIN ? (cc < SW_LX / 2 ? 2 * cc : 2 * (cc - SW_LX / 2) + 1) : cc;
  };
#pragma unroll
  for (int q = 0; q < NX; ++q) {
    const int e = tid + RR_THREADS * q;
    const int r = e / SW_LX, c = xcol(e - r * SW_LX);
    const int gi = i0 - 1 + c, gj = j0 - 1 + r;
    xoff[q] = min(gi, n) + min(gj, n) * (int)sy;  // always inside the grid
  }
  auto prefetch_x = [&](int z, T (&buf)[NX]) {
    if constexpr (XIN) {
      const long zb = (long)min(z, n) * sz;
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        const long p = zb + xoff[q];
        buf[q] = ((p & 1) ? xodd : x)[p >> 1];
      }
    } else {
      const T* __restrict__ xz = x + (long)min(z, n) * sz;
#pragma unroll
      for (int q = 0; q < NX; ++q) buf[q] = xz[xoff[q]];
    }
  };
  auto commit_x = [&](int s, const T (&buf)[NX]) {
    T* dst = &sx[s][0][0];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = tid + RR_THREADS * q;
      if (e < SW_LX * RR_LY) {
        const int r = e / SW_LX;
        dst[r * SW_LX + xcol(e - r * SW_LX)] = buf[q];
      }
    }
  };
  auto window_x = [&](int s, T (&w)[3][4]) {
    using V2 = typename Vec2<T>::type;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const V2* row = reinterpret_cast<const V2*>(&sx[s][ty + r][0]);
      const V2 a = row[tx], c = row[tx + 1];
      w[r][0] = a.x;
      w[r][1] = a.y;
      w[r][2] = c.x;
      w[r][3] = c.y;
    }
  };
  const long pb0 = min(i, n - 1) + min(j, n) * sy;  // clamped into the grid
  T bpf[2] = {T(0), T(0)};
  auto prefetch_b = [&](int k) {
    const long p = pb0 + (long)min(k, n) * sz;
#pragma unroll
    for (int u = 0; u < 2; ++u) bpf[u] = b[lay_idx(p + u, blay)];
  };

  // carried plane parts, as in k_sweep3's residual
  T s2[2][NS], s1[2][NS], g1[2], x1[2], f1[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    g1[q] = x1[q] = f1[q] = T(0);
#pragma unroll
    for (int t = 0; t < NS; ++t) s2[q][t] = s1[q][t] = T(0);
  }
  // waves 0 and 1 each own one coarse node per lane: column 64 bx + 1 + tx
  // (not the last lane's), row 2 by + 1 + ty
  const int ic = 64 * bx + 1 + tx, jc = 2 * by + 1 + ty;
  const bool own = ty < 2 && tx < 63 && ic <= mc && jc <= mc;
  const bool edge_l = tx == 63 && 64 * bx + 64 <= mc;  // columns of a boundary coarse column
  const bool edge_f = tx == 0 && bx > 0;
  T plm = T(0), part = T(0);  // plane 2K-1's row sum; m / 2 + c of coarse plane K
  // k0 - 1 is even, so plane p's LDS slot (and with PF2 its register
  // buffer) is p & 1; the loop body is instantiated per slot, so register
  // indices stay constant
  prefetch_x(k0 - 1, xpf[0]);
  if constexpr (PF2) prefetch_x(k0, xpf[PF2 ? 1 : 0]);
  auto body = [&](int p, auto slot) {
    constexpr int SL = decltype(slot)::value;
    constexpr int B = PF2 ? SL : 0;
    commit_x(SL, xpf[B]);
    prefetch_x(PF2 ? p + 2 : p + 1, xpf[B]);
    const T bcur[2] = {bpf[0], bpf[1]};  // b of plane p-1
    prefetch_b(p);
    __syncthreads();
    T w[3][4];
    window_x(p & 1, w);
    T sn[2][NS], gn[2], xn[2], fn[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      plane_parts<T>(w, q, sn[q][0], sn[q][1], sn[q][2]);
      if constexpr (MASS) sn[q][3] = w[1][q + 1];
      T ea, eb;
      plane_parts<T>(w, q, ea, eb, gn[q]);
      fn[q] = MASS ? ea + eb : T(0);
      xn[q] = w[1][q + 1];
    }
    const int k = p - 1;
    if (k >= k0) {
      T res[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        T ax;
        if constexpr (MASS)
          ax = stencil3_mass_sum(op, x1[q], g1[q], f1[q], s2[q][0], sn[q][0], s2[q][1],
                                 sn[q][1], s2[q][2], sn[q][2], s2[q][3], sn[q][3]);
        else
          ax = stencil3_const_sum(op, x1[q], g1[q], s2[q][0], sn[q][0], s2[q][1], sn[q][1],
                                  s2[q][2], sn[q][2]);
        res[q] = (q == 0 ? ok0 : ok1) ? bcur[q] - ax : T(0);
      }
      if (ty < SW_TY && row_ok) {
        if (edge_l) {
          rv[edge_idx(n, bx, k, j, 0)] = res[0];
          rv[edge_idx(n, bx, k, j, 1)] = res[1];
        }
        if (edge_f) rv[edge_idx(n, bx - 1, k, j, 2)] = res[0];
      }
      const T rn = __shfl_down(res[0], 1);  // the right neighbour's first column
      srow[ty][tx] = restrict_row(res[0], res[1], rn);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        s2[q][t] = s1[q][t];
        s1[q][t] = sn[q][t];
      }
      g1[q] = gn[q];
      x1[q] = xn[q];
      f1[q] = fn[q];
    }
    if (k >= k0) {
      __syncthreads();
      if (ty < 2) {
        const T pl = restrict_sum(srow[2 * ty][tx], srow[2 * ty + 1][tx], srow[2 * ty + 2][tx]);
        if (k & 1) {
          // plane 2K+1 completes coarse plane K = (k-1)/2 and opens K+1
          if (k > k0 && own) bc[lay_idx(ic + jc * syc + (long)(k >> 1) * szc, clay)] =
              fma(T(0.5), pl, part);
          plm = pl;
        } else {
          part = fma(T(0.5), plm, pl);
        }
      }
    }
  };
  for (int p = k0 - 1; p <= k1 + 1; p += 2) {
    body(p, std::integral_constant<int, 0>{});
    if (p + 1 <= k1 + 1) body(p + 1, std::integral_constant<int, 1>{});
  }
}

// The coarse columns 64, 128, ... (<= n/2 - 1) that k_resid_restrict3 leaves
// to the end, from the fine columns it packed (edge_idx), in the
// arithmetic of restrict_node.
//   Item: a = the packed fine columns, c = b_c (layout lay).
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_xcols(Geo gf, int ncols, Batch B) {
  const Item& I = B.it[blockIdx.y];
  const int n = gf.n, mc = (n >> 1) - 1;
  const long q = blockIdx.x * 256L + threadIdx.x;
  const long per = (long)mc * mc;
  if (q >= per * ncols) return;
  const int col = (int)(q / per);
  const int jj = (int)(q % mc) + 1, kk = (int)((q / mc) % mc) + 1;
  const T* __restrict__ v = (const T*)I.a;
  T pl[3];
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {
    T row[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const long e = edge_idx(n, col, 2 * kk + dz - 1, 2 * jj + dy - 1, 0);
      row[dy] = restrict_row(v[e], v[e + 1], v[e + 2]);
    }
    pl[dz] = restrict_sum(row[0], row[1], row[2]);
  }
  const long syc = (n >> 1) + 1;  // coarse nodes per direction
  ((T*)I.c)[lay_idx(64 * (col + 1) + jj * syc + (long)kk * syc * syc, I.lay)] =
      restrict_sum(pl[0], pl[1], pl[2]);
}

// ---------------------------------------------------------------------------
// Two red-black half-sweeps in one pass on the 3D levels k_sweep3 runs:
// colour CA, then colour 1-CA, bitwise what two k_sweep3 half-sweeps give.
// A block owns the same 128 x 4 tile as k_sweep3 and marches its planes in
// z.  At step s it stages plane s of x with a halo of 2 in x and y (LDS
// slot s % 3), updates colour CA on plane s-1 over the tile and a ring of
// width 1 around it (the ring is recomputed by the neighbouring blocks as
// well) into the x' planes (slot (s-1) % 3, colour 1-CA copied), and then
// updates colour 1-CA on plane s-2 of the tile from three x' planes and
// writes both colours of that plane.  x, b and the result cross HBM once
// for the two half-sweeps instead of twice.  Cell layers of kappa are
// staged with the same halo (4 slots).  ZERO: x = 0 (not read).
// ---------------------------------------------------------------------------
constexpr int P2_XX = SW_TX + 4, P2_XY = SW_TY + 4;  // staged x plane, halo 2
constexpr int P2_YX = SW_TX + 2, P2_YY = SW_TY + 2;  // x' plane, halo 1
constexpr int P2_KX = SW_TX + 3, P2_KY = SW_TY + 3;  // cell layer, cells from i0-2, j0-2

template <typename T, int KIND, int CA, bool ZERO>
__global__ __launch_bounds__(256) void k_sweep3_pair(Geo g, StencilParams<T> op, int kz, int nzc,
                                                     int remap, Batch B) {
  constexpr bool KAP = KIND == OP_KAPPA;
  static_assert(KIND != OP_MASS, "paired half-sweeps carry no face couplings");
  constexpr int CB = 1 - CA;
  __shared__ T sxp[ZERO ? 1 : 3][P2_XY][P2_XX];
  __shared__ T syp[3][P2_YY][P2_YX];
  __shared__ T skp[KAP ? 4 : 1][P2_KY][P2_KX];
  const int n = g.n, m = n - 1;
  const long sy = g.sy, sz = g.sz;
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if (remap) {
    const int gxy = gridDim.x * gridDim.y;
    const int nb = gxy * gridDim.z;
    const int L = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
    bx = L % gridDim.x;
    by = (L / gridDim.x) % gridDim.y;
    bz = L / gxy;
  }
  const int item = bz / nzc, zc = bz % nzc;
  const Item& I = B.it[item];
  const T* __restrict__ x = (const T*)I.a;
  const T* __restrict__ b = (const T*)I.b;
  T* __restrict__ out = (T*)I.c;
  const T* __restrict__ kap = (const T*)I.kappa;
  const int i0 = 1 + bx * SW_TX, j0 = 1 + by * SW_TY, k0 = 1 + zc * kz;
  const int k1 = min(k0 + kz - 1, m);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int i = i0 + 2 * tx, j = j0 + ty;
  const bool row_ok = j <= m;
  const bool ok0 = row_ok && i <= m, ok1 = row_ok && i + 1 <= m;
  auto cl = [](int v, int hi) { return min(max(v, 0), hi); };

  // staging of x planes (halo 2) and cell layers: every load at a clamped
  // address and behind no branch (positions off the grid are only seen by
  // stencils of nodes that are not updated)
  constexpr int NXP = (P2_XX * P2_XY + 255) / 256;
  constexpr int NKP = (P2_KX * P2_KY + 255) / 256;
  int xoff[NXP];
  T xpf[NXP];
#pragma unroll
  for (int q = 0; q < NXP; ++q) {
    const int e = tid + 256 * q;
    const int r = e / P2_XX, c = e - r * P2_XX;
    xoff[q] = cl(i0 - 2 + c, n) + cl(j0 - 2 + r, n) * (int)sy;
  }
  auto prefetch_x = [&](int z) {
    const T* __restrict__ xz = x + (long)cl(z, n) * sz;
#pragma unroll
    for (int q = 0; q < NXP; ++q) xpf[q] = xz[xoff[q]];
  };
  auto commit_x = [&](int slot) {
    T* dst = &sxp[ZERO ? 0 : slot][0][0];
#pragma unroll
    for (int q = 0; q < NXP; ++q) {
      const int e = tid + 256 * q;
      if (e < P2_XX * P2_XY) dst[e] = xpf[q];
    }
  };
  int koff[NKP];
  T kpf[NKP];
  if (KAP) {
#pragma unroll
    for (int q = 0; q < NKP; ++q) {
      const int e = tid + 256 * q;
      const int r = e / P2_KX, c = e - r * P2_KX;
      koff[q] = cl(i0 - 2 + c, n - 1) + n * cl(j0 - 2 + r, n - 1);
    }
  }
  auto prefetch_k = [&](int cz) {
    const T* __restrict__ kz_ = kap + (long)n * n * cl(cz, n - 1);
#pragma unroll
    for (int q = 0; q < NKP; ++q) kpf[q] = kz_[koff[q]];
  };
  auto commit_k = [&](int slot) {
    T* dst = &skp[KAP ? slot : 0][0][0];
#pragma unroll
    for (int q = 0; q < NKP; ++q) {
      const int e = tid + 256 * q;
      if (e < P2_KX * P2_KY) dst[e] = kpf[q];
    }
  };
  auto xs = [](int z) { return (z + 3) % 3; };  // slot of x / x' plane z (z >= -1)
  auto ks = [](int z) { return (z + 4) & 3; };  // slot of cell layer z (z >= -2)

  // right-hand sides: of the ring+tile positions of the plane updated next
  // (colour CA) and of this thread's two unknowns (colour 1-CA)
  constexpr int NYP = (P2_YX * P2_YY + 255) / 256;
  int boff[NYP];
#pragma unroll
  for (int q = 0; q < NYP; ++q) {
    const int e = tid + 256 * q;
    const int r = e / P2_YX, c = e - r * P2_YX;
    boff[q] = cl(i0 - 1 + c, n) + cl(j0 - 1 + r, n) * (int)sy;
  }
  T bA[NYP], bB[2];
  auto prefetch_bA = [&](int z) {
    const T* __restrict__ bz_ = b + (long)cl(z, n) * sz;
#pragma unroll
    for (int q = 0; q < NYP; ++q) bA[q] = bz_[boff[q]];
  };
  const long pb0 = min(i, n - 1) + min(j, n) * sy;
  auto prefetch_bB = [&](int z) {
    const long p = pb0 + (long)cl(z, n) * sz;
    bB[0] = b[p];
    bB[1] = b[p + 1];
  };

  // colour CA on plane q over the ring and the tile -> x' plane q
  auto update_a = [&](int q, const T (&bv)[NYP]) {
    T* __restrict__ yd = &syp[xs(q)][0][0];
#pragma unroll
    for (int t = 0; t < NYP; ++t) {
      const int e = tid + 256 * t;
      if (e >= P2_YX * P2_YY) continue;
      const int r = e / P2_YX, c = e - r * P2_YX;
      const int gi = i0 - 1 + c, gj = j0 - 1 + r;
      const bool unk = gi >= 1 && gi <= m && gj >= 1 && gj <= m && q >= 1 && q <= m;
      const bool upd = unk && ((gi + gj + q) & 1) == CA;
      T val;
      if (!upd) {
        val = ZERO ? T(0) : sxp[ZERO ? 0 : xs(q)][r + 1][c + 1];
      } else {
        T kk[2][2][2];
        if (KAP) {
#pragma unroll
          for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
              for (int aa = 0; aa < 2; ++aa) kk[cc][bb][aa] = skp[ks(q - 1 + cc)][r + bb][c + aa];
        }
        if (ZERO) {
          const T dg = KAP ? kappa_diag3(op, kk) : op.wc;
          val = bv[t] / dg;
        } else {
          T v[3][3][3];
#pragma unroll
          for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
              for (int dx = 0; dx < 3; ++dx) v[dz][dy][dx] = sxp[xs(q - 1 + dz)][r + dy][c + dx];
          T ax, dg;
          if (KAP) {
            ax = stencil3_kappa(op, kk, v, dg);
          } else {
            ax = stencil3_const(op, v);
            dg = op.wc;
          }
          val = v[1][1][1] + (bv[t] - ax) / dg;
        }
      }
      yd[e] = val;
    }
  };
  // colour 1-CA on plane q of the tile from the x' planes; both colours out
  auto update_b = [&](int q, const T (&bv)[2]) {
    const long p = i + j * sy + (long)q * sz;
    auto one = [&](auto ubc) {
      constexpr int ub = decltype(ubc)::value;  // updated column
      constexpr int ua = 1 - ub;
      if (ua == 0 ? ok0 : ok1) out[p + ua] = syp[xs(q)][ty + 1][2 * tx + ua + 1];
      if (!(ub == 0 ? ok0 : ok1)) return;
      T v[3][3][3];
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) v[dz][dy][dx] = syp[xs(q - 1 + dz)][ty + dy][2 * tx + ub + dx];
      T ax, dg;
      if (KAP) {
        T kk[2][2][2];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
          for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
              kk[cc][bb][aa] = skp[ks(q - 1 + cc)][ty + 1 + bb][2 * tx + ub + 1 + aa];
        ax = stencil3_kappa(op, kk, v, dg);
      } else {
        ax = stencil3_const(op, v);
        dg = op.wc;
      }
      out[p + ub] = v[1][1][1] + (bv[ub] - ax) / dg;
    };
    if (((i + j + q) & 1) == CB)  // the same for a whole wavefront (row j)
      one(std::integral_constant<int, 0>{});
    else
      one(std::integral_constant<int, 1>{});
  };

  // each load is issued one step before its use
  if (!ZERO) prefetch_x(k0 - 2);
  if (KAP) prefetch_k(k0 - 3);
  prefetch_bA(k0 - 3);
  prefetch_bB(k0 - 4);
  for (int s = k0 - 2; s <= k1 + 2; ++s) {
    if (!ZERO) {
      commit_x(xs(s));  // plane s
      prefetch_x(s + 1);
    }
    if (KAP) {
      commit_k(ks(s - 1));  // cell layer s-1
      prefetch_k(s);
    }
    T bAc[NYP];
#pragma unroll
    for (int q = 0; q < NYP; ++q) bAc[q] = bA[q];  // b of plane s-1
    const T bBs[2] = {bB[0], bB[1]};                // b of plane s-2
    prefetch_bA(s);
    prefetch_bB(s - 1);
    __syncthreads();
    if (s >= k0) update_a(s - 1, bAc);
    __syncthreads();
    if (s >= k0 + 2) update_b(s - 2, bBs);
  }
}

// ---------------------------------------------------------------------------
// batched node kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* __restrict__ v, long count, T val) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long stride = (long)gridDim.x * blockDim.x;
  for (; t < count; t += stride) v[t] = val;
}

template <typename T>
__global__ void k_copy(const T* __restrict__ a, T* __restrict__ b, long count) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long stride = (long)gridDim.x * blockDim.x;
  for (; t < count; t += stride) b[t] = a[t];
}

// Node (i, j, k) of request `item`, and the block's index within its request.
#define NODE_INDEX(DIM, G)                                               \
  const int m = (G).n - 1;                                               \
  const int item = (DIM) == 3 ? (int)blockIdx.z / m : (int)blockIdx.z;   \
  const int plane = (DIM) == 3 ? (int)blockIdx.z % m : 0;                \
  const int i = 1 + blockIdx.x * BX + threadIdx.x;                       \
  const int j = 1 + blockIdx.y * BY + threadIdx.y;                       \
  const int k = (DIM) == 3 ? 1 + plane : 0;                              \
  const bool inside = (i <= m) && (j <= m);                              \
  const long p = i + j * (G).sy + (long)k * (G).sz;                      \
  const Item& I = B.it[item];

// u[p] = the colour-split vector's entry of node p, every node.
template <typename T>
__global__ __launch_bounds__(256) void k_unsplit(long nodes, Batch B) {
  const Item& I = B.it[blockIdx.y];
  const T* __restrict__ ev = (const T*)I.a;
  const T* __restrict__ od = (const T*)I.a2;
  T* __restrict__ u = (T*)I.c;
  for (long p = blockIdx.x * 256L + threadIdx.x; p < nodes; p += 256L * gridDim.x)
    u[p] = ((p & 1) ? od : ev)[p >> 1];
}

template <typename T, int DIM, int KIND, bool NORM>
__global__ __launch_bounds__(256) void k_residual(Geo g, StencilParams<T> op, Batch B) {
  NODE_INDEX(DIM, g)
  const DGeo dg = dgeo(g);
  double sq = 0.0;
  if (inside) {
    const T res = residual_node<T, DIM, KIND>(op, (const T*)I.kappa, dg, (const T*)I.a,
                                              (const T*)I.b, p, i, j, k);
    ((T*)I.c)[p] = res;
    sq = (double)res * (double)res;
  }
  if (NORM) {
    const double t = block_sum(sq);
    if (threadIdx.x == 0 && threadIdx.y == 0)
      I.partials[blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * plane)] = t;
  }
}

template <typename T, int DIM, int KIND, int KS, bool ZERO>
__global__ __launch_bounds__(256) void k_smooth(Geo g, StencilParams<T> op, T omega, Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside) return;
  ((T*)I.c)[p] = smooth_node<T, DIM, KIND>(op, (const T*)I.kappa, dgeo(g), KS,
                                           ZERO ? nullptr : (const T*)I.a, (const T*)I.b,
                                           omega, p, i, j, k);
}

// Gauss-Seidel update of the unknowns of colour `colour` of c in place.
template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(256) void k_smooth_gs(Geo g, StencilParams<T> op, int colour,
                                                   Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside || gs_colour(i, j, k) != colour) return;
  T* x = (T*)I.c;
  x[p] = gs_node<T, DIM, KIND>(op, (const T*)I.kappa, dgeo(g), x, (const T*)I.b, p, i, j, k);
}

// Partial sums of (b - A x)^2 and, written to c, the first smoothing step
// of x: KS = SM_JACOBI updates every unknown, SM_RB0 those of colour 0.
template <typename T, int DIM, int KIND, int KS>
__global__ __launch_bounds__(256) void k_head(Geo g, StencilParams<T> op, T omega, Batch B) {
  NODE_INDEX(DIM, g)
  double sq = 0.0;
  if (inside) {
    const T* __restrict__ x = (const T*)I.a;
    T ax, dg;
    Apply<T, DIM, KIND>::at(op, (const T*)I.kappa, dgeo(g), x, p, i, j, k, ax, dg);
    const T res = ((const T*)I.b)[p] - ax;
    sq = (double)res * (double)res;
    const T q = res / dg;
    const bool upd = KS == SM_JACOBI || ((i + j + k) & 1) == 0;
    ((T*)I.c)[p] = upd ? (KS == SM_JACOBI ? x[p] + omega * q : x[p] + q) : x[p];
  }
  const double t = block_sum(sq);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    I.partials[blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * plane)] = t;
}

// q = A x with per-block partial sums of x.q.
template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(256) void k_apply_dot(Geo g, StencilParams<T> op, Batch B) {
  NODE_INDEX(DIM, g)
  double sq = 0.0;
  if (inside) {
    const T* __restrict__ x = (const T*)I.a;
    T ax, dg;
    Apply<T, DIM, KIND>::at(op, (const T*)I.kappa, dgeo(g), x, p, i, j, k, ax, dg);
    ((T*)I.c)[p] = ax;
    sq = (double)x[p] * (double)ax;
  }
  const double t = block_sum(sq);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    I.partials[blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * plane)] = t;
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, Batch B) {
  NODE_INDEX(DIM, gc)
  if (!inside) return;
  ((T*)I.c)[lay_idx(p, I.lay)] = restrict_node<T, DIM>(dgeo(gf), (const T*)I.a, i, j, k);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_add(Geo gf, Geo gc, Batch B) {
  NODE_INDEX(DIM, gf)
  if (!inside) return;
  T* x = (T*)I.c;
  x[p] += prolong_node<T, DIM>(dgeo(gc), (const T*)I.a, i, j, k);
}

// 3D prolongation + add marching in z: a block of 64 x 4 threads owns a
// 64 x 4 tile of fine (i, j) columns over PZ (even) consecutive fine planes
// starting at an odd plane 2K+1.  Those read the coarse planes K .. K + PZ/2
// only, and within a plane the 33 x 3 coarse nodes under the tile: the
// block stages them in LDS with one coalesced pass (about 0.4 coarse loads
// per thread and coarse plane instead of up to 4 gathers), then every
// thread forms the in-plane interpolant of each coarse plane once (plane(K)
// in prolong_node serves fine planes 2K-1, 2K and 2K+1).  The values
// combined are those of prolong_node, in its order, so the result is
// bitwise that of k_prolong_add.
template <typename T, int PZ>
__global__ __launch_bounds__(256) void k_prolong_add_z(Geo gf, Geo gc, Batch B, int chunks) {
  static_assert(PZ % 2 == 0 && BX == 64 && BY == 4, "tile of 64 x 4 columns, odd first plane");
  constexpr int NC = PZ / 2 + 1, CX = BX / 2 + 1, CY = BY / 2 + 1;
  __shared__ T sc[NC][CY][CX];
  const int m = gf.n - 1, nc = gc.n;
  const int item = (int)blockIdx.z / chunks;
  const int kb = 1 + ((int)blockIdx.z % chunks) * PZ;
  const int nk = min(PZ, m - kb + 1);  // fine planes kb .. kb + nk - 1
  const int cl = (kb + nk) >> 1;       // last coarse plane they read (<= nc)
  const int ci = BX / 2 * blockIdx.x, cj = BY / 2 * blockIdx.y, ck = kb >> 1;
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = 1 + blockIdx.y * BY + threadIdx.y;
  const bool inside = i <= m && j <= m;
  const Item& I = B.it[item];
  const T* __restrict__ e = (const T*)I.a;
  T* __restrict__ x = (T*)I.c;
  const long fz = gf.sz;
  const long p = i + j * gf.sy + (long)kb * fz;
  T xv[PZ];
#pragma unroll
  for (int q = 0; q < PZ; ++q) xv[q] = inside && q < nk ? x[p + q * fz] : T(0);
  const int tid = threadIdx.x + BX * threadIdx.y;
  for (int t = tid; t < NC * CY * CX; t += BX * BY) {
    const int c = t / (CY * CX), r = (t / CX) % CY, a = t % CX;
    const int gi = ci + a, gj = cj + r, gk = ck + c;
    T v = T(0);
    if (gi <= nc && gj <= nc && gk <= cl) v = e[gi + gj * gc.sy + (long)gk * gc.sz];
    (&sc[0][0][0])[t] = v;
  }
  __syncthreads();
  if (!inside) return;
  const int a0 = (i >> 1) - ci, a1 = ((i + 1) >> 1) - ci;
  const int r0 = (j >> 1) - cj, r1 = ((j + 1) >> 1) - cj;
  const T wi = (i & 1) ? T(0.5) : T(1);
  const T wj = (j & 1) ? T(0.5) : T(1);
  auto line = [&](int rr, int c) -> T {
    return (i & 1) ? wi * (sc[c][rr][a0] + sc[c][rr][a1]) : sc[c][rr][a0];
  };
  T pl[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) pl[c] = (j & 1) ? wj * (line(r0, c) + line(r1, c)) : line(r0, c);
#pragma unroll
  for (int q = 0; q < PZ; ++q) {
    // fine plane kb + q: odd for even q (parents ck + q/2 and the next),
    // even for odd q (parent ck + (q + 1)/2)
    const T v = (q & 1) ? pl[(q + 1) / 2] : T(0.5) * (pl[q / 2] + pl[q / 2 + 1]);
    if (q < nk) x[p + q * fz] = xv[q] + v;
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_norm2_partial(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  double sq = 0.0;
  if (inside) {
    const double a = (double)((const T*)I.a)[p];
    sq = a * a;
  }
  const double t = block_sum(sq);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    I.partials[blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * plane)] = t;
}

// The partial sums of k_norm2_partial (same grid, same order) for v = I.a,
// and the colour-split copy of v on the unknowns into I.c (odd half at
// I.lay) in the same pass.  The copy's boundary entries are not written.
template <int DIM>
__global__ __launch_bounds__(256) void k_split_norm(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  double sq = 0.0;
  if (inside) {
    const double a = ((const double*)I.a)[p];
    ((double*)I.c)[lay_idx(p, I.lay)] = a;
    sq = a * a;
  }
  const double t = block_sum(sq);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    I.partials[blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * plane)] = t;
}

// b32 = float(r / s) on the unknowns, s = ir_scale(||b||^2) (read from
// device memory).
template <int DIM>
__global__ __launch_bounds__(256) void k_scale_cast(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside) return;
  const double s = ir_scale(*I.scal);
  ((float*)I.c)[lay_idx(p, I.lay)] = (float)(((const double*)I.a)[p] / s);
}

// u += s * double(c) on the unknowns, s = ir_scale(||b||^2).
template <int DIM>
__global__ __launch_bounds__(256) void k_ir_update(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside) return;
  const double s = ir_scale(*I.scal);
  double* u = (double*)I.c;
  u[p] = u[p] + s * (double)((const float*)I.a)[p];
}

// Sum partials[0..count) of request blockIdx.x in a fixed order with 1024
// threads: thread t owns entries t, t + 1024, ... and keeps 8 independent
// partial sums (so 8 loads are in flight), combined in a fixed order; then
// a wave butterfly and the 16 wave sums in order.
constexpr int RED_THREADS = 1024;
__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(long count, Batch B) {
  __shared__ double ws[RED_THREADS / 64];
  const Item& I = B.it[blockIdx.x];
  const double* __restrict__ partials = I.partials;
  const int t = threadIdx.x;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long q = t;
  for (; q + 7L * RED_THREADS < count; q += 8L * RED_THREADS) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += partials[q + (long)u * RED_THREADS];
  }
  for (int u = 0; q < count; q += RED_THREADS, ++u) a[u & 7] += partials[q];
  double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((t & 63) == 0) ws[t >> 6] = s;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) tot += ws[w];
    *I.scal = tot;
  }
}

// ---------------------------------------------------------------------------
// coarsest solve
// ---------------------------------------------------------------------------

// Dense Cholesky substitution by one block: gather the unknowns of b into
// y, forward substitution L y' = y, back substitution L^T z = y', scatter.
// L is the row-major lower factor (m x m).
template <typename T>
__device__ void cholesky_solve_block(int dim, int n, const double* __restrict__ L, int m,
                                     const T* __restrict__ bc, T* __restrict__ xc, double* y) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int mi = n - 1;
  const long sy = n + 1, sz = dim == 3 ? (long)(n + 1) * (n + 1) : 0;
  for (int q = t; q < m; q += nt) {
    const int qx = q % mi, qy = (q / mi) % mi, qz = dim == 3 ? q / (mi * mi) : 0;
    y[q] = (double)bc[(qx + 1) + (qy + 1) * sy + (long)(qz + 1) * sz];
  }
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    if (t == 0) y[c] = y[c] / L[(long)c * m + c];
    __syncthreads();
    const double yc = y[c];
    for (int q = c + 1 + t; q < m; q += nt) y[q] -= L[(long)q * m + c] * yc;
    __syncthreads();
  }
  for (int c = m - 1; c >= 0; --c) {
    if (t == 0) y[c] = y[c] / L[(long)c * m + c];
    __syncthreads();
    const double yc = y[c];
    for (int q = t; q < c; q += nt) y[q] -= L[(long)c * m + q] * yc;
    __syncthreads();
  }
  for (int q = t; q < m; q += nt) {
    const int qx = q % mi, qy = (q / mi) % mi, qz = dim == 3 ? q / (mi * mi) : 0;
    xc[(qx + 1) + (qy + 1) * sy + (long)(qz + 1) * sz] = (T)y[q];
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(Geo g, int m, Batch B) {
  __shared__ double y[kCoarseMaxUnknowns];
  const Item& I = B.it[blockIdx.x];
  cholesky_solve_block<T>(g.dim, g.n, I.L, m, (const T*)I.b, (T*)I.c, y);
}

// ---------------------------------------------------------------------------
// tail: the V-cycle on the coarse levels l0..L-1 inside one workgroup
// ---------------------------------------------------------------------------

// Calls f(p, i, j, k) for every unknown of a level, the block's threads
// striding over the unknowns in x-fastest order.
template <int DIM, typename F>
__device__ __forceinline__ void for_unknowns(int n, const DGeo& g, F f) {
  const int mi = n - 1;
  const int total = DIM == 3 ? mi * mi * mi : mi * mi;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int i = q % mi + 1;
    const int j = (q / mi) % mi + 1;
    const int k = DIM == 3 ? q / (mi * mi) + 1 : 0;
    f(i + j * g.sy + (long)k * g.sz, i, j, k);
  }
}

// A red-black pass over the unknowns of a level: thread q takes, in one
// grid row, the h-th unknown of colour `colour` (f_upd) and the h-th of the
// other colour (f_oth), so that every lane of a wave computes a stencil
// (enumerating all unknowns would leave every other lane idle in it).
template <int DIM, typename F, typename G>
__device__ __forceinline__ void for_colour_pairs(int n, const DGeo& g, int colour, F f_upd,
                                                 G f_oth) {
  const int mi = n - 1;
  const int half = (mi + 1) / 2;
  const int rows = DIM == 3 ? mi * mi : mi;
  const int total = rows * half;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int h = q % half, row = q / half;
    const int j = row % mi + 1;
    const int k = DIM == 3 ? row / mi + 1 : 0;
    const int iu = ((1 + j + k) & 1) == colour ? 1 : 2;  // first unknown of the colour
    const int i1 = iu + 2 * h, i2 = (3 - iu) + 2 * h;
    const long rb = j * g.sy + (long)k * g.sz;
    if (i1 <= mi) f_upd(i1 + rb, i1, j, k);
    if (i2 <= mi) f_oth(i2 + rb, i2, j, k);
  }
}

// The tail keeps every vector of its levels in the launch's dynamic LDS
// (element offsets in TailDesc): iterate, spare, right-hand side, residual
// and, for OP_KAPPA, the cell coefficients.  The region is zeroed first, so
// boundary entries read 0; the first level's right-hand side and iterate
// (unless it starts at 0) and the coefficients are copied in, the iterate
// is copied out at the end.

// Copies the descriptor at `desc` into D, zeroes the LDS region and copies
// the cell coefficients in.
template <typename T, int DIM, int KIND>
__device__ void tail_load(TailDesc<T>& D, char* tail_lds, const void* desc) {
  {
    const int* src = reinterpret_cast<const int*>(desc);
    int* dst = reinterpret_cast<int*>(&D);
    for (int q = threadIdx.x; q < (int)(sizeof(TailDesc<T>) / sizeof(int)); q += blockDim.x)
      dst[q] = src[q];
  }
  __syncthreads();
  {
    float4* z = reinterpret_cast<float4*>(tail_lds);
    for (int q = threadIdx.x; q < D.lds_bytes / 16; q += blockDim.x)
      z[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  T* const sm = reinterpret_cast<T*>(tail_lds);
  if (KIND == OP_KAPPA) {
    for (int l = 0; l < D.nlev; ++l) {
      const int n = D.lv[l].n;
      const int cells = DIM == 3 ? n * n * n : n * n;
      T* dst = sm + D.lv[l].ok;
      const T* src = D.lv[l].kappa;
      for (int q = threadIdx.x; q < cells; q += blockDim.x) dst[q] = src[q];
    }
  }
}

// The first tail level's current iterate (bit 0 of par: in the spare).
template <typename T>
__device__ __forceinline__ T* tail_x0(const TailDesc<T>& D, char* tail_lds, int par) {
  return reinterpret_cast<T*>(tail_lds) + ((par & 1) ? D.lv[0].ot : D.lv[0].ox);
}

// One cycle over the tail levels, every vector in LDS: from the first
// level's iterate (or from 0 when bit 0 of `flag` is set) to the new one,
// in tail_x0 afterwards.  Bits 1-2 of `flag`: the cycle kind (CycleKind).
// Bit l of `par` tells whether level l's iterate currently sits in its
// spare buffer.
template <typename T, int DIM, int KIND>
__device__ void tail_cycle(const TailDesc<T>& D, char* tail_lds, int& par, int flag) {
  T* const sm = reinterpret_cast<T*>(tail_lds);
  const int nl = D.nlev;
  auto X = [&](int l) { return sm + (((par >> l) & 1) ? D.lv[l].ot : D.lv[l].ox); };
  auto S = [&](int l) { return sm + (((par >> l) & 1) ? D.lv[l].ox : D.lv[l].ot); };
  auto params = [&](int l) {
    return StencilParams<T>{KIND, D.lv[l].wc, D.lv[l].w1, D.lv[l].w2, D.lv[l].s, D.lv[l].wf};
  };
  // nu sweeps on level l from X(l) (or from 0 if *zero)
  auto smooth = [&](int l, bool pre, bool* zero) {
    const int n = D.lv[l].n;
    const DGeo g = dgeo(DIM, n);
    const StencilParams<T> op = params(l);
    const T* kap = sm + D.lv[l].ok;
    const T* b = sm + D.lv[l].ob;
    const T omega = D.omega;
    const int smoother = D.smoother;
    const int nu = pre ? D.nu_pre : D.nu_post;
    if (smoother == 2) {
      // multicolour Gauss-Seidel in place: colours in order (pre) or in
      // reverse order (post)
      if (nu == 0) return;
      T* x = X(l);
      if (*zero) {
        for_unknowns<DIM>(n, g, [&](long p, int, int, int) { x[p] = T(0); });
        __syncthreads();
        *zero = false;
      }
      const int ncol = 1 << DIM;
      for (int it = 0; it < nu; ++it)
        for (int q = 0; q < ncol; ++q) {
          const int col = pre ? q : ncol - 1 - q;
          for_unknowns<DIM>(n, g, [&](long p, int i, int j, int k) {
            if (gs_colour(i, j, k) == col) x[p] = gs_node<T, DIM, KIND>(op, kap, g, x, b, p, i, j, k);
          });
          __syncthreads();
        }
      return;
    }
    for (int it = 0; it < nu; ++it) {
      for (int h = 0; h < (smoother == 0 ? 1 : 2); ++h) {
        const int ks = smoother == 0 ? SM_JACOBI : ((h == 0) == pre ? SM_RB0 : SM_RB1);
        const T* xin = *zero ? nullptr : X(l);
        T* xout = S(l);
        // the step kind is a constant in each instance, as in the grid
        // kernels, so both contract the update the same way
        auto sweep = [&](auto kind) {
          constexpr int KS = decltype(kind)::value;
          auto node = [&](long p, int i, int j, int k) {
            xout[p] = smooth_node<T, DIM, KIND>(op, kap, g, KS, xin, b, omega, p, i, j, k);
          };
          if (KS == SM_JACOBI)
            for_unknowns<DIM>(n, g, node);
          else
            for_colour_pairs<DIM>(n, g, KS == SM_RB1 ? 1 : 0, node, node);
        };
        if (ks == SM_JACOBI)
          sweep(std::integral_constant<int, SM_JACOBI>{});
        else if (ks == SM_RB0)
          sweep(std::integral_constant<int, SM_RB0>{});
        else
          sweep(std::integral_constant<int, SM_RB1>{});
        __syncthreads();
        par ^= 1 << l;
        *zero = false;
      }
    }
  };
  // pre-smoothing of level l (from 0 when `zero`) and restriction of its
  // residual to level l+1
  auto down = [&](int l, bool zero) {
    const int n = D.lv[l].n;
    const DGeo g = dgeo(DIM, n);
    smooth(l, true, &zero);
    T* x = X(l);
    if (zero) {
      for_unknowns<DIM>(n, g, [&](long p, int, int, int) { x[p] = T(0); });
      __syncthreads();
    }
    const StencilParams<T> op = params(l);
    const T* kap = sm + D.lv[l].ok;
    const T* b = sm + D.lv[l].ob;
    const int nc = D.lv[l + 1].n;
    T* bc = sm + D.lv[l + 1].ob;
    auto resid_restrict = [&](T* r) {
      for_unknowns<DIM>(n, g, [&](long p, int i, int j, int k) {
        r[p] = residual_node<T, DIM, KIND>(op, kap, g, x, b, p, i, j, k);
      });
      __syncthreads();
      for_unknowns<DIM>(nc, dgeo(DIM, nc), [&](long p, int i, int j, int k) {
        bc[p] = restrict_node<T, DIM>(g, r, i, j, k);
      });
      __syncthreads();
    };
    if (l == 0 && D.r0 != nullptr)
      resid_restrict(D.r0);  // device memory
    else
      resid_restrict(sm + D.lv[l].orr);
  };
  // prolongation of level l+1's correction into level l, post-smoothing
  auto up = [&](int l) {
    const int n = D.lv[l].n;
    const DGeo gc = dgeo(DIM, D.lv[l + 1].n);
    T* x = X(l);
    const T* e = X(l + 1);
    for_unknowns<DIM>(n, dgeo(DIM, n), [&](long p, int i, int j, int k) {
      x[p] += prolong_node<T, DIM>(gc, e, i, j, k);
    });
    __syncthreads();
    bool zero = false;
    smooth(l, false, &zero);
  };
  auto coarse = [&]() {
    cholesky_solve_block<T>(DIM, D.lv[nl - 1].n, D.L, D.m, sm + D.lv[nl - 1].ob, X(nl - 1),
                            reinterpret_cast<double*>(tail_lds + D.oy));
    __syncthreads();
  };
  // The cycle over the tail levels, iteratively: each level visited by a
  // cycle of some kind (V, W or F) runs that kind's coarse cycles (V: one V;
  // W: two W; F: an F then a V; one exact solve directly above the
  // coarsest level) before its post-smoothing.  Level l's kind and the
  // number of its coarse cycles started are kept in 2-bit fields of `kinds`
  // and `starts`; every thread runs the same control flow.
  if (nl == 1) {
    coarse();
  } else {
    unsigned kinds = (unsigned)(flag >> 1) & 3u, starts = 0;
    auto kind_of = [&](int l) { return (int)((kinds >> (2 * l)) & 3u); };
    auto started = [&](int l) { return (int)((starts >> (2 * l)) & 3u); };
    int l = 0;
    down(0, (flag & 1) != 0);
    for (;;) {
      const int kd = kind_of(l);
      const int nsub = kd == CYC_V ? 1 : 2;
      if (l + 1 < nl - 1 && started(l) < nsub) {
        const int i = started(l);
        const int sub = kd == CYC_W ? CYC_W : (kd == CYC_F && i == 0 ? CYC_F : CYC_V);
        starts += 1u << (2 * l);
        ++l;
        kinds = (kinds & ~(3u << (2 * l))) | ((unsigned)sub << (2 * l));
        starts &= ~(3u << (2 * l));
        down(l, i == 0);
        continue;
      }
      if (l + 1 == nl - 1) coarse();
      up(l);
      if (l == 0) break;
      --l;
    }
  }
}

template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(Batch B) {
  extern __shared__ __align__(16) char tail_lds[];
  __shared__ TailDesc<T> D;
  const Item& I = B.it[blockIdx.x];
  tail_load<T, DIM, KIND>(D, tail_lds, I.a);
  T* const sm = reinterpret_cast<T*>(tail_lds);
  T* const x0g = (T*)I.c;
  const T* const b0g = (const T*)I.b;
  {
    T* xd = sm + D.lv[0].ox;
    T* bd = sm + D.lv[0].ob;
    const bool cx = !(I.flag & 1);
    for_unknowns<DIM>(D.lv[0].n, dgeo(DIM, D.lv[0].n), [&](long p, int, int, int) {
      bd[p] = b0g[p];
      if (cx) xd[p] = x0g[p];
    });
  }
  __syncthreads();
  int par = 0;
  tail_cycle<T, DIM, KIND>(D, tail_lds, par, I.flag);
  const T* src = tail_x0(D, tail_lds, par);
  for_unknowns<DIM>(D.lv[0].n, dgeo(DIM, D.lv[0].n),
                    [&](long p, int, int, int) { x0g[p] = src[p]; });
}

// Sum of v over the TAIL_THREADS threads of a tail block, in a fixed order
// (wave butterflies, then the wave sums in wave order); every thread gets
// the sum.  ws: TAIL_THREADS / 64 doubles of shared memory.
__device__ __forceinline__ double tail_block_sum(double v, double* ws) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < TAIL_THREADS / 64; ++w) t += ws[w];
  __syncthreads();
  return t;
}

// A whole FP64 solve of a hierarchy the tail holds from its finest level
// on, in one workgroup: u_0 = 0, then cycles of the descriptor's kind until
// ||b - A u_k||_2 / ||b||_2 <= tol (the outer iteration of Sec. 5.5.1, the
// stopping rule of the cycle-by-cycle solve), with the iterate kept in LDS
// between cycles.  Item: a = TailDesc<double>* (device), b = b (every node
// of the finest level, boundary entries ignored), c = u (every node
// written, boundary 0), scal = results: [0] status (TailSolveStatus),
// [1] cycles done, [2 + k] the relative residual after cycle k ([2] = 1).
// flag: the cycle kind in bits 1-2.

template <int DIM, int KIND>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_solve(Batch B, double tol, int max_iter) {
  extern __shared__ __align__(16) char tail_lds[];
  __shared__ TailDesc<double> D;
  __shared__ double ws[TAIL_THREADS / 64];
  const Item& I = B.it[blockIdx.x];
  tail_load<double, DIM, KIND>(D, tail_lds, I.a);
  double* const sm = reinterpret_cast<double*>(tail_lds);
  double* const ug = (double*)I.c;
  const double* const bg = (const double*)I.b;
  double* const res = I.scal;
  const int n0 = D.lv[0].n;
  const DGeo g0 = dgeo(DIM, n0);
  double* const bd = sm + D.lv[0].ob;
  double sb = 0.0;
  for_unknowns<DIM>(n0, g0, [&](long p, int, int, int) {
    const double v = bg[p];
    bd[p] = v;
    sb += v * v;
  });
  const double nb2 = tail_block_sum(sb, ws);  // also orders the stores to bd
  const StencilParams<double> op{KIND, D.lv[0].wc, D.lv[0].w1, D.lv[0].w2, D.lv[0].s,
                                 D.lv[0].wf};
  const double* kap = sm + D.lv[0].ok;
  int status = TS_MAXIT, k = 0, par = 0;
  if (!isfinite(nb2)) {
    status = TS_NONFINITE_B;
  } else if (nb2 == 0.0) {
    status = TS_OK;  // u = 0 (the LDS iterate is zero)
  } else {
    const double nb = sqrt(nb2);
    if (threadIdx.x == 0) res[kTailSolveHead] = 1.0;
    while (k < max_iter) {
      tail_cycle<double, DIM, KIND>(D, tail_lds, par, (k == 0 ? 1 : 0) | (I.flag & 6));
      ++k;
      const double* x = tail_x0(D, tail_lds, par);
      double sr = 0.0;
      for_unknowns<DIM>(n0, g0, [&](long p, int i, int j, int kk) {
        const double r = residual_node<double, DIM, KIND>(op, kap, g0, x, bd, p, i, j, kk);
        sr += r * r;
      });
      const double rho = sqrt(tail_block_sum(sr, ws)) / nb;
      if (threadIdx.x == 0) res[kTailSolveHead + k] = rho;
      if (!isfinite(rho) || rho > 1e3) {
        status = TS_DIVERGED;
        break;
      }
      if (rho <= tol) {
        status = TS_OK;
        break;
      }
    }
  }
  // every node of u: the iterate's boundary entries in LDS are 0
  const double* src = tail_x0(D, tail_lds, par);
  const long nodes = DIM == 3 ? g0.sz * (n0 + 1) : g0.sy * (n0 + 1);
  for (long q = threadIdx.x; q < nodes; q += blockDim.x) ug[q] = src[q];
  if (threadIdx.x == 0) {
    res[0] = (double)status;
    res[1] = (double)k;
  }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// Coarse cell value = exp(mean(log kappa)) over the 2^dim children.
template <int DIM>
__global__ void k_kappa_coarsen(int nf, const double* __restrict__ kf, double* __restrict__ kc) {
  const int nc = nf / 2;
  const long total = DIM == 3 ? (long)nc * nc * nc : (long)nc * nc;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int cx = t % nc, cy = (t / nc) % nc, cz = DIM == 3 ? t / ((long)nc * nc) : 0;
  double g = 0.0;
  const long sfy = nf, sfz = (long)nf * nf;
  for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        g += log(kf[(2 * cx + a) + sfy * (2 * cy + b) + sfz * (2 * cz + c)]);
  kc[t] = exp(g / (DIM == 3 ? 8.0 : 4.0));
}

__global__ void k_cast_f32(const double* __restrict__ a, float* __restrict__ b, long count) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long stride = (long)gridDim.x * blockDim.x;
  for (; t < count; t += stride) b[t] = (float)a[t];
}

__global__ void k_count_bad_kappa(const double* __restrict__ k, long count, int* nonpos,
                                  int* nonfinite) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long stride = (long)gridDim.x * blockDim.x;
  int a = 0, b = 0;
  for (; t < count; t += stride) {
    const double v = k[t];
    if (!isfinite(v)) ++b;
    else if (!(v > 0.0)) ++a;
  }
  if (a) atomicAdd(nonpos, a);
  if (b) atomicAdd(nonfinite, b);
}

// ---------------------------------------------------------------------------
// Crank-Nicolson right-hand side (launch_cn_rhs), FP64:
//   b = Wb x0 - Wa x1 + cf F  on the unknowns,
// x0 = u inside and c0 g0 on the boundary, x1 = c1 g1 on the boundary and 0
// inside; guess (optional) = 2 u - guess.  k_cn_rhs: one thread per
// unknown, the 3^dim neighbours summed per class (centre, faces, edges,
// corners) and weighted per class; blocks whose unknowns all lie away from
// the boundary read u without boundary tests.  On the large 3D levels the
// interior part Wb u + cf F comes from k_sweep3 (SW_CN) with u's staged
// boundary values, and k_cn_bnd then adds, at the unknowns next to the
// boundary, Wb (c0 g0 - u) - Wa c1 g1 over their boundary neighbours.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(256) void k_cn_rhs(Geo g, CnWeights w, const double* __restrict__ u,
                                                double* __restrict__ guess,
                                                const double* __restrict__ g0,
                                                const double* __restrict__ g1,
                                                const double* __restrict__ F,
                                                double* __restrict__ b) {
  const int n = g.n, m = n - 1;
  const int i0 = 1 + blockIdx.x * BX, j0 = 1 + blockIdx.y * BY;
  const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
  const int k = DIM == 3 ? 1 + (int)blockIdx.z : 0;
  if (i > m || j > m) return;
  const long p = i + j * g.sy + (long)k * g.sz;
  const bool inner = i0 > 1 && i0 + BX - 1 < m && j0 > 1 && j0 + BY - 1 < m &&
                     (DIM == 2 || (k > 1 && k < m));
  constexpr int DZ = DIM == 3 ? 1 : 0;
  double s0[DIM + 1], s1[DIM + 1];
#pragma unroll
  for (int c = 0; c <= DIM; ++c) s0[c] = s1[c] = 0.0;
  if (inner) {
#pragma unroll
    for (int dz = -DZ; dz <= DZ; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int cls = (dx != 0) + (dy != 0) + (dz != 0);
          s0[cls] += u[p + dx + dy * g.sy + dz * g.sz];
        }
  } else {
#pragma unroll
    for (int dz = -DZ; dz <= DZ; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int cls = (dx != 0) + (dy != 0) + (dz != 0);
          const long q = p + dx + dy * g.sy + dz * g.sz;
          const int qi = i + dx, qj = j + dy, qk = k + dz;
          const bool bnd =
              qi == 0 || qi == n || qj == 0 || qj == n || (DIM == 3 && (qk == 0 || qk == n));
          if (bnd) {
            if (g0) s0[cls] += w.c0 * g0[q];
            if (g1) s1[cls] += w.c1 * g1[q];
          } else {
            s0[cls] += u[q];
          }
        }
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c <= DIM; ++c) acc += w.wb[c] * s0[c] - w.wa[c] * s1[c];
  b[p] = F ? acc + w.cf * F[p] : acc;
  if (guess) guess[p] = 2.0 * u[p] - guess[p];
}

// Boundary terms after a k_sweep3 SW_CN pass (3D): thread t covers one
// unknown of the layer next to the boundary, enumerated once each: the
// planes k = 1 and k = m whole, then for 1 < k < m the rows j = 1 and j = m,
// then the columns i = 1 and i = m of the remaining rows.
__global__ __launch_bounds__(256) void k_cn_bnd(Geo g, CnWeights w, const double* __restrict__ u,
                                                const double* __restrict__ g0,
                                                const double* __restrict__ g1,
                                                double* __restrict__ b) {
  const int n = g.n, m = n - 1;
  const long P = (long)m * m;                 // plane k = 1 or k = m
  const long R = 2L * m * (m - 2);            // rows j = 1, m of the inner planes
  const long C = 2L * (m - 2) * (m - 2);      // columns i = 1, m of the rest
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < 2 * P) {
    k = t < P ? 1 : m;
    const long r = t < P ? t : t - P;
    i = 1 + (int)(r % m);
    j = 1 + (int)(r / m);
  } else if ((t -= 2 * P) < R) {
    const long half = (long)m * (m - 2);
    j = t < half ? 1 : m;
    const long r = t < half ? t : t - half;
    i = 1 + (int)(r % m);
    k = 2 + (int)(r / m);
  } else if ((t -= R) < C) {
    const long half = (long)(m - 2) * (m - 2);
    i = t < half ? 1 : m;
    const long r = t < half ? t : t - half;
    j = 2 + (int)(r % (m - 2));
    k = 2 + (int)(r / (m - 2));
  } else {
    return;
  }
  const long p = i + j * g.sy + (long)k * g.sz;
  double s0[4] = {0.0, 0.0, 0.0, 0.0}, s1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int qi = i + dx, qj = j + dy, qk = k + dz;
        if (!(qi == 0 || qi == n || qj == 0 || qj == n || qk == 0 || qk == n)) continue;
        const int cls = (dx != 0) + (dy != 0) + (dz != 0);
        const long q = p + dx + dy * g.sy + dz * g.sz;
        s0[cls] += (g0 ? w.c0 * g0[q] : 0.0) - u[q];
        if (g1) s1[cls] += w.c1 * g1[q];
      }
  double acc = 0.0;
  for (int c = 0; c <= 3; ++c) acc += w.wb[c] * s0[c] - w.wa[c] * s1[c];
  b[p] += acc;
}

// v = 0 on the boundary nodes; thread t covers one node of the 2 dim faces.
template <int DIM>
__global__ void k_zero_boundary(Geo g, double* __restrict__ v) {
  const long N1 = g.n + 1;
  const long face = DIM == 3 ? N1 * N1 : N1;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= 2 * DIM * face) return;
  const int fi = (int)(t / face);
  const long r = t - fi * face;
  const long side = (fi & 1) ? g.n : 0;
  const long a = r % N1, c = DIM == 3 ? r / N1 : 0;
  long i, j, k;
  if ((fi >> 1) == 0) {
    i = side; j = a; k = c;
  } else if ((fi >> 1) == 1) {
    i = a; j = side; k = c;
  } else {
    i = a; j = c; k = side;
  }
  v[i + j * g.sy + k * g.sz] = 0.0;
}

inline unsigned flat_blocks(long count) {
  long b = (count + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
// Whether k_sweep3 (and its fused forms) runs the level: Geo::s3, set by
// make_geo for the 3D levels with at least 31 unknowns per direction and
// narrowed by the runtime per level.
inline bool use_sweep3(const Geo& g) { return g.s3; }

inline dim3 sweep3_grid(const Geo& g, int count, int* kz, int* nzc, int elem) {
  const int m = g.n - 1;
  *kz = sweep3_kz(m, elem);
  *nzc = (int)cdiv(m, *kz);
  return dim3(cdiv(m, SW_TX), cdiv(m, SW_TY), (unsigned)(*nzc * count));
}

// Whether sweep3 launches map tiles to XCDs (always, unless a tuning build
// is told otherwise by MG_SWEEP3_REMAP=0).
inline int sweep3_remap() {
#ifdef MG_TUNING_KNOBS
  static const int v = [] {
    const char* e = getenv("MG_SWEEP3_REMAP");
    return e ? (atoi(e) != 0) : 1;
  }();
  return v;
#else
  return 1;
#endif
}

template <typename T, int K, int MODE, bool ZERO, bool NORM, int XL = 0, bool IRU = false,
          bool CAST = false>
void launch_sweep3(const Geo& g, const StencilParams<T>& op, T omega, const Batch& B,
                   hipStream_t s) {
  int kz, nzc;
  const dim3 gr = sweep3_grid(g, B.count, &kz, &nzc, (int)sizeof(T));
  MG_LAUNCH((k_sweep3<T, K, MODE, ZERO, NORM, false, XL, IRU, CAST>), gr,
            dim3(64, SW_TY), 0, s, g, op, omega, kz, nzc, sweep3_remap(), B);
}

}  // namespace

long norm2_blocks(const Geo& g) {
  dim3 gr = node_grid(g, 1);
  return (long)gr.x * gr.y * gr.z;
}

long grid_blocks(const Geo& g) {
  if (use_sweep3(g)) {
    // (the launches that write partial sums are FP64)
    int kz, nzc;
    const dim3 gr = sweep3_grid(g, 1, &kz, &nzc, (int)sizeof(double));
    return (long)gr.x * gr.y * gr.z;
  }
  dim3 gr = node_grid(g, 1);
  return (long)gr.x * gr.y * gr.z;
}

template <typename T>
void launch_fill(T* v, long count, T val, hipStream_t s) {
  MG_LAUNCH(k_fill<T>, dim3(flat_blocks(count)), dim3(256), 0, s, v, count, val);
}
template <typename T>
void launch_copy(const T* a, T* b, long count, hipStream_t s) {
  MG_LAUNCH(k_copy<T>, dim3(flat_blocks(count)), dim3(256), 0, s, a, b, count);
}

// 2D operators are OP_CONST (any sigma) or OP_KAPPA; 3D ones any kind.
#define DISPATCH_DIM_KIND(dim, kind, MACRO)                                      \
  do {                                                                           \
    if ((dim) == 2) {                                                            \
      if ((kind) == OP_KAPPA) MACRO(2, OP_KAPPA); else MACRO(2, OP_CONST);       \
    } else {                                                                     \
      if ((kind) == OP_KAPPA) MACRO(3, OP_KAPPA);                                \
      else if ((kind) == OP_MASS) MACRO(3, OP_MASS);                             \
      else MACRO(3, OP_CONST);                                                   \
    }                                                                            \
  } while (0)

// f(std::integral_constant<int, K>) for the operator kind K of a 3D level.
template <typename F>
inline void with_kind3(int kind, F f) {
  if (kind == OP_KAPPA)
    f(std::integral_constant<int, OP_KAPPA>{});
  else if (kind == OP_MASS)
    f(std::integral_constant<int, OP_MASS>{});
  else
    f(std::integral_constant<int, OP_CONST>{});
}

template <typename T>
void launch_residual(const Geo& g, const StencilParams<T>& op, bool norm, const Batch& B,
                     hipStream_t s, int xl, bool cast) {
  if (cast) {
    // (the runtime asks for it on k_sweep3 levels in FP64 with norm)
    if constexpr (std::is_same<T, double>::value) {
      with_kind3(op.kind, [&](auto k) {
        constexpr int K = decltype(k)::value;
        launch_sweep3<T, K, SW_RESID, false, true, 0, false, true>(g, op, T(0), B, s);
      });
    }
    return;
  }
  if (xl == XL_SPLIT) {
    // (split iterates exist on k_sweep3 levels of the constant-coefficient
    // and mass-shifted kinds)
    if (op.kind == OP_MASS) {
      if (norm) launch_sweep3<T, OP_MASS, SW_RESID, false, true, XL_SPLIT>(g, op, T(0), B, s);
      else launch_sweep3<T, OP_MASS, SW_RESID, false, false, XL_SPLIT>(g, op, T(0), B, s);
    } else {
      if (norm) launch_sweep3<T, OP_CONST, SW_RESID, false, true, XL_SPLIT>(g, op, T(0), B, s);
      else launch_sweep3<T, OP_CONST, SW_RESID, false, false, XL_SPLIT>(g, op, T(0), B, s);
    }
    return;
  }
  if (use_sweep3(g)) {
    with_kind3(op.kind, [&](auto k) {
      constexpr int K = decltype(k)::value;
      if (norm)
        launch_sweep3<T, K, SW_RESID, false, true>(g, op, T(0), B, s);
      else
        launch_sweep3<T, K, SW_RESID, false, false>(g, op, T(0), B, s);
    });
    return;
  }
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
#define L_RES(D, K)                                                                   \
  do {                                                                                \
    if (norm)                                                                         \
      MG_LAUNCH((k_residual<T, D, K, true>), gr, bl, 0, s, g, op, B);                 \
    else                                                                              \
      MG_LAUNCH((k_residual<T, D, K, false>), gr, bl, 0, s, g, op, B);                \
  } while (0)
  DISPATCH_DIM_KIND(g.dim, op.kind, L_RES);
#undef L_RES
}

template <typename T, int D, int K, bool Z>
static void launch_smooth_k(const Geo& g, const StencilParams<T>& op, int kind, T omega,
                            const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (kind == SM_JACOBI)
    MG_LAUNCH((k_smooth<T, D, K, SM_JACOBI, Z>), gr, bl, 0, s, g, op, omega, B);
  else if (kind == SM_RB0)
    MG_LAUNCH((k_smooth<T, D, K, SM_RB0, Z>), gr, bl, 0, s, g, op, omega, B);
  else
    MG_LAUNCH((k_smooth<T, D, K, SM_RB1, Z>), gr, bl, 0, s, g, op, omega, B);
}

template <typename T, int K, bool Z>
static void launch_sweep3_smooth(const Geo& g, const StencilParams<T>& op, int kind, T omega,
                                 const Batch& B, hipStream_t s) {
  if (kind == SM_JACOBI)
    launch_sweep3<T, K, SM_JACOBI, Z, false>(g, op, omega, B, s);
  else if (kind == SM_RB0)
    launch_sweep3<T, K, SM_RB0, Z, false>(g, op, omega, B, s);
  else
    launch_sweep3<T, K, SM_RB1, Z, false>(g, op, omega, B, s);
}

// red-black half-sweeps with a colour-split iterate (constant-coefficient
// and mass-shifted kinds)
template <typename T, int K, int M>
static void launch_sweep3_split(const Geo& g, const StencilParams<T>& op, bool zero, int xl,
                                const Batch& B, hipStream_t s) {
  if (xl == XL_TO_SPLIT) {
    if (zero)
      launch_sweep3<T, K, M, true, false, XL_TO_SPLIT>(g, op, T(0), B, s);
    else
      launch_sweep3<T, K, M, false, false, XL_TO_SPLIT>(g, op, T(0), B, s);
  } else if (xl == XL_SPLIT) {
    launch_sweep3<T, K, M, false, false, XL_SPLIT>(g, op, T(0), B, s);
  } else {
    launch_sweep3<T, K, M, false, false, XL_TO_NATURAL>(g, op, T(0), B, s);
  }
}

bool use_split_x(const Geo& g) { return use_sweep3(g); }

template <typename T>
void launch_resid_restrict(const Geo& g, const StencilParams<T>& op, bool xin, const Batch& B,
                           hipStream_t s) {
  const int m = g.n - 1, mc = (g.n >> 1) - 1;
  // coarse planes per block: half the fine planes of a k_sweep3 block, and
  // in FP64 at most 512 blocks per launch (about 110 VGPRs: at most three
  // of these 5-wave blocks fit on a CU, two per CU measured fastest, 4%
  // faster 256^3 solves than four per CU in two rounds)
  int kzc = std::max(1, sweep3_kz(m, (int)sizeof(T)) / 2);
  if (sizeof(T) == 8) {
    const long xy = (long)cdiv(m, SW_TX) * cdiv(mc, 2) * B.count;
    while (kzc < mc && xy * (long)cdiv(mc, kzc) > 512) ++kzc;
  }
  const int nzc = (int)cdiv(mc, kzc);
  const dim3 gr(cdiv(m, SW_TX), cdiv(mc, 2), (unsigned)(nzc * B.count)), bl(64, RR_TY);
  auto go = [&](auto kc, auto xc) {
    constexpr int K = decltype(kc)::value;
    constexpr bool X = decltype(xc)::value;
    MG_LAUNCH((k_resid_restrict3<T, K, X>), gr, bl, 0, s, g, op, kzc, nzc,
              sweep3_remap(), B);
  };
  using MassK = std::integral_constant<int, OP_MASS>;
  using ConstK = std::integral_constant<int, OP_CONST>;
  if (op.kind == OP_MASS) {
    if (xin) go(MassK{}, std::true_type{});
    else go(MassK{}, std::false_type{});
  } else {
    if (xin) go(ConstK{}, std::true_type{});
    else go(ConstK{}, std::false_type{});
  }
}

int resid_restrict_xcols(const Geo& gf) { return ((gf.n >> 1) - 1) / 64; }

template <typename T>
void launch_restrict_xcols(const Geo& gf, const Batch& B, hipStream_t s) {
  const int mc = (gf.n >> 1) - 1, ncols = resid_restrict_xcols(gf);
  if (ncols == 0) return;
  const long total = (long)mc * mc * ncols;
  MG_LAUNCH((k_restrict_xcols<T>), dim3((unsigned)cdiv(total, 256), B.count), dim3(256),
            0, s, gf, ncols, B);
}

namespace {
// The last FP32 smoothing step of a refinement cycle with the refinement
// update fused (IRU): natural output (xl 0) or split input (xl 3).
template <typename T>
void launch_sweep3_iru(const Geo& g, const StencilParams<T>& op, int kind, T omega, int xl,
                       const Batch& B, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    with_kind3(op.kind, [&](auto kc) {
      constexpr int K = decltype(kc)::value;
      if (xl == XL_TO_NATURAL) {
        if (kind == SM_RB0)
          launch_sweep3<T, K, SM_RB0, false, false, XL_TO_NATURAL, true>(g, op, omega, B, s);
        else
          launch_sweep3<T, K, SM_RB1, false, false, XL_TO_NATURAL, true>(g, op, omega, B, s);
      } else {
        if (kind == SM_RB0)
          launch_sweep3<T, K, SM_RB0, false, false, 0, true>(g, op, omega, B, s);
        else if (kind == SM_RB1)
          launch_sweep3<T, K, SM_RB1, false, false, 0, true>(g, op, omega, B, s);
        else
          launch_sweep3<T, K, SM_JACOBI, false, false, 0, true>(g, op, omega, B, s);
      }
    });
  }
}
}  // namespace

template <typename T>
void launch_smooth(const Geo& g, const StencilParams<T>& op, int kind, bool zero, T omega,
                   const Batch& B, hipStream_t s, int xl, bool iru) {
  if (iru) {
    launch_sweep3_iru<T>(g, op, kind, omega, xl, B, s);
    return;
  }
  if (xl != XL_NATURAL) {
    // (the runtime splits iterates only for red-black on k_sweep3 levels
    // of the constant-coefficient and mass-shifted kinds)
    if (op.kind == OP_MASS) {
      if (kind == SM_RB0)
        launch_sweep3_split<T, OP_MASS, SM_RB0>(g, op, zero, xl, B, s);
      else
        launch_sweep3_split<T, OP_MASS, SM_RB1>(g, op, zero, xl, B, s);
    } else {
      if (kind == SM_RB0)
        launch_sweep3_split<T, OP_CONST, SM_RB0>(g, op, zero, xl, B, s);
      else
        launch_sweep3_split<T, OP_CONST, SM_RB1>(g, op, zero, xl, B, s);
    }
    return;
  }
  if (kind >= SM_GS0) {
    const dim3 gr = node_grid(g, B.count), bl(BX, BY);
#define L_GS(D, K) \
  MG_LAUNCH((k_smooth_gs<T, D, K>), gr, bl, 0, s, g, op, kind - SM_GS0, B)
    DISPATCH_DIM_KIND(g.dim, op.kind, L_GS);
#undef L_GS
    return;
  }
  if (use_sweep3(g)) {
    with_kind3(op.kind, [&](auto k) {
      constexpr int K = decltype(k)::value;
      if (zero)
        launch_sweep3_smooth<T, K, true>(g, op, kind, omega, B, s);
      else
        launch_sweep3_smooth<T, K, false>(g, op, kind, omega, B, s);
    });
    return;
  }
#define L_SM(D, K)                                                       \
  do {                                                                   \
    if (zero)                                                            \
      launch_smooth_k<T, D, K, true>(g, op, kind, omega, B, s);          \
    else                                                                 \
      launch_smooth_k<T, D, K, false>(g, op, kind, omega, B, s);         \
  } while (0)
  DISPATCH_DIM_KIND(g.dim, op.kind, L_SM);
#undef L_SM
}

bool pair_sweeps(const Geo& g) { return use_sweep3(g); }

template <typename T>
void launch_smooth_prolong(const Geo& g, const StencilParams<T>& op, int kind, T omega,
                           const Batch& B, hipStream_t s, int xl) {
  int kz, nzc;
  const dim3 gr = sweep3_grid(g, B.count, &kz, &nzc, (int)sizeof(T));
  const dim3 bl(64, SW_TY);
  const int rm = sweep3_remap();
  if (xl == XL_TO_SPLIT || xl == XL_SPLIT_BOTH) {
    // (red-black on split-iterate levels: constant-coefficient and
    // mass-shifted kinds; the iterate read natural or split)
#define L_SPX(K, M, X)                                                                     \
  MG_LAUNCH((k_sweep3<T, K, M, false, false, true, X>), gr, bl, 0, s, g, op, omega, kz,          \
            nzc, rm, B)
#define L_SPX_X(K, M)                                                      \
  do {                                                                     \
    if (xl == XL_TO_SPLIT) L_SPX(K, M, XL_TO_SPLIT); else L_SPX(K, M, XL_SPLIT_BOTH); \
  } while (0)
    if (op.kind == OP_MASS) {
      if (kind == SM_RB0) L_SPX_X(OP_MASS, SM_RB0); else L_SPX_X(OP_MASS, SM_RB1);
    } else {
      if (kind == SM_RB0) L_SPX_X(OP_CONST, SM_RB0); else L_SPX_X(OP_CONST, SM_RB1);
    }
#undef L_SPX_X
#undef L_SPX
    return;
  }
#define L_SP(K, M) \
  MG_LAUNCH((k_sweep3<T, K, M, false, false, true>), gr, bl, 0, s, g, op, omega, kz, nzc, rm, B)
#define L_SP_K(K)                                          \
  do {                                                     \
    if (kind == SM_JACOBI) L_SP(K, SM_JACOBI);             \
    else if (kind == SM_RB0) L_SP(K, SM_RB0);              \
    else L_SP(K, SM_RB1);                                  \
  } while (0)
  if (op.kind == OP_KAPPA)
    L_SP_K(OP_KAPPA);
  else if (op.kind == OP_MASS)
    L_SP_K(OP_MASS);
  else
    L_SP_K(OP_CONST);
#undef L_SP_K
#undef L_SP
}

template <typename T>
void launch_smooth_pair(const Geo& g, const StencilParams<T>& op, int first, bool zero,
                        const Batch& B, hipStream_t s) {
  int kz, nzc;
  const dim3 gr = sweep3_grid(g, B.count, &kz, &nzc, (int)sizeof(T));
  const dim3 bl(64, SW_TY);
  const int rm = sweep3_remap();
#define L_PAIR(K, CA, Z) \
  MG_LAUNCH((k_sweep3_pair<T, K, CA, Z>), gr, bl, 0, s, g, op, kz, nzc, rm, B)
#define L_PAIR_K(K)                                  \
  do {                                               \
    if (first == SM_RB0) {                           \
      if (zero) L_PAIR(K, 0, true); else L_PAIR(K, 0, false); \
    } else {                                         \
      if (zero) L_PAIR(K, 1, true); else L_PAIR(K, 1, false); \
    }                                                \
  } while (0)
  // (the runtime pairs half-sweeps only for OP_CONST and OP_KAPPA levels)
  if (op.kind == OP_KAPPA)
    L_PAIR_K(OP_KAPPA);
  else
    L_PAIR_K(OP_CONST);
#undef L_PAIR_K
#undef L_PAIR
}

template <typename T>
void launch_head(const Geo& g, const StencilParams<T>& op, int kind, T omega, const Batch& B,
                 hipStream_t s, int xl) {
  const bool jac = kind == SM_JACOBI;
  if (xl == XL_TO_SPLIT || xl == XL_SPLIT) {
    // (red-black heads on split-iterate levels: constant-coefficient and
    // mass-shifted kinds; the iterate read natural or split)
    if (op.kind == OP_MASS) {
      if (xl == XL_TO_SPLIT)
        launch_sweep3<T, OP_MASS, SW_HEAD_RB0, false, true, XL_TO_SPLIT>(g, op, omega, B, s);
      else
        launch_sweep3<T, OP_MASS, SW_HEAD_RB0, false, true, XL_SPLIT>(g, op, omega, B, s);
    } else {
      if (xl == XL_TO_SPLIT)
        launch_sweep3<T, OP_CONST, SW_HEAD_RB0, false, true, XL_TO_SPLIT>(g, op, omega, B, s);
      else
        launch_sweep3<T, OP_CONST, SW_HEAD_RB0, false, true, XL_SPLIT>(g, op, omega, B, s);
    }
    return;
  }
  if (use_sweep3(g)) {
    with_kind3(op.kind, [&](auto k) {
      constexpr int K = decltype(k)::value;
      if (jac)
        launch_sweep3<T, K, SW_HEAD_JAC, false, true>(g, op, omega, B, s);
      else
        launch_sweep3<T, K, SW_HEAD_RB0, false, true>(g, op, omega, B, s);
    });
    return;
  }
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
#define L_HEAD(D, K)                                                                        \
  do {                                                                                      \
    if (jac)                                                                                \
      MG_LAUNCH((k_head<T, D, K, SM_JACOBI>), gr, bl, 0, s, g, op, omega, B);               \
    else                                                                                    \
      MG_LAUNCH((k_head<T, D, K, SM_RB0>), gr, bl, 0, s, g, op, omega, B);                  \
  } while (0)
  DISPATCH_DIM_KIND(g.dim, op.kind, L_HEAD);
#undef L_HEAD
}

template <typename T>
void launch_apply_dot(const Geo& g, const StencilParams<T>& op, const Batch& B, hipStream_t s) {
  if (use_sweep3(g)) {
    with_kind3(op.kind, [&](auto k) {
      launch_sweep3<T, decltype(k)::value, SW_APPLY, false, true>(g, op, T(0), B, s);
    });
    return;
  }
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
#define L_AD(D, K) MG_LAUNCH((k_apply_dot<T, D, K>), gr, bl, 0, s, g, op, B)
  DISPATCH_DIM_KIND(g.dim, op.kind, L_AD);
#undef L_AD
}

void launch_cn_rhs(const Geo& g, const CnWeights& w, const double* u, double* guess,
                   const double* g0, const double* g1, const double* F, double* b,
                   hipStream_t s) {
  if (use_sweep3(g)) {
    // the interior part with the operator Wb (face-coupled constant kind),
    // then the boundary terms on the layer next to the boundary
    StencilParams<double> op{OP_MASS, w.wb[0], w.wb[2], w.wb[3], 0.0, w.wb[1]};
    Batch B{};
    B.count = 1;
    B.it[0].a = u;
    B.it[0].b = F ? F : u;  // without F: cf = 0 and any readable array
    B.it[0].c = b;
    B.it[0].e = guess;
    launch_sweep3<double, OP_MASS, SW_CN, false, false>(g, op, F ? w.cf : 0.0, B, s);
    const long m = g.n - 1;
    const long total = 2 * m * m + 2 * m * (m - 2) + 2 * (m - 2) * (m - 2);
    MG_LAUNCH(k_cn_bnd, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g, w,
              u, g0, g1, b);
    return;
  }
  const dim3 gr = node_grid(g, 1), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH(k_cn_rhs<2>, gr, bl, 0, s, g, w, u, guess, g0, g1, F, b);
  else
    MG_LAUNCH(k_cn_rhs<3>, gr, bl, 0, s, g, w, u, guess, g0, g1, F, b);
}

void launch_cn_rhs_nodes(const Geo& g, const CnWeights& w, const double* u, const double* g0,
                         double* b, hipStream_t s) {
  const dim3 gr = node_grid(g, 1), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH(k_cn_rhs<2>, gr, bl, 0, s, g, w, u, nullptr, g0, nullptr, nullptr, b);
  else
    MG_LAUNCH(k_cn_rhs<3>, gr, bl, 0, s, g, w, u, nullptr, g0, nullptr, nullptr, b);
}

void launch_zero_boundary(const Geo& g, double* v, hipStream_t s) {
  const long N1 = g.n + 1;
  const long total = 2L * g.dim * (g.dim == 3 ? N1 * N1 : N1);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (g.dim == 2)
    MG_LAUNCH(k_zero_boundary<2>, dim3(blocks), dim3(256), 0, s, g, v);
  else
    MG_LAUNCH(k_zero_boundary<3>, dim3(blocks), dim3(256), 0, s, g, v);
}

template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(gc, B.count), bl(BX, BY);
  if (gf.dim == 2)
    MG_LAUNCH((k_restrict<T, 2>), gr, bl, 0, s, gf, gc, B);
  else
    MG_LAUNCH((k_restrict<T, 3>), gr, bl, 0, s, gf, gc, B);
}

// Fine planes per thread of the z-marching 3D prolongation: 1 (one thread
// per node), 2, 4 or 8.  (A tuning build reads MG_PROLONG_PZ.)
int prolong_pz(const Geo& gf) {
  if (gf.dim != 3) return 1;
#ifdef MG_TUNING_KNOBS
  static const int env = [] {
    const char* v = std::getenv("MG_PROLONG_PZ");
    const int z = v ? std::atoi(v) : 0;
    return z == 1 || z == 2 || z == 4 || z == 8 ? z : 0;
  }();
  if (env > 0) return env;
#endif
  const int m = gf.n - 1;
  return m >= 191 ? 8 : m >= 95 ? 4 : m >= 47 ? 2 : 1;
}

template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s) {
  const int pz = prolong_pz(gf);
  if (pz > 1) {
    const long m = gf.n - 1, chunks = cdiv(m, pz);
    const dim3 gr(cdiv(m, BX), cdiv(m, BY), (unsigned)(chunks * B.count)), bl(BX, BY);
    if (pz == 2)
      MG_LAUNCH((k_prolong_add_z<T, 2>), gr, bl, 0, s, gf, gc, B, (int)chunks);
    else if (pz == 4)
      MG_LAUNCH((k_prolong_add_z<T, 4>), gr, bl, 0, s, gf, gc, B, (int)chunks);
    else
      MG_LAUNCH((k_prolong_add_z<T, 8>), gr, bl, 0, s, gf, gc, B, (int)chunks);
    return;
  }
  const dim3 gr = node_grid(gf, B.count), bl(BX, BY);
  if (gf.dim == 2)
    MG_LAUNCH((k_prolong_add<T, 2>), gr, bl, 0, s, gf, gc, B);
  else
    MG_LAUNCH((k_prolong_add<T, 3>), gr, bl, 0, s, gf, gc, B);
}

template <typename T>
void launch_coarse_solve(const Geo& gc, int m, const Batch& B, hipStream_t s) {
  MG_LAUNCH((k_coarse_solve<T>), dim3(B.count), dim3(256), 0, s, gc, m, B);
}

template <typename T>
void launch_norm2_partial(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH((k_norm2_partial<T, 2>), gr, bl, 0, s, g, B);
  else
    MG_LAUNCH((k_norm2_partial<T, 3>), gr, bl, 0, s, g, B);
}

void launch_split_norm(const Geo& g, const double* src, double* dst, long lay,
                       double* partials, hipStream_t s) {
  Batch B{};
  B.count = 1;
  B.it[0].a = src;
  B.it[0].c = dst;
  B.it[0].lay = lay;
  B.it[0].partials = partials;
  const dim3 gr = node_grid(g, 1), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH(k_split_norm<2>, gr, bl, 0, s, g, B);
  else
    MG_LAUNCH(k_split_norm<3>, gr, bl, 0, s, g, B);
}

void launch_reduce_final(long count, const Batch& B, hipStream_t s) {
  MG_LAUNCH(k_reduce_final, dim3(B.count), dim3(RED_THREADS), 0, s, count, B);
}

void launch_scale_cast(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH(k_scale_cast<2>, gr, bl, 0, s, g, B);
  else
    MG_LAUNCH(k_scale_cast<3>, gr, bl, 0, s, g, B);
}

void launch_ir_update(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    MG_LAUNCH(k_ir_update<2>, gr, bl, 0, s, g, B);
  else
    MG_LAUNCH(k_ir_update<3>, gr, bl, 0, s, g, B);
}

template <typename T, int D, int K>
static void launch_tail_k(int lds_bytes, const Batch& B, hipStream_t s) {
  static const bool attr = [] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<T, D, K>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               kTailLdsBytes) == hipSuccess;
  }();
  (void)attr;
  MG_LAUNCH((k_tail<T, D, K>), dim3(B.count), dim3(TAIL_THREADS), lds_bytes, s, B);
}

template <typename T>
void launch_tail(int dim, int kind, int lds_bytes, const Batch& B, hipStream_t s) {
#define L_TAIL(D, K) launch_tail_k<T, D, K>(lds_bytes, B, s)
  DISPATCH_DIM_KIND(dim, kind, L_TAIL);
#undef L_TAIL
}

template <int D, int K>
static void launch_tail_solve_k(int lds_bytes, const Batch& B, double tol, int max_iter,
                                hipStream_t s) {
  static const bool attr = [] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail_solve<D, K>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               kTailLdsBytes) == hipSuccess;
  }();
  (void)attr;
  MG_LAUNCH((k_tail_solve<D, K>), dim3(B.count), dim3(TAIL_THREADS), lds_bytes, s, B,
            tol, max_iter);
}

void launch_tail_solve(int dim, int kind, int lds_bytes, const Batch& B, double tol, int max_iter,
                       hipStream_t s) {
#define L_TSOLVE(D, K) launch_tail_solve_k<D, K>(lds_bytes, B, tol, max_iter, s)
  DISPATCH_DIM_KIND(dim, kind, L_TSOLVE);
#undef L_TSOLVE
}

template <typename T>
void launch_unsplit(const Geo& g, const Batch& B, hipStream_t s) {
  const unsigned bx = (unsigned)std::min<long>((g.nodes + 255) / 256, 8192);
  MG_LAUNCH(k_unsplit<T>, dim3(bx, B.count), dim3(256), 0, s, g.nodes, B);
}

void launch_kappa_coarsen(int dim, int nf, const double* kf, double* kc, hipStream_t s) {
  const int nc = nf / 2;
  const long total = dim == 3 ? (long)nc * nc * nc : (long)nc * nc;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (dim == 2)
    MG_LAUNCH(k_kappa_coarsen<2>, dim3(blocks), dim3(256), 0, s, nf, kf, kc);
  else
    MG_LAUNCH(k_kappa_coarsen<3>, dim3(blocks), dim3(256), 0, s, nf, kf, kc);
}

void launch_cast_f32(const double* a, float* b, long count, hipStream_t s) {
  MG_LAUNCH(k_cast_f32, dim3(flat_blocks(count)), dim3(256), 0, s, a, b, count);
}

void launch_count_bad_kappa(const double* k, long count, int* nonpos, int* nonfinite,
                            hipStream_t s) {
  MG_LAUNCH(k_count_bad_kappa, dim3(flat_blocks(count)), dim3(256), 0, s, k, count,
            nonpos, nonfinite);
}

#define INST(T)                                                                             \
  template void launch_fill<T>(T*, long, T, hipStream_t);                                   \
  template void launch_copy<T>(const T*, T*, long, hipStream_t);                            \
  template void launch_residual<T>(const Geo&, const StencilParams<T>&, bool, const Batch&, \
                                   hipStream_t, int, bool);                                 \
  template void launch_unsplit<T>(const Geo&, const Batch&, hipStream_t);                   \
  template void launch_smooth_pair<T>(const Geo&, const StencilParams<T>&, int, bool,      \
                                      const Batch&, hipStream_t);                           \
  template void launch_smooth_prolong<T>(const Geo&, const StencilParams<T>&, int, T,       \
                                         const Batch&, hipStream_t, int);                   \
  template void launch_smooth<T>(const Geo&, const StencilParams<T>&, int, bool, T,         \
                                 const Batch&, hipStream_t, int, bool);                     \
  template void launch_head<T>(const Geo&, const StencilParams<T>&, int, T, const Batch&,   \
                               hipStream_t, int);                                           \
  template void launch_apply_dot<T>(const Geo&, const StencilParams<T>&, const Batch&,      \
                                    hipStream_t);                                           \
  template void launch_restrict<T>(const Geo&, const Geo&, const Batch&, hipStream_t);      \
  template void launch_resid_restrict<T>(const Geo&, const StencilParams<T>&, bool,         \
                                         const Batch&, hipStream_t);                        \
  template void launch_restrict_xcols<T>(const Geo&, const Batch&, hipStream_t);            \
  template void launch_prolong_add<T>(const Geo&, const Geo&, const Batch&, hipStream_t);   \
  template void launch_coarse_solve<T>(const Geo&, int, const Batch&, hipStream_t);         \
  template void launch_norm2_partial<T>(const Geo&, const Batch&, hipStream_t);             \
  template void launch_tail<T>(int, int, int, const Batch&, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace mg
