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

// 3D, kappa = 1: 8h/3 centre, -h/6 on the 12 edge neighbours, -h/12 on the
// 8 corners, 0 on the 6 face neighbours.
template <typename T>
struct Apply<T, 3, OP_CONST> {
  __device__ static void at(const StencilParams<T>& op, const T*, const DGeo& g,
                            const T* __restrict__ x, long p, int, int, int, T& ax, T& dg) {
    const long sy = g.sy, sz = g.sz;
    T e = ((x[p - 1 - sy] + x[p + 1 - sy]) + (x[p - 1 + sy] + x[p + 1 + sy])) +
          ((x[p - 1 - sz] + x[p + 1 - sz]) + (x[p - 1 + sz] + x[p + 1 + sz])) +
          ((x[p - sy - sz] + x[p + sy - sz]) + (x[p - sy + sz] + x[p + sy + sz]));
    T c = ((x[p - 1 - sy - sz] + x[p + 1 - sy - sz]) + (x[p - 1 + sy - sz] + x[p + 1 + sy - sz])) +
          ((x[p - 1 - sy + sz] + x[p + 1 - sy + sz]) + (x[p - 1 + sy + sz] + x[p + 1 + sy + sz]));
    ax = op.wc * x[p] + op.w1 * e + op.w2 * c;
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

// 3D, kappa per cell.  Cell (a, b, c) of the eight around p (side
// sx = 2a-1, sy = 2b-1, sz = 2c-1) contributes
//   kappa_abc * h/12 * (4 x_p - x_{p+sx+sy} - x_{p+sx+sz} - x_{p+sy+sz}
//                       - x_{p+sx+sy+sz});
// face neighbours have element weight 0.
template <typename T>
struct Apply<T, 3, OP_KAPPA> {
  __device__ static void at(const StencilParams<T>& op, const T* __restrict__ kappa,
                            const DGeo& g, const T* __restrict__ x, long p, int i, int j, int k,
                            T& ax, T& dg) {
    const long sy = g.sy, sz = g.sz;
    const long n = g.n, cz = (long)g.n * g.n;
    const T* kp = kappa + (i - 1) + n * (j - 1) + cz * (k - 1);
    const T xp = x[p];
    T acc = 0, ks = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const T kc = kp[a + n * b + cz * c];
          const long dx = a ? 1 : -1;
          const long dy = b ? sy : -sy;
          const long dz = c ? sz : -sz;
          acc += kc * (T(4) * xp - x[p + dx + dy] - x[p + dx + dz] - x[p + dy + dz] -
                       x[p + dx + dy + dz]);
          ks += kc;
        }
      }
    }
    ax = op.s * acc;
    dg = op.s * T(4) * ks;
  }
  __device__ static T diag(const StencilParams<T>& op, const T* __restrict__ kappa,
                           const DGeo& g, int i, int j, int k) {
    const long n = g.n, cz = (long)g.n * g.n;
    const T* kp = kappa + (i - 1) + n * (j - 1) + cz * (k - 1);
    T ks = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) ks += kp[a + n * b + cz * c];
    return op.s * T(4) * ks;
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

template <typename T, int DIM, int KIND>
__device__ __forceinline__ T residual_node(const StencilParams<T>& op, const T* kappa,
                                           const DGeo& g, const T* __restrict__ x,
                                           const T* __restrict__ b, long p, int i, int j,
                                           int k) {
  T ax, dg;
  Apply<T, DIM, KIND>::at(op, kappa, g, x, p, i, j, k, ax, dg);
  return b[p] - ax;
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
  T acc = 0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    T pl = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const long o = pf + dy * sy + dz * sz;
      const T row = r[o] + h * (r[o - 1] + r[o + 1]);
      pl += (dy == 0 ? T(1) : h) * row;
    }
    acc += (dz == 0 ? T(1) : h) * pl;
  }
  return acc;
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

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, Batch B) {
  NODE_INDEX(DIM, gc)
  if (!inside) return;
  ((T*)I.c)[p] = restrict_node<T, DIM>(dgeo(gf), (const T*)I.a, i, j, k);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_add(Geo gf, Geo gc, Batch B) {
  NODE_INDEX(DIM, gf)
  if (!inside) return;
  T* x = (T*)I.c;
  x[p] += prolong_node<T, DIM>(dgeo(gc), (const T*)I.a, i, j, k);
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

// b32 = float(r / ||r||) on the unknowns, ||r||^2 read from device memory.
template <int DIM>
__global__ __launch_bounds__(256) void k_scale_cast(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside) return;
  const double s = sqrt(*I.scal);
  ((float*)I.c)[p] = (float)(((const double*)I.a)[p] / s);
}

// u += ||r|| * double(c) on the unknowns.
template <int DIM>
__global__ __launch_bounds__(256) void k_ir_update(Geo g, Batch B) {
  NODE_INDEX(DIM, g)
  if (!inside) return;
  const double s = sqrt(*I.scal);
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

template <typename T, int DIM, int KIND>
__device__ void tail_smooth(const TailDesc<T>& D, int l, bool pre, T** cur, T** spr,
                            bool* zero, const T* b) {
  const TailLevel<T>& Lv = D.lv[l];
  const DGeo g = dgeo(DIM, Lv.n);
  const StencilParams<T> op{KIND, Lv.wc, Lv.w1, Lv.w2, Lv.s};
  const int nu = pre ? D.nu_pre : D.nu_post;
  for (int it = 0; it < nu; ++it) {
    const int nsteps = D.smoother == 0 ? 1 : 2;
    for (int h = 0; h < nsteps; ++h) {
      const int ks = D.smoother == 0 ? SM_JACOBI : ((h == 0) == pre ? SM_RB0 : SM_RB1);
      const T* xin = *zero ? nullptr : *cur;
      T* xout = *spr;
      for_unknowns<DIM>(Lv.n, g, [&](long p, int i, int j, int k) {
        xout[p] = smooth_node<T, DIM, KIND>(op, Lv.kappa, g, ks, xin, b, D.omega, p, i, j, k);
      });
      __syncthreads();
      T* tmp = *cur;
      *cur = *spr;
      *spr = tmp;
      *zero = false;
    }
  }
}

template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(Batch B) {
  __shared__ double ysh[kCoarseMaxUnknowns];
  const Item& I = B.it[blockIdx.x];
  const TailDesc<T>& D = *(const TailDesc<T>*)I.a;
  const int nl = D.nlev;
  T* cur[kTailMaxLevels];
  T* spr[kTailMaxLevels];
  const T* bb[kTailMaxLevels];
  for (int l = 0; l < nl; ++l) {
    cur[l] = l == 0 ? (T*)I.c : D.lv[l].x;
    spr[l] = D.lv[l].t;
    bb[l] = l == 0 ? (const T*)I.b : D.lv[l].b;
  }
  for (int l = 0; l + 1 < nl; ++l) {
    const TailLevel<T>& Lv = D.lv[l];
    const DGeo g = dgeo(DIM, Lv.n);
    bool zero = (l > 0) || I.flag;
    tail_smooth<T, DIM, KIND>(D, l, true, &cur[l], &spr[l], &zero, bb[l]);
    T* x = cur[l];
    if (zero) {
      for_unknowns<DIM>(Lv.n, g, [&](long p, int, int, int) { x[p] = T(0); });
      __syncthreads();
    }
    const StencilParams<T> op{KIND, Lv.wc, Lv.w1, Lv.w2, Lv.s};
    T* r = Lv.r;
    const T* b = bb[l];
    for_unknowns<DIM>(Lv.n, g, [&](long p, int i, int j, int k) {
      r[p] = residual_node<T, DIM, KIND>(op, Lv.kappa, g, x, b, p, i, j, k);
    });
    __syncthreads();
    const DGeo gc = dgeo(DIM, D.lv[l + 1].n);
    T* bc = D.lv[l + 1].b;
    for_unknowns<DIM>(D.lv[l + 1].n, gc, [&](long p, int i, int j, int k) {
      bc[p] = restrict_node<T, DIM>(g, r, i, j, k);
    });
    __syncthreads();
  }
  cholesky_solve_block<T>(DIM, D.lv[nl - 1].n, D.L, D.m, bb[nl - 1], cur[nl - 1], ysh);
  for (int l = nl - 2; l >= 0; --l) {
    const DGeo g = dgeo(DIM, D.lv[l].n);
    const DGeo gc = dgeo(DIM, D.lv[l + 1].n);
    T* x = cur[l];
    const T* e = cur[l + 1];
    for_unknowns<DIM>(D.lv[l].n, g, [&](long p, int i, int j, int k) {
      x[p] += prolong_node<T, DIM>(gc, e, i, j, k);
    });
    __syncthreads();
    bool zero = false;
    tail_smooth<T, DIM, KIND>(D, l, false, &cur[l], &spr[l], &zero, bb[l]);
  }
  if (cur[0] != (T*)I.c) {
    T* out = (T*)I.c;
    const T* src = cur[0];
    const DGeo g = dgeo(DIM, D.lv[0].n);
    for_unknowns<DIM>(D.lv[0].n, g, [&](long p, int, int, int) { out[p] = src[p]; });
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
long grid_blocks(const Geo& g) {
  dim3 gr = node_grid(g, 1);
  return (long)gr.x * gr.y * gr.z;
}

template <typename T>
void launch_fill(T* v, long count, T val, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, dim3(flat_blocks(count)), dim3(256), 0, s, v, count, val);
}
template <typename T>
void launch_copy(const T* a, T* b, long count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(flat_blocks(count)), dim3(256), 0, s, a, b, count);
}

#define DISPATCH_DIM_KIND(dim, kind, MACRO)                                      \
  do {                                                                           \
    if ((dim) == 2) {                                                            \
      if ((kind) == OP_CONST) MACRO(2, OP_CONST); else MACRO(2, OP_KAPPA);       \
    } else {                                                                     \
      if ((kind) == OP_CONST) MACRO(3, OP_CONST); else MACRO(3, OP_KAPPA);       \
    }                                                                            \
  } while (0)

template <typename T>
void launch_residual(const Geo& g, const StencilParams<T>& op, bool norm, const Batch& B,
                     hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
#define L_RES(D, K)                                                                   \
  do {                                                                                \
    if (norm)                                                                         \
      hipLaunchKernelGGL((k_residual<T, D, K, true>), gr, bl, 0, s, g, op, B);        \
    else                                                                              \
      hipLaunchKernelGGL((k_residual<T, D, K, false>), gr, bl, 0, s, g, op, B);       \
  } while (0)
  DISPATCH_DIM_KIND(g.dim, op.kind, L_RES);
#undef L_RES
}

template <typename T, int D, int K, bool Z>
static void launch_smooth_k(const Geo& g, const StencilParams<T>& op, int kind, T omega,
                            const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (kind == SM_JACOBI)
    hipLaunchKernelGGL((k_smooth<T, D, K, SM_JACOBI, Z>), gr, bl, 0, s, g, op, omega, B);
  else if (kind == SM_RB0)
    hipLaunchKernelGGL((k_smooth<T, D, K, SM_RB0, Z>), gr, bl, 0, s, g, op, omega, B);
  else
    hipLaunchKernelGGL((k_smooth<T, D, K, SM_RB1, Z>), gr, bl, 0, s, g, op, omega, B);
}

template <typename T>
void launch_smooth(const Geo& g, const StencilParams<T>& op, int kind, bool zero, T omega,
                   const Batch& B, hipStream_t s) {
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

template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(gc, B.count), bl(BX, BY);
  if (gf.dim == 2)
    hipLaunchKernelGGL((k_restrict<T, 2>), gr, bl, 0, s, gf, gc, B);
  else
    hipLaunchKernelGGL((k_restrict<T, 3>), gr, bl, 0, s, gf, gc, B);
}

template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(gf, B.count), bl(BX, BY);
  if (gf.dim == 2)
    hipLaunchKernelGGL((k_prolong_add<T, 2>), gr, bl, 0, s, gf, gc, B);
  else
    hipLaunchKernelGGL((k_prolong_add<T, 3>), gr, bl, 0, s, gf, gc, B);
}

template <typename T>
void launch_coarse_solve(const Geo& gc, int m, const Batch& B, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(B.count), dim3(256), 0, s, gc, m, B);
}

template <typename T>
void launch_norm2_partial(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL((k_norm2_partial<T, 2>), gr, bl, 0, s, g, B);
  else
    hipLaunchKernelGGL((k_norm2_partial<T, 3>), gr, bl, 0, s, g, B);
}

void launch_reduce_final(long count, const Batch& B, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(B.count), dim3(RED_THREADS), 0, s, count, B);
}

void launch_scale_cast(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_scale_cast<2>, gr, bl, 0, s, g, B);
  else
    hipLaunchKernelGGL(k_scale_cast<3>, gr, bl, 0, s, g, B);
}

void launch_ir_update(const Geo& g, const Batch& B, hipStream_t s) {
  const dim3 gr = node_grid(g, B.count), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_ir_update<2>, gr, bl, 0, s, g, B);
  else
    hipLaunchKernelGGL(k_ir_update<3>, gr, bl, 0, s, g, B);
}

template <typename T>
void launch_tail(int dim, int kind, const Batch& B, hipStream_t s) {
#define L_TAIL(D, K) \
  hipLaunchKernelGGL((k_tail<T, D, K>), dim3(B.count), dim3(TAIL_THREADS), 0, s, B)
  DISPATCH_DIM_KIND(dim, kind, L_TAIL);
#undef L_TAIL
}

void launch_kappa_coarsen(int dim, int nf, const double* kf, double* kc, hipStream_t s) {
  const int nc = nf / 2;
  const long total = dim == 3 ? (long)nc * nc * nc : (long)nc * nc;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (dim == 2)
    hipLaunchKernelGGL(k_kappa_coarsen<2>, dim3(blocks), dim3(256), 0, s, nf, kf, kc);
  else
    hipLaunchKernelGGL(k_kappa_coarsen<3>, dim3(blocks), dim3(256), 0, s, nf, kf, kc);
}

void launch_cast_f32(const double* a, float* b, long count, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f32, dim3(flat_blocks(count)), dim3(256), 0, s, a, b, count);
}

void launch_count_bad_kappa(const double* k, long count, int* nonpos, int* nonfinite,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_count_bad_kappa, dim3(flat_blocks(count)), dim3(256), 0, s, k, count,
                     nonpos, nonfinite);
}

#define INST(T)                                                                             \
  template void launch_fill<T>(T*, long, T, hipStream_t);                                   \
  template void launch_copy<T>(const T*, T*, long, hipStream_t);                            \
  template void launch_residual<T>(const Geo&, const StencilParams<T>&, bool, const Batch&, \
                                   hipStream_t);                                            \
  template void launch_smooth<T>(const Geo&, const StencilParams<T>&, int, bool, T,         \
                                 const Batch&, hipStream_t);                                \
  template void launch_restrict<T>(const Geo&, const Geo&, const Batch&, hipStream_t);      \
  template void launch_prolong_add<T>(const Geo&, const Geo&, const Batch&, hipStream_t);   \
  template void launch_coarse_solve<T>(const Geo&, int, const Batch&, hipStream_t);         \
  template void launch_norm2_partial<T>(const Geo&, const Batch&, hipStream_t);             \
  template void launch_tail<T>(int, int, const Batch&, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace mg
