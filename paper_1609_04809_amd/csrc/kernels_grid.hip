// Grid kernels of the Q1 multigrid V-cycle for gfx950: matrix-free operator
// application (residual, smoothers), grid transfers, coarsest solve, norms
// and the iterative-refinement helpers.
//
// Thread layout of the node kernels: a block of 64 x 4 threads covers 64
// consecutive x and 4 consecutive y of one z plane of interior nodes, so one
// wavefront (64 lanes) reads 64 consecutive doubles of a grid row.
#include "mg_internal.h"

namespace mg {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

inline dim3 node_grid(const Geo& g) {
  const long m = g.n - 1;  // interior nodes per direction
  return dim3(cdiv(m, BX), cdiv(m, BY), g.dim == 3 ? (unsigned)m : 1u);
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

__device__ __forceinline__ long block_linear() {
  return blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
}

// ---------------------------------------------------------------------------
// Operator application at one interior node p = (i, j[, k]).
// Returns (A x)_p in ax and the diagonal entry a_pp in dg.
// ---------------------------------------------------------------------------
template <typename T, int DIM, int KIND>
struct Apply;

// 2D, kappa = 1: 8/3 centre, -1/3 for all eight neighbours.
template <typename T>
struct Apply<T, 2, OP_CONST> {
  __device__ static void at(const StencilOp<T>& op, const Geo& g, const T* __restrict__ x,
                            long p, int, int, int, T& ax, T& dg) {
    const long sy = g.sy;
    T f = (x[p - 1] + x[p + 1]) + (x[p - sy] + x[p + sy]);
    T c = (x[p - 1 - sy] + x[p + 1 - sy]) + (x[p - 1 + sy] + x[p + 1 + sy]);
    ax = op.wc * x[p] + op.w1 * f + op.w2 * c;
    dg = op.wc;
  }
  __device__ static T diag(const StencilOp<T>& op, const Geo&, int, int, int) { return op.wc; }
};

// 3D, kappa = 1: 8h/3 centre, -h/6 on the 12 edge neighbours, -h/12 on the
// 8 corners, 0 on the 6 face neighbours.
template <typename T>
struct Apply<T, 3, OP_CONST> {
  __device__ static void at(const StencilOp<T>& op, const Geo& g, const T* __restrict__ x,
                            long p, int, int, int, T& ax, T& dg) {
    const long sy = g.sy, sz = g.sz;
    T e = ((x[p - 1 - sy] + x[p + 1 - sy]) + (x[p - 1 + sy] + x[p + 1 + sy])) +
          ((x[p - 1 - sz] + x[p + 1 - sz]) + (x[p - 1 + sz] + x[p + 1 + sz])) +
          ((x[p - sy - sz] + x[p + sy - sz]) + (x[p - sy + sz] + x[p + sy + sz]));
    T c = ((x[p - 1 - sy - sz] + x[p + 1 - sy - sz]) + (x[p - 1 + sy - sz] + x[p + 1 + sy - sz])) +
          ((x[p - 1 - sy + sz] + x[p + 1 - sy + sz]) + (x[p - 1 + sy + sz] + x[p + 1 + sy + sz]));
    ax = op.wc * x[p] + op.w1 * e + op.w2 * c;
    dg = op.wc;
  }
  __device__ static T diag(const StencilOp<T>& op, const Geo&, int, int, int) { return op.wc; }
};

// 2D, kappa per cell.  Cell (a, b) of the four around p (a, b in {0,1}, on
// the side sx = 2a-1, sy = 2b-1) contributes
//   kappa_ab / 6 * (4 x_p - x_{p+sx} - x_{p+sy} - 2 x_{p+sx+sy}).
template <typename T>
struct Apply<T, 2, OP_KAPPA> {
  __device__ static void at(const StencilOp<T>& op, const Geo& g, const T* __restrict__ x,
                            long p, int i, int j, int, T& ax, T& dg) {
    const long sy = g.sy;
    const long n = g.n;
    const T* kp = op.kappa + (i - 1) + n * (j - 1);
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
  __device__ static T diag(const StencilOp<T>& op, const Geo& g, int i, int j, int) {
    const long n = g.n;
    const T* kp = op.kappa + (i - 1) + n * (j - 1);
    return op.s * T(4) * ((kp[0] + kp[1]) + (kp[n] + kp[n + 1]));
  }
};

// 3D, kappa per cell.  Cell (a, b, c) of the eight around p (side
// sx = 2a-1, sy = 2b-1, sz = 2c-1) contributes
//   kappa_abc * h/12 * (4 x_p - x_{p+sx+sy} - x_{p+sx+sz} - x_{p+sy+sz}
//                       - x_{p+sx+sy+sz});
// face neighbours have element weight 0.
template <typename T>
struct Apply<T, 3, OP_KAPPA> {
  __device__ static void at(const StencilOp<T>& op, const Geo& g, const T* __restrict__ x,
                            long p, int i, int j, int k, T& ax, T& dg) {
    const long sy = g.sy, sz = g.sz;
    const long n = g.n, cz = (long)g.n * g.n;
    const T* kp = op.kappa + (i - 1) + n * (j - 1) + cz * (k - 1);
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
  __device__ static T diag(const StencilOp<T>& op, const Geo& g, int i, int j, int k) {
    const long n = g.n, cz = (long)g.n * g.n;
    const T* kp = op.kappa + (i - 1) + n * (j - 1) + cz * (k - 1);
    T ks = ((kp[0] + kp[1]) + (kp[n] + kp[n + 1])) +
           ((kp[cz] + kp[cz + 1]) + (kp[cz + n] + kp[cz + n + 1]));
    return op.s * T(4) * ks;
  }
};

// ---------------------------------------------------------------------------
// node kernels
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

#define NODE_INDEX(DIM)                                   \
  const int m = g.n - 1;                                  \
  const int i = 1 + blockIdx.x * BX + threadIdx.x;        \
  const int j = 1 + blockIdx.y * BY + threadIdx.y;        \
  const int k = (DIM) == 3 ? 1 + (int)blockIdx.z : 0;     \
  const bool inside = (i <= m) && (j <= m);               \
  const long p = i + j * g.sy + (long)k * g.sz;

// r = b - A x on the unknowns; optional per-block partial sums of r^2.
template <typename T, int DIM, int KIND, bool NORM>
__global__ __launch_bounds__(256) void k_residual(Geo g, StencilOp<T> op,
                                                  const T* __restrict__ x,
                                                  const T* __restrict__ b,
                                                  T* __restrict__ r,
                                                  double* __restrict__ partials) {
  NODE_INDEX(DIM)
  double sq = 0.0;
  if (inside) {
    T ax, dg;
    Apply<T, DIM, KIND>::at(op, g, x, p, i, j, k, ax, dg);
    const T res = b[p] - ax;
    r[p] = res;
    sq = (double)res * (double)res;
  }
  if (NORM) {
    const double t = block_sum(sq);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[block_linear()] = t;
  }
}

// One smoothing step.  KIND_S = SM_JACOBI: every unknown gets
// x + omega (b - A x)/a_pp.  SM_RB0/SM_RB1: unknowns of that colour get
// x + (b - A x)/a_pp, the others keep x.  xin == nullptr means x = 0.
template <typename T, int DIM, int KIND, int KIND_S>
__global__ __launch_bounds__(256) void k_smooth(Geo g, StencilOp<T> op,
                                                const T* __restrict__ xin,
                                                const T* __restrict__ b,
                                                T* __restrict__ xout, T omega) {
  NODE_INDEX(DIM)
  if (!inside) return;
  const int colour = KIND_S == SM_RB1 ? 1 : 0;
  const bool upd = (KIND_S == SM_JACOBI) || (((i + j + k) & 1) == colour);
  T xo;
  if (xin == nullptr) {
    if (upd) {
      const T dg = Apply<T, DIM, KIND>::diag(op, g, i, j, k);
      xo = KIND_S == SM_JACOBI ? omega * (b[p] / dg) : b[p] / dg;
    } else {
      xo = T(0);
    }
  } else if (upd) {
    T ax, dg;
    Apply<T, DIM, KIND>::at(op, g, xin, p, i, j, k, ax, dg);
    const T q = (b[p] - ax) / dg;
    xo = KIND_S == SM_JACOBI ? xin[p] + omega * q : xin[p] + q;
  } else {
    xo = xin[p];
  }
  xout[p] = xo;
}

// Coarse node I (interior of the coarse grid) gathers the fine residual
// around fine node 2I with weights prod_d (o_d == 0 ? 1 : 1/2).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, const T* __restrict__ r,
                                                  T* __restrict__ bc) {
  const Geo& g = gc;
  NODE_INDEX(DIM)
  if (!inside) return;
  const long pf = 2 * i + 2 * j * gf.sy + 2L * k * gf.sz;
  const T h = T(0.5), q = T(0.25);
  T v;
  if (DIM == 2) {
    const long sy = gf.sy;
    v = r[pf] + h * ((r[pf - 1] + r[pf + 1]) + (r[pf - sy] + r[pf + sy])) +
        q * ((r[pf - 1 - sy] + r[pf + 1 - sy]) + (r[pf - 1 + sy] + r[pf + 1 + sy]));
  } else {
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
    v = acc;
  }
  bc[p] = v;
}

// Fine node i gets the multilinear interpolant of the coarse correction:
// per direction an even coordinate has the single parent i/2 (weight 1), an
// odd one the parents (i-1)/2 and (i+1)/2 (weight 1/2 each).  Coarse
// boundary entries of e are read and must be 0.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_add(Geo gf, Geo gc, const T* __restrict__ e,
                                                     T* __restrict__ x) {
  const Geo& g = gf;
  NODE_INDEX(DIM)
  if (!inside) return;
  const int i0 = i >> 1, i1 = (i + 1) >> 1;
  const int j0 = j >> 1, j1 = (j + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1);
  const T wj = (j & 1) ? T(0.5) : T(1);
  T v;
  if (DIM == 2) {
    const long sy = gc.sy;
    T r0 = (i & 1) ? wi * (e[i0 + j0 * sy] + e[i1 + j0 * sy]) : e[i0 + j0 * sy];
    T r1 = (i & 1) ? wi * (e[i0 + j1 * sy] + e[i1 + j1 * sy]) : e[i0 + j1 * sy];
    v = (j & 1) ? wj * (r0 + r1) : r0;
  } else {
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
    v = (k & 1) ? wk * (plane(k0) + plane(k1)) : plane(k0);
  }
  x[p] += v;
}

// Coarsest solve with the dense FP64 Cholesky factor L (row major, m x m):
// gather the unknowns of b, forward substitution L y = b, back substitution
// L^T z = y, scatter z.  One block.
constexpr int COARSE_MAX = kCoarseMaxUnknowns;

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(Geo g, const double* __restrict__ L,
                                                      int m, const T* __restrict__ bc,
                                                      T* __restrict__ xc) {
  __shared__ double y[COARSE_MAX];
  const int t = threadIdx.x;
  const int mi = g.n - 1;
  for (int q = t; q < m; q += blockDim.x) {
    const int qx = q % mi, qy = (q / mi) % mi, qz = g.dim == 3 ? q / (mi * mi) : 0;
    y[q] = (double)bc[(qx + 1) + (qy + 1) * g.sy + (long)(qz + 1) * g.sz];
  }
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    if (t == 0) y[c] = y[c] / L[(long)c * m + c];
    __syncthreads();
    const double yc = y[c];
    for (int q = c + 1 + t; q < m; q += blockDim.x) y[q] -= L[(long)q * m + c] * yc;
    __syncthreads();
  }
  for (int c = m - 1; c >= 0; --c) {
    if (t == 0) y[c] = y[c] / L[(long)c * m + c];
    __syncthreads();
    const double yc = y[c];
    for (int q = t; q < c; q += blockDim.x) y[q] -= L[(long)c * m + q] * yc;
    __syncthreads();
  }
  for (int q = t; q < m; q += blockDim.x) {
    const int qx = q % mi, qy = (q / mi) % mi, qz = g.dim == 3 ? q / (mi * mi) : 0;
    xc[(qx + 1) + (qy + 1) * g.sy + (long)(qz + 1) * g.sz] = (T)y[q];
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_norm2_partial(Geo g, const T* __restrict__ v,
                                                       double* __restrict__ partials) {
  NODE_INDEX(DIM)
  double sq = 0.0;
  if (inside) {
    const double a = (double)v[p];
    sq = a * a;
  }
  const double t = block_sum(sq);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[block_linear()] = t;
}

// Sum partials[0..count) in a fixed order with one block of 64x4 threads.
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partials,
                                                      long count, double* __restrict__ out) {
  const int t = threadIdx.x + BX * threadIdx.y;
  double s = 0.0;
  for (long q = t; q < count; q += 256) s += partials[q];
  const double tot = block_sum(s);
  if (t == 0) *out = tot;
}

// b32 = float(r / ||r||) on the unknowns, ||r||^2 read from device memory.
template <int DIM>
__global__ __launch_bounds__(256) void k_scale_cast(Geo g, const double* __restrict__ r,
                                                    const double* __restrict__ norm2,
                                                    float* __restrict__ b32) {
  NODE_INDEX(DIM)
  if (!inside) return;
  const double s = sqrt(*norm2);
  b32[p] = (float)(r[p] / s);
}

// u += ||r|| * double(c) on the unknowns.
template <int DIM>
__global__ __launch_bounds__(256) void k_ir_update(Geo g, double* __restrict__ u,
                                                   const float* __restrict__ c,
                                                   const double* __restrict__ norm2) {
  NODE_INDEX(DIM)
  if (!inside) return;
  const double s = sqrt(*norm2);
  u[p] = u[p] + s * (double)c[p];
}

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
  dim3 gr = node_grid(g);
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

#define DISPATCH_DIM_KIND(g, op, MACRO)                                   \
  do {                                                                    \
    if ((g).dim == 2) {                                                   \
      if ((op).kind == OP_CONST) MACRO(2, OP_CONST); else MACRO(2, OP_KAPPA); \
    } else {                                                              \
      if ((op).kind == OP_CONST) MACRO(3, OP_CONST); else MACRO(3, OP_KAPPA); \
    }                                                                     \
  } while (0)

template <typename T>
void launch_residual(const Geo& g, const StencilOp<T>& op, const T* x, const T* b, T* r,
                     double* partials, hipStream_t s) {
  const dim3 gr = node_grid(g), bl(BX, BY);
#define L_RES(D, K)                                                                     \
  do {                                                                                  \
    if (partials)                                                                       \
      hipLaunchKernelGGL((k_residual<T, D, K, true>), gr, bl, 0, s, g, op, x, b, r, partials); \
    else                                                                                \
      hipLaunchKernelGGL((k_residual<T, D, K, false>), gr, bl, 0, s, g, op, x, b, r, partials); \
  } while (0)
  DISPATCH_DIM_KIND(g, op, L_RES);
#undef L_RES
}

template <typename T>
void launch_smooth(const Geo& g, const StencilOp<T>& op, int kind, const T* xin, const T* b,
                   T* xout, T omega, hipStream_t s) {
  const dim3 gr = node_grid(g), bl(BX, BY);
#define L_SM(D, K)                                                                          \
  do {                                                                                      \
    if (kind == SM_JACOBI)                                                                  \
      hipLaunchKernelGGL((k_smooth<T, D, K, SM_JACOBI>), gr, bl, 0, s, g, op, xin, b, xout, omega); \
    else if (kind == SM_RB0)                                                                \
      hipLaunchKernelGGL((k_smooth<T, D, K, SM_RB0>), gr, bl, 0, s, g, op, xin, b, xout, omega);    \
    else                                                                                    \
      hipLaunchKernelGGL((k_smooth<T, D, K, SM_RB1>), gr, bl, 0, s, g, op, xin, b, xout, omega);    \
  } while (0)
  DISPATCH_DIM_KIND(g, op, L_SM);
#undef L_SM
}

template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const T* r, T* bc, hipStream_t s) {
  const dim3 gr = node_grid(gc), bl(BX, BY);
  if (gf.dim == 2)
    hipLaunchKernelGGL((k_restrict<T, 2>), gr, bl, 0, s, gf, gc, r, bc);
  else
    hipLaunchKernelGGL((k_restrict<T, 3>), gr, bl, 0, s, gf, gc, r, bc);
}

template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const T* e, T* x, hipStream_t s) {
  const dim3 gr = node_grid(gf), bl(BX, BY);
  if (gf.dim == 2)
    hipLaunchKernelGGL((k_prolong_add<T, 2>), gr, bl, 0, s, gf, gc, e, x);
  else
    hipLaunchKernelGGL((k_prolong_add<T, 3>), gr, bl, 0, s, gf, gc, e, x);
}

template <typename T>
void launch_coarse_solve(const Geo& gc, const double* L, int m, const T* bc, T* xc,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(256), 0, s, gc, L, m, bc, xc);
}

template <typename T>
void launch_norm2_partial(const Geo& g, const T* v, double* partials, hipStream_t s) {
  const dim3 gr = node_grid(g), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL((k_norm2_partial<T, 2>), gr, bl, 0, s, g, v, partials);
  else
    hipLaunchKernelGGL((k_norm2_partial<T, 3>), gr, bl, 0, s, g, v, partials);
}

void launch_reduce_final(const double* partials, long count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BX, BY), 0, s, partials, count, out);
}

void launch_scale_cast(const Geo& g, const double* r, const double* norm2, float* b32,
                       hipStream_t s) {
  const dim3 gr = node_grid(g), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_scale_cast<2>, gr, bl, 0, s, g, r, norm2, b32);
  else
    hipLaunchKernelGGL(k_scale_cast<3>, gr, bl, 0, s, g, r, norm2, b32);
}

void launch_ir_update(const Geo& g, double* u, const float* c, const double* norm2,
                      hipStream_t s) {
  const dim3 gr = node_grid(g), bl(BX, BY);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_ir_update<2>, gr, bl, 0, s, g, u, c, norm2);
  else
    hipLaunchKernelGGL(k_ir_update<3>, gr, bl, 0, s, g, u, c, norm2);
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

#define INST(T)                                                                            \
  template void launch_fill<T>(T*, long, T, hipStream_t);                                  \
  template void launch_copy<T>(const T*, T*, long, hipStream_t);                           \
  template void launch_residual<T>(const Geo&, const StencilOp<T>&, const T*, const T*, T*, \
                                   double*, hipStream_t);                                  \
  template void launch_smooth<T>(const Geo&, const StencilOp<T>&, int, const T*, const T*, \
                                 T*, T, hipStream_t);                                      \
  template void launch_restrict<T>(const Geo&, const Geo&, const T*, T*, hipStream_t);     \
  template void launch_prolong_add<T>(const Geo&, const Geo&, const T*, T*, hipStream_t);  \
  template void launch_coarse_solve<T>(const Geo&, const double*, int, const T*, T*,       \
                                       hipStream_t);                                       \
  template void launch_norm2_partial<T>(const Geo&, const T*, double*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace mg
