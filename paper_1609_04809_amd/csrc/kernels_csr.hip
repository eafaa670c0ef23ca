// CSR kernels of the Q1 multigrid V-cycle for gfx950: operator build,
// residual and smoothing sweeps on an assembled matrix.
//
// Row kernels stream the nonzeros of a block's rows: a block of NTH threads
// owns ROWS consecutive rows, reads their values and column indices
// contiguously (coalesced), multiplies by the gathered x and stages the
// products in LDS; NTH / ROWS threads then sum each row in a fixed order.
#include "mg_internal.h"

namespace mg {

namespace {

constexpr int CSR_MAX_ROW = 27;  // 3^dim entries at most
// Row kernel launch shape: rows per block and threads per block.
constexpr int CSR_ROWS = 64;
constexpr int CSR_NTH = 256;

// Sum of v over the NTH threads of a block; result valid in thread 0.
// Wave-level butterfly, then the wave sums in a fixed order.
template <int NTH>
__device__ __forceinline__ double block_sum_1d(double v) {
  __shared__ double ws[NTH / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (NTH == 64) return v;
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    t = ws[0];
#pragma unroll
    for (int w = 1; w < NTH / 64; ++w) t += ws[w];
  }
  return t;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MODE 0: out = b - A x (residual) with per-block partial sums of out^2.
// MODE 1: damped Jacobi update of rows [r_begin, r_end).
// MODE 2: red-black update of the rows of one colour [r_begin, r_end); the
//         other colour's unknowns are copied alongside (see below).
// MODE 3: over all rows, the residual partial sums of MODE 0 and, written to
//         out, the colour-0 red-black update with colour-1 unknowns copied.
// MODE 4: over all rows, the residual partial sums and the Jacobi update.
// MODE 5: out = A x over all rows with partial sums of x.(A x).
// MODE 6: Gauss-Seidel update of the rows of one colour [r_begin, r_end) in
//         place (out == xin): no row of the colour reads another's unknown.
// ZERO: x = 0 (x is not read).
// A block of CSR_NTH threads owns CSR_ROWS consecutive rows.  Each thread
// takes groups of 4 consecutive nonzeros starting at the block's first
// nonzero rounded down to a multiple of 4, with one 16-byte load of the
// columns and 16-byte loads of the values (the arrays are 256-byte aligned
// and padded by kCsrPad valid entries), so the matrix stream takes few load
// instructions; products of nonzeros outside the block's range land in LDS
// slots that no row sums.  The loads carry no branches: a thread past the
// block's last group re-reads that group, so all column and value loads of
// a thread are issued before the first gather waits.
template <typename T, int MODE, bool ZERO>
__global__ __launch_bounds__(CSR_NTH) void k_csr_rows(CsrOp<T> A, int r_begin, int r_end,
                                                      const T* __restrict__ xin,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ out, T omega,
                                                      double* __restrict__ partials) {
  constexpr int ROWS = CSR_ROWS, NTH = CSR_NTH;
  constexpr int MAXNNZ = ROWS * CSR_MAX_ROW;
  constexpr int PG = (MAXNNZ + 3 + 4 * NTH - 1) / (4 * NTH);  // groups per thread
  constexpr int SLOTS = 4 * PG * NTH + 3;
  constexpr int SOFF = 3;  // slot of the block's first nonzero
  constexpr int TPR = NTH / ROWS;  // threads summing one row
  __shared__ T prod[SLOTS];
  const int tid = threadIdx.x;
  const int blk = (int)blockIdx.x;
  const int r0 = r_begin + blk * ROWS;
  const int nr = min(ROWS, r_end - r0);
  // The block's nonzero range comes from two uniform (scalar) loads, so the
  // matrix stream starts after one round trip.  Every thread loads at
  // clamped indices (no branch around a load), so the loads of a phase are
  // all in flight before the first wait: its row's bounds and node, then,
  // with the matrix, the row's operands -- right-hand side, current value,
  // diagonal and (red-black) the other-colour neighbours to copy (all TPR
  // threads of a row read the same addresses; the row's owner, lane 0 of
  // its group, uses them).
  const int lr = tid / TPR, lane = tid % TPR;
  const bool owner = lane == 0 && lr < nr;
  const int lrc = min(lr, nr - 1);
  const int base = A.rowptr[r0];
  const int last = A.rowptr[r0 + nr] - base - 1;  // every row holds its diagonal
  const int rb = A.rowptr[r0 + lrc] - base, re = A.rowptr[r0 + lrc + 1] - base;
  const int node = A.rowmap[r0 + lrc];
  const T bv = b[node];
  T x0 = T(0), dg = T(1), xr = T(0), xl = T(0);
  if (!ZERO && MODE != 0) x0 = xin[node];
  if (MODE != 0) dg = A.val[base + rb];
  const int ix = node % (int)A.sy;
  const bool copy_r = MODE == 2 && ix + 1 <= A.n - 1;
  const bool copy_l = MODE == 2 && ix == 2;
  if (MODE == 2 && !ZERO) {
    xr = xin[node + 1];  // interior node: both neighbours lie in the grid
    xl = xin[node - 1];
  }
  if (!ZERO) {
    const int e0 = base & ~3;
    const int ng = (base + last + 1 - e0 + 3) >> 2;
    i32x4 c4[PG];
    T v4[PG][4];
#pragma unroll
    for (int q = 0; q < PG; ++q) {
      const int g = min(tid + q * NTH, ng - 1);
      c4[q] = *reinterpret_cast<const i32x4*>(A.col + e0 + 4 * g);
      if constexpr (sizeof(T) == 8) {
        const f64x2* vp = reinterpret_cast<const f64x2*>(A.val + e0 + 4 * g);
        const f64x2 lo = vp[0], hi = vp[1];
        v4[q][0] = lo.x;
        v4[q][1] = lo.y;
        v4[q][2] = hi.x;
        v4[q][3] = hi.y;
      } else {
        const f32x4 f = *reinterpret_cast<const f32x4*>(A.val + e0 + 4 * g);
        v4[q][0] = f.x;
        v4[q][1] = f.y;
        v4[q][2] = f.z;
        v4[q][3] = f.w;
      }
    }
    T xg[PG][4];
#pragma unroll
    for (int q = 0; q < PG; ++q) {
      xg[q][0] = xin[c4[q].x];
      xg[q][1] = xin[c4[q].y];
      xg[q][2] = xin[c4[q].z];
      xg[q][3] = xin[c4[q].w];
    }
    const int so = SOFF + (e0 - base) + 4 * tid;
#pragma unroll
    for (int q = 0; q < PG; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) prod[so + 4 * q * NTH + i] = v4[q][i] * xg[q][i];
  }
  __syncthreads();
  T s = T(0);
  if (!ZERO && lr < nr)
    for (int e = rb + lane; e < re; e += TPR) s += prod[SOFF + e];
#pragma unroll
  for (int off = 1; off < TPR; off <<= 1) s += __shfl_xor(s, off);
  double sq = 0.0;
  if (owner) {
    const T res = bv - s;
    if (MODE == 0) {
      out[node] = res;
      sq = (double)res * (double)res;
    } else if (MODE == 5) {
      out[node] = s;
      sq = (double)x0 * (double)s;
    } else if (MODE == 3 || MODE == 4) {
      // residual of every row plus the first smoothing step: Jacobi (4)
      // updates every row, red-black (3) the colour-0 rows, which come first
      sq = (double)res * (double)res;
      const bool upd = MODE == 4 || r0 + lr < A.coff[1];  // MODE 3 or 4
      const T q = res / dg;
      out[node] = upd ? (MODE == 4 ? x0 + omega * q : x0 + q) : x0;
    } else {
      const T q = res / dg;
      out[node] = MODE == 1 ? x0 + omega * q : x0 + q;  // MODE 1, 2, 6
      if (MODE == 2) {
        // Copy the other colour along the grid row: node p+1 (and p-1 for
        // the colour's first node at x = 2).  Every other-colour unknown of
        // the row is copied exactly once, by the block that also writes its
        // neighbour, so each cache line is written by one block.
        if (copy_r) out[node + 1] = xr;
        if (copy_l) out[node - 1] = xl;
      }
    }
  }
  if ((MODE == 0 || MODE == 3 || MODE == 4 || MODE == 5) && partials != nullptr) {
    const double t = block_sum_1d<NTH>(sq);
    if (tid == 0) partials[blk] = t;
  }
}

// One thread per row: diagonal first, then the neighbours q = p + d,
// d in {-1,0,1}^dim \ {0} in lexicographic (z, y, x) order, that are
// unknowns.  Entry value: sum over the cells containing both p and q of
// kappa_c * s_elem * f(#nonzero components of d), with the element-matrix
// classes f = {4, -1, -2} (2D, s_elem = 1/6) and {4, 0, -1, -1}
// (3D, s_elem = h/12).  kappa == nullptr means kappa = 1.  Values are
// formed in FP64 and rounded to T.
template <typename T, int DIM>
__global__ void k_csr_build(Geo g, const double* __restrict__ kappa, double s_elem,
                            double s_mass, int rows,
                            const int* __restrict__ rowmap, const int* __restrict__ rowptr,
                            int* __restrict__ col, T* __restrict__ val) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int node = rowmap[r];
  const int n = g.n;
  const int i = node % g.sy;
  const int j = (node / g.sy) % g.sy;
  const int k = DIM == 3 ? (int)(node / g.sz) : 0;
  const double f3[4] = {4.0, 0.0, -1.0, -1.0};
  const double f2[3] = {4.0, -1.0, -2.0};
  auto weight = [&](int dx, int dy, int dz) -> double {
    const int cls = abs(dx) + abs(dy) + abs(dz);
    double ks = 0.0;
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
      for (int bb = 0; bb < 2; ++bb)
        for (int a = 0; a < 2; ++a) {
          if (dx != 0 && a != (dx > 0)) continue;
          if (dy != 0 && bb != (dy > 0)) continue;
          if (DIM == 3 && dz != 0 && c != (dz > 0)) continue;
          if (kappa == nullptr) {
            ks += 1.0;
          } else {
            const long cell = (long)(i - 1 + a) + (long)n * (j - 1 + bb) +
                              (DIM == 3 ? (long)n * n * (k - 1 + c) : 0L);
            ks += kappa[cell];
          }
        }
    // the mass entry: (h/6)^dim 2^(dim-cls) per cell, on 2^(dim-cls) cells
    const double mass = s_mass * (double)(1 << (2 * (DIM - cls)));
    return s_elem * (DIM == 3 ? f3[cls] : f2[cls]) * ks + mass;
  };
  int pos = rowptr[r];
  col[pos] = node;
  val[pos] = (T)weight(0, 0, 0);
  ++pos;
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const int qi = i + dx, qj = j + dy, qk = k + dz;
        if (qi < 1 || qi > n - 1 || qj < 1 || qj > n - 1) continue;
        if (DIM == 3 && (qk < 1 || qk > n - 1)) continue;
        col[pos] = (int)(qi + qj * g.sy + (long)qk * g.sz);
        val[pos] = (T)weight(dx, dy, dz);
        ++pos;
      }
}

inline int cdiv_i(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T, int MODE>
void launch_rows(const CsrOp<T>& A, int rb, int re, const T* xin, const T* b, T* out, T omega,
                 double* partials, hipStream_t s) {
  const int nb = cdiv_i(re - rb, CSR_ROWS);
  if (nb == 0) return;
  if (xin == nullptr)
    MG_LAUNCH((k_csr_rows<T, MODE, true>), dim3(nb), dim3(CSR_NTH), 0, s, A, rb, re,
              xin, b, out, omega, partials);
  else
    MG_LAUNCH((k_csr_rows<T, MODE, false>), dim3(nb), dim3(CSR_NTH), 0, s, A, rb, re,
              xin, b, out, omega, partials);
}

}  // namespace

long csr_residual_blocks(int rows) { return cdiv_i(rows, CSR_ROWS); }
long csr_residual_blocks_max(int rows) { return cdiv_i(rows, CSR_ROWS); }

template <typename T>
void launch_csr_build(const Geo& g, const double* kappa, double s_elem, double s_mass, int rows,
                      const int* rowmap, const int* rowptr, int* col, T* val, hipStream_t s) {
  const unsigned blocks = (unsigned)cdiv_i(rows, 256);
  if (blocks == 0) return;
  if (g.dim == 2)
    MG_LAUNCH((k_csr_build<T, 2>), dim3(blocks), dim3(256), 0, s, g, kappa, s_elem,
              s_mass, rows, rowmap, rowptr, col, val);
  else
    MG_LAUNCH((k_csr_build<T, 3>), dim3(blocks), dim3(256), 0, s, g, kappa, s_elem,
              s_mass, rows, rowmap, rowptr, col, val);
}

template <typename T>
void launch_csr_residual(const Geo&, const CsrOp<T>& A, const T* x, const T* b, T* r,
                         double* partials, hipStream_t s) {
  launch_rows<T, 0>(A, 0, A.rows, x, b, r, T(0), partials, s);
}

template <typename T>
void launch_csr_head(const Geo&, const CsrOp<T>& A, int kind, const T* x, const T* b, T* xout,
                     T omega, double* partials, hipStream_t s) {
  if (kind == SM_JACOBI)
    launch_rows<T, 4>(A, 0, A.rows, x, b, xout, omega, partials, s);
  else
    launch_rows<T, 3>(A, 0, A.rows, x, b, xout, omega, partials, s);
}

template <typename T>
void launch_csr_apply_dot(const Geo&, const CsrOp<T>& A, const T* x, T* q, double* partials,
                          hipStream_t s) {
  // b is not used by MODE 5; x stands in for it so that every load is valid
  launch_rows<T, 5>(A, 0, A.rows, x, x, q, T(0), partials, s);
}

template <typename T>
void launch_csr_smooth(const Geo&, const CsrOp<T>& A, int kind, const T* xin, const T* b,
                       T* xout, T omega, hipStream_t s) {
  if (kind == SM_JACOBI) {
    launch_rows<T, 1>(A, 0, A.rows, xin, b, xout, omega, nullptr, s);
  } else if (kind >= SM_GS0) {
    const int c = kind - SM_GS0;
    launch_rows<T, 6>(A, A.coff[c], A.coff[c + 1], xout, b, xout, omega, nullptr, s);
  } else {
    const int c = kind == SM_RB1 ? 1 : 0;
    launch_rows<T, 2>(A, A.coff[c], A.coff[c + 1], xin, b, xout, omega, nullptr, s);
  }
}

#define INST(T)                                                                              \
  template void launch_csr_build<T>(const Geo&, const double*, double, double, int,         \
                                    const int*, const int*, int*, T*, hipStream_t);          \
  template void launch_csr_residual<T>(const Geo&, const CsrOp<T>&, const T*, const T*, T*,  \
                                       double*, hipStream_t);                                \
  template void launch_csr_smooth<T>(const Geo&, const CsrOp<T>&, int, const T*, const T*,   \
                                     T*, T, hipStream_t);                                    \
  template void launch_csr_head<T>(const Geo&, const CsrOp<T>&, int, const T*, const T*, T*, \
                                   T, double*, hipStream_t);                                 \
  template void launch_csr_apply_dot<T>(const Geo&, const CsrOp<T>&, const T*, T*, double*,  \
                                        hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace mg
