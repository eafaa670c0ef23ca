// Vector kernels of the multigrid-preconditioned conjugate gradient
// iteration on the finest level, for gfx950.  Vectors are full-grid FP64
// arrays whose boundary entries are 0, so a sum over all nodes is the sum
// over the unknowns.  Each kernel streams its vectors once, coalesced, in a
// grid-stride loop over a fixed number of blocks; a dot product leaves one
// partial sum per block, reduced afterwards in a fixed order
// (launch_reduce_final), so results do not depend on scheduling.  The
// iteration's scalars live in device memory (scal[] of the context) and are
// read by every thread, so one iteration needs no host round trip.
#include "mg_internal.h"

namespace mg {

namespace {

constexpr int PT = 256;  // threads per block

__device__ __forceinline__ double block_sum_pcg(double v) {
  __shared__ double ws[PT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  return t;
}

// partial sums of z.r and z.r_old
__global__ __launch_bounds__(PT) void k_pcg_dots2(const double* __restrict__ z,
                                                  const double* __restrict__ r,
                                                  const double* __restrict__ ro, long n,
                                                  double* __restrict__ pa,
                                                  double* __restrict__ pb) {
  double a = 0.0, c = 0.0;
  for (long e = blockIdx.x * (long)PT + threadIdx.x; e < n; e += (long)gridDim.x * PT) {
    const double zv = z[e];
    a += zv * r[e];
    c += zv * ro[e];
  }
  a = block_sum_pcg(a);
  __syncthreads();
  c = block_sum_pcg(c);
  if (threadIdx.x == 0) {
    pa[blockIdx.x] = a;
    pb[blockIdx.x] = c;
  }
}

// beta = (z.r - z.r_old) / rz (0 on the first iteration), then rz = z.r
__global__ void k_pcg_scalars(double* __restrict__ scal, int first) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal[PCG_BETA] = first ? 0.0 : (scal[PCG_ZR] - scal[PCG_ZRO]) / scal[PCG_RZ];
    scal[PCG_RZ] = scal[PCG_ZR];
  }
}

// p = z + beta p  (p = z on the first iteration: p is not read)
__global__ __launch_bounds__(PT) void k_pcg_dir(const double* __restrict__ z,
                                                double* __restrict__ p,
                                                const double* __restrict__ scal, long n,
                                                int first) {
  const double beta = scal[PCG_BETA];
  for (long e = blockIdx.x * (long)PT + threadIdx.x; e < n; e += (long)gridDim.x * PT)
    p[e] = first ? z[e] : z[e] + beta * p[e];
}

// alpha = rz / p.q;  u += alpha p;  r_old = r;  r -= alpha q;  partials of r.r
__global__ __launch_bounds__(PT) void k_pcg_update(double* __restrict__ u,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ r,
                                                   double* __restrict__ ro,
                                                   const double* __restrict__ q,
                                                   const double* __restrict__ scal, long n,
                                                   double* __restrict__ part) {
  const double alpha = scal[PCG_RZ] / scal[PCG_PQ];
  double sq = 0.0;
  for (long e = blockIdx.x * (long)PT + threadIdx.x; e < n; e += (long)gridDim.x * PT) {
    const double rv = r[e];
    const double rn = rv - alpha * q[e];
    u[e] += alpha * p[e];
    ro[e] = rv;
    r[e] = rn;
    sq += rn * rn;
  }
  sq = block_sum_pcg(sq);
  if (threadIdx.x == 0) part[blockIdx.x] = sq;
}

// z = s * double(c), s = ir_scale(scal[0] = ||r||^2) (the FP32
// preconditioner's correction scaled back)
__global__ __launch_bounds__(PT) void k_pcg_zscale(const float* __restrict__ c,
                                                   double* __restrict__ z,
                                                   const double* __restrict__ scal, long n) {
  const double s = ir_scale(scal[0]);
  for (long e = blockIdx.x * (long)PT + threadIdx.x; e < n; e += (long)gridDim.x * PT)
    z[e] = s * (double)c[e];
}

inline unsigned pcg_grid(long n) {
  const long b = (n + PT - 1) / PT;
  return (unsigned)(b < kPcgBlocks ? b : kPcgBlocks);
}

}  // namespace

long pcg_blocks(long n) { return pcg_grid(n); }

void launch_pcg_dots2(const double* z, const double* r, const double* ro, long n, double* pa,
                      double* pb, hipStream_t s) {
  MG_LAUNCH(k_pcg_dots2, dim3(pcg_grid(n)), dim3(PT), 0, s, z, r, ro, n, pa, pb);
}

void launch_pcg_scalars(double* scal, int first, hipStream_t s) {
  MG_LAUNCH(k_pcg_scalars, dim3(1), dim3(64), 0, s, scal, first);
}

void launch_pcg_dir(const double* z, double* p, const double* scal, long n, int first,
                    hipStream_t s) {
  MG_LAUNCH(k_pcg_dir, dim3(pcg_grid(n)), dim3(PT), 0, s, z, p, scal, n, first);
}

void launch_pcg_update(double* u, const double* p, double* r, double* ro, const double* q,
                       const double* scal, long n, double* part, hipStream_t s) {
  MG_LAUNCH(k_pcg_update, dim3(pcg_grid(n)), dim3(PT), 0, s, u, p, r, ro, q, scal, n,
            part);
}

void launch_pcg_zscale(const float* c, double* z, const double* scal, long n, hipStream_t s) {
  MG_LAUNCH(k_pcg_zscale, dim3(pcg_grid(n)), dim3(PT), 0, s, c, z, scal, n);
}

}  // namespace mg
