// Internal interfaces of the Q1 multigrid library: level geometry, operator
// descriptors, batched launch descriptors and the host-side launchers of
// the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
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
  bool s3;    // the plane-marching kernels (k_sweep3 and its fused forms) run the level
};

inline Geo make_geo(int dim, int n) {
  Geo g;
  g.dim = dim;
  g.n = n;
  g.sy = n + 1;
  g.sz = dim == 3 ? (long)(n + 1) * (n + 1) : 0;
  g.nodes = dim == 3 ? (long)(n + 1) * (n + 1) * (n + 1) : (long)(n + 1) * (n + 1);
  g.s3 = dim == 3 && n >= 32;
  return g;
}

// Timing of one profiled step: while `start` is set, the first kernel the
// step launches through MG_LAUNCH records its own start and end into
// start / stop (hipExtLaunchKernelGGL), so their elapsed time is that
// kernel's execution alone, with no gap before or after it; `launches`
// counts the kernels the step issued.  Every launch of the library goes
// through MG_LAUNCH; with `start` unset it is a plain hipLaunchKernelGGL.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  int launches = 0;
};
extern thread_local KernelEvents g_kernel_events;

#define MG_LAUNCH(KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                 \
  do {                                                                                   \
    ::mg::KernelEvents& kev_ = ::mg::g_kernel_events;                                    \
    if (kev_.start && kev_.launches++ == 0)                                              \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, kev_.start, kev_.stop, 0u, \
                            __VA_ARGS__);                                                \
    else                                                                                 \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                 \
  } while (0)

// Workgroups are dispatched round-robin over the 8 XCDs of the chip (each
// with its own L2) in linear order.  xcd_remap maps a dispatch index to a
// logical one such that every XCD owns one contiguous range of logical
// indices, so neighbouring tiles share an L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Entries past the last nonzero of a CSR level's column and value arrays,
// set to column 0 and value 0 at setup: a row kernel loads the nonzeros in
// aligned groups of 4 and may read up to 3 past the end (never summed).
constexpr int kCsrPad = 4;

// Largest coarsest system (unknowns) solved by the one-block Cholesky kernel.
constexpr int kCoarseMaxUnknowns = 4096;

// Levels with at most this many unknowns are cycled by one workgroup per
// request (the "tail" of the V-cycle), in one launch.
constexpr int kTailMaxUnknowns = 4096;
constexpr int kTailMaxLevels = 12;

// Rows of a 3D CSR colour are ordered by tiles of kCsrTile x kCsrTile grid
// rows in (y, z).
constexpr int kCsrTile = 8;

// Requests fused into one batched launch at most.
constexpr int kMaxBatch = 16;

enum OpKind { OP_CONST = 0, OP_KAPPA = 1, OP_MASS = 2 };

// Launch-wide parameters of the matrix-free Q1 operator of one level; the
// per-cell coefficients of OP_KAPPA travel per request in Item::kappa.
//  OP_CONST: kappa = 1, the assembled stencil weights of K + sigma M
//     2D: wc = 8/3, w1 = -1/3 (x/y neighbours), w2 = -1/3 (diagonals),
//         each plus sigma times the mass weight (h/6)^2 * {16, 4, 1};
//     3D (sigma = 0): wc = 8h/3, w1 = -h/6 (edge neighbours), w2 = -h/12
//         (corners); face neighbours have weight 0.
//  OP_MASS (3D, sigma > 0): K + sigma M with kappa = 1: wc, w1 (edges) and
//     w2 (corners) as for OP_CONST plus sigma (h/6)^3 * {64, 4, 1}, and
//     wf = sigma (h/6)^3 * 16 on the six face neighbours.
//  OP_KAPPA: element matrix scale s = 1/6 (2D), h/12 (3D).
template <typename T>
struct StencilParams {
  int kind;
  T wc, w1, w2;
  T s;
  T wf;
};

// One request's buffers in a batched launch.  The role of each pointer is
// given at each launcher below.
struct Item {
  const void* a;
  const void* b;
  void* c;
  const void* kappa;
  double* partials;
  double* scal;
  const double* L;
  const void* e;  // coarse correction (prolongation fused into a sweep)
  const void* a2;  // colour-split iterate: the odd half read (a: the even half)
  void* c2;        // colour-split iterate: the other colour's half written
  int flag;
  // Colour-split layout of the level's right-hand side read by a sweep (or
  // of the vector a restriction / FP32 cast writes): node p is stored at
  // p / 2 (even p) or lay + p / 2 (odd p); 0 = the natural layout.
  long lay;
};

// Index of node p in a vector stored colour-split with odd half at `lay`
// (lay = 0: natural).  For even n the parity of p is the red-black colour
// of the node, so a half-sweep reads its colour's half contiguously.
__host__ __device__ inline long lay_idx(long p, long lay) {
  return lay ? (p >> 1) + (p & 1) * lay : p;
}

// Scale s of the FP32 correction equations of iterative refinement, from
// ||b||^2: the power of two 2^e with ||b|| = m 2^e, 1/2 <= m < 1.  The
// cycle gets float(r / s) and u += s c; dividing and multiplying by a power
// of two is exact, so the scale changes no rounding, it only keeps the FP32
// values near unit size.
__host__ __device__ inline double ir_scale(double b_norm2) {
  int e;
  (void)frexp(sqrt(b_norm2), &e);
  return ldexp(1.0, e);
}

struct Batch {
  Item it[kMaxBatch];
  int count;
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
  int coff[9];  // colour c rows: [coff[c], coff[c+1]) (2 colours, or 2^dim
                // for multicolour Gauss-Seidel)
  int n;        // cells per direction of the level
  long sy;      // node stride in y
};

// Cycle kinds (the values of mg_cycle): how a level's coarse residual
// equation is solved -- one V-cycle, two W-cycles, or an F-cycle then a
// V-cycle.
enum CycleKind { CYC_V = 0, CYC_W = 1, CYC_F = 2 };

// Smoothing step kinds (mg_apply_smooth "step" 0..2); SM_GS0 + c, c <
// 2^dim: the Gauss-Seidel update of the unknowns of colour c (sum_d (x_d mod
// 2) 2^d) in place -- no two of them are coupled.
enum SmoothKind { SM_JACOBI = 0, SM_RB0 = 1, SM_RB1 = 2, SM_GS0 = 8 };

// Colour of node (i, j, k) for multicolour Gauss-Seidel.
__host__ __device__ inline int gs_colour(int i, int j, int k) {
  return (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
}

// Device-resident description of the tail levels l0..L-1 of one request:
// the V-cycle below level l0 runs inside one workgroup, with every vector
// of these levels in the launch's dynamic LDS.  Offsets are in elements of
// T from the start of that LDS region.
template <typename T>
struct TailLevel {
  int n;
  int ox, ot, ob, orr;  // iterate, spare, right-hand side, residual
  int ok;               // cell coefficients (OP_KAPPA)
  const T* kappa;       // device copy of the level's coefficients (OP_KAPPA)
  T wc, w1, w2, s, wf;  // operator parameters of the level
};
template <typename T>
struct TailDesc {
  int nlev;        // levels in the tail (the last one is the coarsest)
  int dim;
  int kind;        // OpKind
  int smoother;    // 0 Jacobi, 1 red-black
  int nu_pre, nu_post;
  T omega;
  int m;           // coarsest unknowns
  const double* L; // coarsest Cholesky factor (device memory)
  int oy;          // byte offset of the coarsest solve's m doubles
  int lds_bytes;   // dynamic LDS of the launch
  T* r0;           // first level's residual in device memory (nullptr: in LDS)
  TailLevel<T> lv[kTailMaxLevels];
};

// LDS a tail launch may use (gfx950 has 160 KB per workgroup).
constexpr int kTailLdsBytes = 150 * 1024;

// LDS bytes the tail needs for levels l0..levels-1 of a hierarchy (with the
// first level's residual in device memory when r0_global).
inline long tail_lds_bytes(int dim, int n, int levels, int l0, bool kappa, int elem,
                           bool r0_global) {
  long bytes = 0;
  for (int l = l0; l < levels; ++l) {
    const long nl = n >> l;
    long nodes = (nl + 1) * (nl + 1), cells = nl * nl;
    if (dim == 3) {
      nodes *= nl + 1;
      cells *= nl;
    }
    bytes += (l == l0 && r0_global ? 3 : 4) * ((nodes * elem + 15) / 16 * 16);
    if (kappa) bytes += (cells * elem + 15) / 16 * 16;
  }
  long nc = n >> (levels - 1), m = 1;
  for (int d = 0; d < dim; ++d) m *= nc - 1;
  return bytes + (m * 8 + 15) / 16 * 16;
}

// ---- grid kernels (kernels_grid.hip) -------------------------------------
template <typename T> void launch_fill(T* v, long count, T val, hipStream_t s);
template <typename T> void launch_copy(const T* a, T* b, long count, hipStream_t s);

// Number of per-block partial sums per request written by a residual
// launch (grid_blocks) and by a norm launch (norm2_blocks).
long grid_blocks(const Geo& g);
long norm2_blocks(const Geo& g);

// r = b - A x (+ per-block partial sums of r^2 when `norm`):
//   a = x, b = b, c = r, kappa, partials.
// xl = XL_SPLIT (k_sweep3 levels, constant-coefficient or mass-shifted):
// x read colour-split, a = its even half, a2 = its odd half.
// cast (FP64, k_sweep3 levels, x and b natural): r is not stored; instead
// float(r / ir_scale(*scal)) goes to the FP32 vector c in the layout lay
// (the right-hand side of the refinement's FP32 cycle).
template <typename T>
void launch_residual(const Geo& g, const StencilParams<T>& op, bool norm, const Batch& B,
                     hipStream_t s, int xl = 0, bool cast = false);
// b_c = R (b - A x) on a 3D level where use_split_x(g), constant-coefficient
// or mass-shifted operator, without storing r (the three fine columns of
// r under each of the coarse columns 64, 128, ... go to e, packed;
// launch_restrict_xcols restricts those columns afterwards):  a = x (xin:
// its even half, a2 the odd half), b = b (layout lay), c = b_c
// (colour-split when flag), e = scratch of the level's node count.
// Bitwise the result of launch_residual followed by launch_restrict.
template <typename T>
void launch_resid_restrict(const Geo& g, const StencilParams<T>& op, bool xin, const Batch& B,
                           hipStream_t s);
// The coarse columns launch_resid_restrict leaves (their number:
// resid_restrict_xcols(gf)):  a = the packed columns (its e), c = b_c
// (layout lay).
int resid_restrict_xcols(const Geo& gf);
template <typename T>
void launch_restrict_xcols(const Geo& gf, const Batch& B, hipStream_t s);
// u = the natural layout of a colour-split vector (every node; the halves'
// boundary entries are 0):  a = even half, a2 = odd half, c = u.
template <typename T>
void launch_unsplit(const Geo& g, const Batch& B, hipStream_t s);
// One smoothing step (SmoothKind); a == nullptr means x = 0 (then for every
// item):  a = x_in, b = b, c = x_out, kappa.  Gauss-Seidel colour steps
// (kind >= SM_GS0) update c in place (a is ignored, zero is not allowed).
// xl (red-black on levels where use_split_x(g), XLayout): the iterate's
// layout in and out -- split halves are a (even) / a2 (odd) when read, c
// (the updated colour) and c2 (the other colour, XL_TO_SPLIT) when written.
// iru (FP32, k_sweep3 levels, a step with natural output: xl 0 or
// XL_TO_NATURAL, kind SM_JACOBI / SM_RB0 / SM_RB1): the step's result c is
// not stored; instead u += ir_scale(*scal) c with c = u (FP64), scal.
template <typename T>
void launch_smooth(const Geo& g, const StencilParams<T>& op, int kind, bool zero, T omega,
                   const Batch& B, hipStream_t s, int xl = 0, bool iru = false);
enum XLayout {
  XL_NATURAL = 0,
  XL_TO_SPLIT = 1,     // natural in, both halves out
  XL_SPLIT = 2,        // split in, the updated colour's half out
  XL_TO_NATURAL = 3,   // split in, natural out
  XL_SPLIT_BOTH = 4    // split in, both halves out (the fused prolongation)
};
// Whether k_sweep3 runs the level (Geo::s3: 3D levels with n >= 32; the
// runtime keeps coarse levels below n = 96 on the per-node kernels under
// graph replay), which is where split iterates are possible.
bool use_split_x(const Geo& g);
// Two red-black half-sweeps in one pass, colour `first` (SM_RB0 / SM_RB1)
// then the other; bitwise the result of two launch_smooth calls.  Only on
// levels where pair_sweeps(g):  a = x_in (nullptr: x = 0), b = b, c = x_out.
bool pair_sweeps(const Geo& g);
// x + P e, then one smoothing step (SM_JACOBI / SM_RB0 / SM_RB1) of it, in
// one pass; bitwise launch_prolong_add followed by launch_smooth.  Only on
// levels where pair_sweeps(g):  a = x (the level's iterate before the
// correction), e = e (coarse correction), b = b, c = x_out (with xl =
// XL_TO_SPLIT, red-black: c the updated colour's half, c2 the other's).
template <typename T>
void launch_smooth_prolong(const Geo& g, const StencilParams<T>& op, int kind, T omega,
                           const Batch& B, hipStream_t s, int xl = 0);
template <typename T>
void launch_smooth_pair(const Geo& g, const StencilParams<T>& op, int first, bool zero,
                        const Batch& B, hipStream_t s);
// b_c = P^T r:  a = r (fine), c = b_c (coarse).
template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s);
// x += P e:  a = e (coarse), c = x (fine).
template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const Batch& B, hipStream_t s);
// Coarsest solve, one block per request:  b = b_c, c = x_c, L (m x m).
template <typename T>
void launch_coarse_solve(const Geo& gc, int m, const Batch& B, hipStream_t s);
// In one pass over x: per-block partial sums of (b - A x)^2 (as the residual
// launch writes them) and the first smoothing step of the next cycle, kind
// SM_JACOBI or SM_RB0:  a = x, b = b, c = x_out, kappa, partials.  With xl =
// XL_TO_SPLIT (red-black on split-iterate levels) x_out is written
// colour-split: c = the even half, c2 = the odd half.
template <typename T>
void launch_head(const Geo& g, const StencilParams<T>& op, int kind, T omega, const Batch& B,
                 hipStream_t s, int xl = 0);
// Per-block partial sums of v^2:  a = v, partials.
template <typename T>
void launch_norm2_partial(const Geo& g, const Batch& B, hipStream_t s);
// scal = sum of partials[0..count), fixed order, one block per request.
void launch_reduce_final(long count, const Batch& B, hipStream_t s);
// b32 = float(r / ir_scale(*scal)):  a = r (double), c = b32 (float), scal
// (= ||b||^2), lay (b32's layout).
void launch_scale_cast(const Geo& g, const Batch& B, hipStream_t s);
// u += ir_scale(*scal) * double(c):  a = c (float), c = u (double), scal.
void launch_ir_update(const Geo& g, const Batch& B, hipStream_t s);
// The V-cycle on the tail levels, one block per request:  a = TailDesc<T>*
// (device), b = level-l0 right-hand side, c = level-l0 iterate (updated in
// place), flag = 1 when the level-l0 iterate starts at 0 (not read).
template <typename T>
void launch_tail(int dim, int kind, int lds_bytes, const Batch& B, hipStream_t s);

// A whole FP64 solve by one workgroup per request, for hierarchies the
// tail holds from their finest level on (TailDesc from level 0):  a =
// TailDesc<double>* (device), b = b (finest level, natural layout), c = u
// (out: every node), scal = results (kTailSolveHead + max_iter + 1
// doubles: status (TailSolveStatus), cycles done, then the relative
// residual history from cycle 0), flag = cycle kind << 1.  Stops at the
// first cycle whose relative residual is <= tol, or on divergence (not
// finite or > 1e3), or after max_iter cycles.
enum TailSolveStatus { TS_OK = 0, TS_MAXIT = 1, TS_DIVERGED = 2, TS_NONFINITE_B = 3 };
constexpr int kTailSolveHead = 2;
void launch_tail_solve(int dim, int kind, int lds_bytes, const Batch& B, double tol, int max_iter,
                       hipStream_t s);

void launch_kappa_coarsen(int dim, int nf, const double* kf, double* kc, hipStream_t s);
void launch_cast_f32(const double* a, float* b, long count, hipStream_t s);
void launch_count_bad_kappa(const double* k, long count, int* bad_nonpos, int* bad_nonfinite,
                            hipStream_t s);

// q = A x with per-block partial sums of x.q (the operator-apply step of
// preconditioned CG):  a = x, c = q, kappa, partials.
template <typename T>
void launch_apply_dot(const Geo& g, const StencilParams<T>& op, const Batch& B, hipStream_t s);

// Crank-Nicolson right-hand side (FP64) on the unknowns of a level with
// kappa = 1:  b = Wb x0 - Wa x1 + cf F, where x0 is u inside and c0 g0 on
// the boundary, x1 is c1 g1 on the boundary and 0 inside, and Wb, Wa are
// constant 3^dim stencils with weights wb, wa per neighbour class |dx| +
// |dy| (+ |dz|) (sigma M - K and sigma M + K; with wb = the mass weights,
// u = g0 = f, c0 = 1 and wa = 0 this is the load M f).  g0, g1, F and
// guess may be nullptr; guess (in/out) becomes 2 u - guess.
struct CnWeights {
  double wb[4], wa[4];
  double c0, c1, cf;
};
void launch_cn_rhs(const Geo& g, const CnWeights& w, const double* u, double* guess,
                   const double* g0, const double* g1, const double* F, double* b,
                   hipStream_t s);
// The same with the node kernel at every size, without x1, F and guess.
void launch_cn_rhs_nodes(const Geo& g, const CnWeights& w, const double* u, const double* g0,
                         double* b, hipStream_t s);
// v = 0 on the boundary nodes of the level (interior untouched).
void launch_zero_boundary(const Geo& g, double* v, hipStream_t s);
// dst[lay_idx(p, lay)] = src[p] on the unknowns p (natural -> colour-split;
// the boundary entries of dst are not written), with the per-block partial
// sums of src^2 that launch_norm2_partial writes (same grid and order, so
// the same bits), in one pass.
void launch_split_norm(const Geo& g, const double* src, double* dst, long lay,
                       double* partials, hipStream_t s);

// ---- CSR kernels (kernels_csr.hip) ----------------------------------------
// Entries of K + sigma M: s_elem scales the stiffness element factors,
// s_mass = sigma (h/6)^dim the mass ones.
template <typename T>
void launch_csr_build(const Geo& g, const double* kappa, double s_elem, double s_mass, int rows,
                      const int* rowmap, const int* rowptr, int* col, T* val, hipStream_t s);
template <typename T>
void launch_csr_residual(const Geo& g, const CsrOp<T>& A, const T* x, const T* b, T* r,
                         double* partials, hipStream_t s);
long csr_residual_blocks(int rows);      // partial sums of one residual launch
long csr_residual_blocks_max(int rows);  // upper bound over launch variants
// Residual partial sums of x (as launch_csr_residual) and the smoothing
// step SM_JACOBI / SM_RB0 from x into xout, over all rows in one pass.
template <typename T>
void launch_csr_head(const Geo& g, const CsrOp<T>& A, int kind, const T* x, const T* b, T* xout,
                     T omega, double* partials, hipStream_t s);
// q = A x with per-block partial sums of x.q, over all rows.
template <typename T>
void launch_csr_apply_dot(const Geo& g, const CsrOp<T>& A, const T* x, T* q, double* partials,
                          hipStream_t s);
// Gauss-Seidel colour steps (kind >= SM_GS0) need xin == xout (in place)
// and rows blocked by 2^dim colours.
template <typename T>
void launch_csr_smooth(const Geo& g, const CsrOp<T>& A, int kind, const T* xin, const T* b,
                       T* xout, T omega, hipStream_t s);

// ---- preconditioned CG vector kernels (kernels_pcg.hip) -------------------
// Device scalars of the iteration (indices into the context's scal[]);
// scal[0] holds ||r||^2 and scal[1] ||b||^2 as for every solve.
enum PcgScalar { PCG_PQ = 3, PCG_RZ = 4, PCG_ZR = 5, PCG_ZRO = 6, PCG_BETA = 7 };
constexpr int kPcgBlocks = 1024;  // blocks (and partial sums) of a vector kernel
long pcg_blocks(long n);
void launch_pcg_dots2(const double* z, const double* r, const double* ro, long n, double* pa,
                      double* pb, hipStream_t s);
void launch_pcg_scalars(double* scal, int first, hipStream_t s);
void launch_pcg_dir(const double* z, double* p, const double* scal, long n, int first,
                    hipStream_t s);
void launch_pcg_update(double* u, const double* p, double* r, double* ro, const double* q,
                       const double* scal, long n, double* part, hipStream_t s);
void launch_pcg_zscale(const float* c, double* z, const double* scal, long n, hipStream_t s);

}  // namespace mg
