// Host runtime of the Q1 multigrid library: option validation, the device
// arena, the level hierarchy (Sec. 5.1), the V-cycle driver (Algorithm 1,
// Sec. 5.3), the outer cycle iteration (Sec. 5.5.1), the FP32-inner /
// FP64-outer refinement loop, HIP graph replay of whole cycles and the
// solver part of the C ABI declared in mg.h.
//
// A cycle is produced as a list of recorded kernel launches (OpRec); a
// single solve launches them one by one (or replays them as one captured
// graph), the serving scheduler fuses equal ops of different requests into
// batched launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "mg_ctx.h"

using namespace mg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace mg {
thread_local std::string g_err;
thread_local KernelEvents g_kernel_events;

mg_status fail(mg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
}  // namespace mg

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(MG_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                             \
  } while (0)

namespace {

constexpr size_t kAlign = 256;

// Bump allocator over the arena; with base == nullptr it only measures.
struct Planner {
  char* base;
  size_t off = 0;
  explicit Planner(char* b) : base(b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

long ipow(long b, int e) {
  long r = 1;
  while (e--) r *= b;
  return r;
}

long csr_nnz(int dim, int n) { return ipow(3L * n - 5, dim); }

bool valid_options(const mg_options* o, std::string& why) {
  char buf[256];
  if (!o) { why = "options is NULL"; return false; }
  if (o->dim != 2 && o->dim != 3) { why = "dim must be 2 or 3"; return false; }
  if (o->n < 2) { why = "n must be >= 2"; return false; }
  if (o->levels < 1 || o->levels > 30) { why = "levels must be in 1..30"; return false; }
  if (o->n % (1 << (o->levels - 1)) != 0 || (o->n >> (o->levels - 1)) < 2) {
    snprintf(buf, sizeof buf,
             "n = %d needs to be divisible by 2^(levels-1) with n >> (levels-1) >= 2", o->n);
    why = buf;
    return false;
  }
  if (o->op != MG_OP_STENCIL && o->op != MG_OP_CSR) { why = "op must be MG_OP_STENCIL or MG_OP_CSR"; return false; }
  if (o->smoother != MG_SMOOTH_JACOBI && o->smoother != MG_SMOOTH_RBGS && o->smoother != MG_SMOOTH_GS) { why = "unknown smoother"; return false; }
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post > 64) { why = "nu_pre/nu_post out of range"; return false; }
  if (o->smoother == MG_SMOOTH_JACOBI && !(o->omega > 0.0 && o->omega <= 1.0)) { why = "omega must be in (0, 1]"; return false; }
  if (o->precision != MG_PREC_FP64 && o->precision != MG_PREC_FP32_IR) { why = "unknown precision"; return false; }
  if (o->max_iter < 1) { why = "max_iter must be >= 1"; return false; }
  if (o->flags & ~(MG_FLAG_NO_GRAPH | MG_FLAG_NO_TAIL | MG_FLAG_NO_FUSE | MG_FLAG_PCG | MG_FLAG_PAIR | MG_FLAG_WARM | MG_FLAG_NO_SPLIT)) { why = "unknown flags"; return false; }
  if (!(std::isfinite(o->sigma) && o->sigma >= 0.0)) { why = "sigma must be finite and >= 0"; return false; }
  if (o->sigma > 0.0 && (o->flags & MG_FLAG_PAIR)) { why = "MG_FLAG_PAIR needs sigma == 0"; return false; }
  if (o->cycle != MG_CYCLE_V && o->cycle != MG_CYCLE_W && o->cycle != MG_CYCLE_F) { why = "cycle must be V, W or F"; return false; }
  if ((o->flags & MG_FLAG_PCG) && (o->nu_pre != o->nu_post || o->cycle == MG_CYCLE_F)) { why = "CG needs a symmetric cycle (V or W, nu_pre == nu_post)"; return false; }
  const long nc = o->n >> (o->levels - 1);
  const long m = ipow(nc - 1, o->dim);
  if (m > kCoarseMaxUnknowns) {
    snprintf(buf, sizeof buf, "coarsest level has %ld unknowns (max %d): use more levels", m,
             kCoarseMaxUnknowns);
    why = buf;
    return false;
  }
  const long nodes = ipow(o->n + 1L, o->dim);
  if (nodes >= (1L << 31)) { why = "grid too large for 32-bit node indices"; return false; }
  if (o->op == MG_OP_CSR && csr_nnz(o->dim, o->n) + kCsrPad >= (1L << 31)) {
    why = "CSR matrix too large for 32-bit offsets";
    return false;
  }
  return true;
}

// First level handled by the tail kernel: the finest level from which on
// every level has at most kTailMaxUnknowns unknowns and all their vectors
// (FP64) fit the tail's LDS (at most kTailMaxLevels levels); -1 if not even
// the coarsest level fits.  The tail applies each level's operator
// matrix-free, also in a CSR hierarchy: the CSR matrices hold the same
// rediscretised entries (up to the rounding of each entry).
int tail_start(const mg_options& o, bool kappa) {
  if (o.flags & MG_FLAG_NO_TAIL) return -1;
  // the tail's per-cell operator has no mass term
  if (kappa && o.sigma > 0.0) return -1;
  auto fits = [&](int l) {
    return tail_lds_bytes(o.dim, o.n, o.levels, l, kappa, 8, true) <= kTailLdsBytes;
  };
  int l0 = o.levels - 1;
  if (!fits(l0)) return -1;
  while (l0 > 0 && ipow((o.n >> (l0 - 1)) - 1, o.dim) <= kTailMaxUnknowns &&
         o.levels - (l0 - 1) <= kTailMaxLevels && fits(l0 - 1))
    --l0;
  return l0;
}

// Whether the right-hand sides of a level with n_l cells, in elements of
// `elem` bytes, are stored colour-split (Item::lay): 3D matrix-free levels
// swept by k_sweep3 with red-black or Jacobi smoothing on single
// half-sweeps, even n_l (then a node's index parity is its colour), and
// vectors of at least 64 MB, which stream largely from HBM (smaller levels
// stay in the 256 MB last-level cache, where the split layout measured no
// gain; the 256^3 FP32 level, 68 MB per vector, gains 2% of the solve).
constexpr long kSplitMinBytes = 64L << 20;
bool split_level(const mg_options& o, int nl, int elem) {
  const long nodes = (long)(nl + 1) * (nl + 1) * (nl + 1);
  return o.op == MG_OP_STENCIL && o.dim == 3 && nl >= 32 && nl % 2 == 0 &&
         nodes * elem >= kSplitMinBytes && o.smoother != MG_SMOOTH_GS &&
         !(o.flags & (MG_FLAG_PAIR | MG_FLAG_NO_SPLIT));
}

// FP64 solves without CG keep a colour-split copy of the caller's b.
bool split_b0(const mg_options& o) {
  return o.precision == MG_PREC_FP64 && !(o.flags & MG_FLAG_PCG) && split_level(o, o.n, 8);
}

// Odd-half offset (Item::lay) of level l's right-hand side in precision
// prec (0 FP64, 1 FP32), 0 for the natural layout.  Level 0 in FP64 is the
// caller's b (or, in mg_solve without CG, its split copy); in FP32 the
// cast of the scaled residual, written split.
long b_split_half(const mg_ctx* c, int l, int prec) {
  if (c->natural || !split_level(c->o, c->lv[l].g.n, prec == 0 ? 8 : 4)) return 0;
  if (l == 0 && prec == 0 && !c->b0_split) return 0;
  return (c->lv[l].g.nodes + 1) / 2;
}

// Whether the red-black half-sweeps of a level (elements of elem bytes)
// keep the iterate colour-split between the first and the last half-sweep
// of a smoothing run: matrix-free constant-coefficient or mass-shifted
// levels where the right-hand side is split too.
bool split_x_level(const mg_options& o, bool has_kappa, int nl, int elem) {
  return !has_kappa && o.smoother == MG_SMOOTH_RBGS && split_level(o, nl, elem);
}

// Lay out every buffer of a context; with base == nullptr only sizes.
size_t plan(const mg_options& o, bool has_kappa, char* base, mg_ctx* c) {
  Planner P(base);
  const bool ir = o.precision == MG_PREC_FP32_IR;
  const bool csr = o.op == MG_OP_CSR;
  long maxpart = 1;
  for (int l = 0; l < o.levels; ++l) {
    const int nl = o.n >> l;
    Geo g = make_geo(o.dim, nl);
    // The plane-marching kernels run the 3D levels with n >= 32, except the
    // coarse levels below n = 96 of a context whose cycles are replayed from
    // graphs: there the per-node kernels are faster (their separate launches
    // cost little in a graph; measured 2-3% of the 256^3 FP32-refinement and
    // 192^3 kappa solves).  Launched one by one (MG_FLAG_NO_GRAPH, the
    // server), the fused kernels' fewer launches pay.  Both compute every
    // node bitwise alike, and no norm is formed on a coarse level, so the
    // choice changes no result.
    g.s3 = g.s3 && (l == 0 || nl >= 96 || (o.flags & MG_FLAG_NO_GRAPH));
    Level tmp;
    Level& L = c ? c->lv[l] : tmp;
    L.g = g;
    // right-hand sides: one element past the nodes pads the odd half of a
    // colour-split b (read, unused, by a red-black half-sweep's clamped lanes)
    if (l > 0) {
      L.x64 = P.take<double>(g.nodes);
      L.b64 = P.take<double>(g.nodes + 1);
    } else if (split_b0(o)) {
      L.b64 = P.take<double>(g.nodes + 1);  // colour-split copy of the caller's b
    }
    L.t64 = P.take<double>(g.nodes);
    L.r64 = P.take<double>(g.nodes);
    if (l == 0 && (o.flags & MG_FLAG_PCG)) {
      L.p64 = P.take<double>(g.nodes);
      L.q64 = P.take<double>(g.nodes);
      L.z64 = P.take<double>(g.nodes);
      L.rk64 = P.take<double>(g.nodes);
      L.ro64 = P.take<double>(g.nodes);
      maxpart = std::max(maxpart, 2 * (long)kPcgBlocks);
    }
    if (ir) {
      L.x32 = P.take<float>(g.nodes);
      L.b32 = P.take<float>(g.nodes + 1);
      L.t32 = P.take<float>(g.nodes);
      L.r32 = P.take<float>(g.nodes);
    }
    // colour-split iterates for the red-black runs of the cycles (FP64
    // cycles, or the FP32 inner cycles)
    if (split_x_level(o, has_kappa, nl, ir ? 4 : 8)) {
      for (int q = 0; q < 2; ++q) {
        if (ir)
          L.xs32[q] = P.take<float>(g.nodes + 1);
        else
          L.xs64[q] = P.take<double>(g.nodes + 1);
      }
    }
    const long cells = ipow(nl, o.dim);
    if (has_kappa) {
      L.kap64 = P.take<double>(cells);
      if (ir) L.kap32 = P.take<float>(cells);
    }
    if (csr) {
      const long rows = ipow(nl - 1, o.dim);
      const long nnz = csr_nnz(o.dim, nl);
      L.rows = (int)rows;
      L.nnz = nnz;
      L.rowptr = P.take<int>(rows + 1);
      L.col = P.take<int>(nnz + kCsrPad);
      L.rowmap = P.take<int>(rows);
      L.val64 = P.take<double>(nnz + kCsrPad);
      if (ir) L.val32 = P.take<float>(nnz + kCsrPad);
      maxpart = std::max(maxpart, csr_residual_blocks_max((int)rows));
    }
    maxpart = std::max(maxpart, std::max(grid_blocks(g), norm2_blocks(g)));
  }
  const long nc = o.n >> (o.levels - 1);
  const int m = (int)ipow(nc - 1, o.dim);
  double* Lc = P.take<double>((size_t)m * m);
  double* part = P.take<double>(maxpart);
  double* scal = P.take<double>(8);
  int* ibuf = P.take<int>(8);
  double* tres = P.take<double>(kTailSolveHead + o.max_iter + 1);
  void* t64 = P.take<TailDesc<double>>(1);
  void* t32 = ir ? (void*)P.take<TailDesc<float>>(1) : nullptr;
  if (c) {
    c->Lc = Lc;
    c->m = m;
    c->partials = part;
    c->npart = maxpart;
    c->scal = scal;
    c->ibuf = ibuf;
    c->tres = tres;
    c->tail64 = t64;
    c->tail32 = t32;
  }
  return (P.off + kAlign - 1) / kAlign * kAlign;
}

// Entry of the rediscretised Q1 matrix between node (i,j,k) and its
// neighbour at offset d, from the cell coefficients kap (nullptr = 1):
// the sum over the cells containing both nodes of kappa_c times the element
// matrix entry, which depends only on the number of nonzero components of d.
double q1_entry(int dim, int n, const double* kap, double sigma, int i, int j, int k,
                int dx, int dy, int dz) {
  const double h = 1.0 / n;
  const double f3[4] = {4.0, 0.0, -1.0, -1.0};
  const double f2[3] = {4.0, -1.0, -2.0};
  const int cls = std::abs(dx) + std::abs(dy) + std::abs(dz);
  double ks = 0.0;
  for (int c = 0; c < (dim == 3 ? 2 : 1); ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        if (dx != 0 && a != (dx > 0)) continue;
        if (dy != 0 && b != (dy > 0)) continue;
        if (dim == 3 && dz != 0 && c != (dz > 0)) continue;
        if (!kap) {
          ks += 1.0;
        } else {
          const long cell = (long)(i - 1 + a) + (long)n * (j - 1 + b) +
                            (dim == 3 ? (long)n * n * (k - 1 + c) : 0L);
          ks += kap[cell];
        }
      }
  // mass: (h/6)^dim 2^(dim-cls) per cell on the 2^(dim-cls) shared cells
  const double mass = sigma * std::pow(h / 6.0, dim) * (double)(1 << (2 * (dim - cls)));
  return (dim == 3 ? (h / 12.0) * f3[cls] * ks : (1.0 / 6.0) * f2[cls] * ks) + mass;
}

// Dense matrix of a level with n cells (its m unknowns) from the cell
// coefficients kap (host, n^d, nullptr = 1), and its Cholesky factor in
// place (row major, lower): A = L L^T.  A holds m * m doubles.
mg_status coarse_cholesky(int dim, int n, const double* kap, double sigma, int m, double* A) {
  const int mi = n - 1;
  for (long q = 0; q < (long)m * m; ++q) A[q] = 0.0;
  for (int q = 0; q < m; ++q) {
    const int i = q % mi + 1, j = (q / mi) % mi + 1, k = dim == 3 ? q / (mi * mi) + 1 : 0;
    for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int qi = i + dx, qj = j + dy, qk = k + dz;
          if (qi < 1 || qi > mi || qj < 1 || qj > mi) continue;
          if (dim == 3 && (qk < 1 || qk > mi)) continue;
          const int q2 = (qi - 1) + mi * (qj - 1) + (dim == 3 ? mi * mi * (qk - 1) : 0);
          A[(size_t)q * m + q2] = q1_entry(dim, n, kap, sigma, i, j, k, dx, dy, dz);
        }
  }
  for (int jj = 0; jj < m; ++jj) {
    double d = A[(size_t)jj * m + jj];
    for (int p = 0; p < jj; ++p) d -= A[(size_t)jj * m + p] * A[(size_t)jj * m + p];
    if (!(d > 0.0)) return fail(MG_E_NOT_SPD, "coarsest matrix: pivot %d is %g", jj, d);
    const double ljj = std::sqrt(d);
    A[(size_t)jj * m + jj] = ljj;
    for (int ii = jj + 1; ii < m; ++ii) {
      double v = A[(size_t)ii * m + jj];
      for (int p = 0; p < jj; ++p) v -= A[(size_t)ii * m + p] * A[(size_t)jj * m + p];
      A[(size_t)ii * m + jj] = v / ljj;
    }
    for (int p = jj + 1; p < m; ++p) A[(size_t)jj * m + p] = 0.0;
  }
  return MG_OK;
}

// The context's coarsest factor, built on the host and copied to c->Lc.
mg_status coarse_factor(mg_ctx* c, hipStream_t s) {
  const Level& Lv = c->lv[c->L - 1];
  const int dim = c->o.dim, n = Lv.g.n, m = c->m;
  std::vector<double> kap;
  if (c->kappa) {
    kap.resize(ipow(n, dim));
    HIP_TRY(hipMemcpyAsync(kap.data(), Lv.kap64, kap.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<double> A((size_t)m * m, 0.0);
  mg_status st = coarse_cholesky(dim, n, c->kappa ? kap.data() : nullptr, c->o.sigma, m, A.data());
  if (st != MG_OK) return st;
  HIP_TRY(hipMemcpyAsync(c->Lc, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MG_OK;
}

// Rows of level l ordered by colour (colour 0 first); within a colour, 3D
// rows run over tiles of kCsrTile x kCsrTile grid rows in (y, z) so that a
// tile's x neighbours stay in L2, lexicographic inside a tile.  Row lengths
// follow from the number of unknown neighbours per direction.
mg_status build_csr(mg_ctx* c, int l, hipStream_t s) {
  Level& Lv = c->lv[l];
  const int dim = c->o.dim, n = Lv.g.n;
  const int rows = Lv.rows;
  std::vector<int> rowmap(rows), rowptr(rows + 1);
  rowptr[0] = 0;
  int idx = 0;
  auto cnt = [&](int i) { return 1 + (i > 1) + (i < n - 1); };
  const int T = dim == 3 ? kCsrTile : n;
  const int kmin = dim == 3 ? 1 : 0, kmax = dim == 3 ? n - 1 : 0;
  // two colours (red-black, sum of coordinates mod 2) or, for multicolour
  // Gauss-Seidel, the 2^dim colours of gs_colour
  const bool gs = c->o.smoother == MG_SMOOTH_GS;
  const int ncol = gs ? (1 << dim) : 2;
  for (int colour = 0; colour < ncol; ++colour) {
    Lv.coff[colour] = idx;
    for (int k0 = kmin; k0 <= kmax; k0 += T)
      for (int j0 = 1; j0 <= n - 1; j0 += T)
        for (int k = k0; k <= std::min(kmax, k0 + T - 1); ++k)
          for (int j = j0; j <= std::min(n - 1, j0 + T - 1); ++j)
            for (int i = 1; i <= n - 1; ++i) {
              if ((gs ? gs_colour(i, j, k) : ((i + j + k) & 1)) != colour) continue;
              rowmap[idx] = (int)(i + j * Lv.g.sy + (long)k * Lv.g.sz);
              const int len = cnt(i) * cnt(j) * (dim == 3 ? cnt(k) : 1);
              rowptr[idx + 1] = rowptr[idx] + len;
              ++idx;
            }
  }
  Lv.coff[ncol] = rows;
  if (idx != rows || rowptr[rows] != Lv.nnz)
    return fail(MG_E_ARG, "internal: CSR layout mismatch on level %d", l);
  HIP_TRY(hipMemcpyAsync(Lv.rowmap, rowmap.data(), rows * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(Lv.rowptr, rowptr.data(), (rows + 1) * sizeof(int),
                         hipMemcpyHostToDevice, s));
  const double selem = dim == 3 ? (1.0 / n) / 12.0 : 1.0 / 6.0;
  const double smass = c->o.sigma * std::pow((1.0 / n) / 6.0, dim);
  HIP_TRY(hipMemsetAsync(Lv.col + Lv.nnz, 0, kCsrPad * sizeof(int), s));
  HIP_TRY(hipMemsetAsync(Lv.val64 + Lv.nnz, 0, kCsrPad * sizeof(double), s));
  if (Lv.val32) HIP_TRY(hipMemsetAsync(Lv.val32 + Lv.nnz, 0, kCsrPad * sizeof(float), s));
  launch_csr_build<double>(Lv.g, Lv.kap64, selem, smass, rows, Lv.rowmap, Lv.rowptr, Lv.col,
                           Lv.val64, s);
  if (Lv.val32)
    launch_csr_build<float>(Lv.g, Lv.kap64, selem, smass, rows, Lv.rowmap, Lv.rowptr, Lv.col,
                            Lv.val32, s);
  HIP_TRY(hipGetLastError());
  // the host vectors must stay alive until the copies finish
  HIP_TRY(hipStreamSynchronize(s));
  auto fill = [&](auto& op, auto* val) {
    op.rowptr = Lv.rowptr;
    op.col = Lv.col;
    op.val = val;
    op.rowmap = Lv.rowmap;
    op.rows = rows;
    for (int q = 0; q < 9; ++q) op.coff[q] = Lv.coff[q];
    op.n = Lv.g.n;
    op.sy = Lv.g.sy;
  };
  fill(Lv.csr64, Lv.val64);
  if (Lv.val32) fill(Lv.csr32, Lv.val32);
  return MG_OK;
}

// Operator kind of the matrix-free levels: per-cell kappa, or constant
// coefficients with (3D) or without face couplings.
int op_kind(const mg_ctx* c) {
  if (c->kappa) return OP_KAPPA;
  return c->o.dim == 3 && c->o.sigma > 0.0 ? OP_MASS : OP_CONST;
}

// Mass weights (h/6)^dim 4^(dim-cls) of the assembled Q1 mass matrix for a
// neighbour class cls = |dx| + |dy| (+ |dz|), and the stiffness weights
// (kappa = 1) of the same classes.
double mass_weight(int dim, double h, int cls) {
  return std::pow(h / 6.0, dim) * (double)(1 << (2 * (dim - cls)));
}
double stiff_weight(int dim, double h, int cls) {
  if (dim == 2) return cls == 0 ? 8.0 / 3.0 : -1.0 / 3.0;
  const double w[4] = {8.0 * h / 3.0, 0.0, -h / 6.0, -h / 12.0};
  return w[cls];
}

// Matrix-free operator of a level with n_l cells (see StencilParams).
StencilParams<double> stencil_of(int dim, int nl, double sg, int kind) {
  const double h = 1.0 / nl;
  double wc, w1, w2, s, wf = 0.0;
  if (dim == 2) {
    wc = 8.0 / 3.0;
    w1 = -1.0 / 3.0;
    w2 = -1.0 / 3.0;
    s = 1.0 / 6.0;
    if (sg > 0.0) {
      wc += sg * mass_weight(2, h, 0);
      w1 += sg * mass_weight(2, h, 1);
      w2 += sg * mass_weight(2, h, 2);
    }
  } else {
    wc = 8.0 * h / 3.0;
    w1 = -h / 6.0;
    w2 = -h / 12.0;
    s = h / 12.0;
    if (sg > 0.0) {
      wc += sg * mass_weight(3, h, 0);
      wf = sg * mass_weight(3, h, 1);
      w1 += sg * mass_weight(3, h, 2);
      w2 += sg * mass_weight(3, h, 3);
    }
  }
  return StencilParams<double>{kind, wc, w1, w2, s, wf};
}

void set_stencil(mg_ctx* c, int l) {
  Level& Lv = c->lv[l];
  const StencilParams<double> p = stencil_of(c->o.dim, Lv.g.n, c->o.sigma, op_kind(c));
  Lv.st64 = p;
  Lv.st32 = StencilParams<float>{p.kind, (float)p.wc, (float)p.w1, (float)p.w2, (float)p.s,
                                 (float)p.wf};
}

// ---------------------------------------------------------------------------
// typed access to per-level buffers and operators
// ---------------------------------------------------------------------------
template <typename T> struct Bufs;
template <> struct Bufs<double> {
  static constexpr int prec = 0;
  static double* x(Level& L) { return L.x64; }
  static double* b(Level& L) { return L.b64; }
  static double* t(Level& L) { return L.t64; }
  static double* r(Level& L) { return L.r64; }
  static const double* kap(Level& L) { return L.kap64; }
  static const StencilParams<double>& st(Level& L) { return L.st64; }
  static const CsrOp<double>* csr(Level& L) { return &L.csr64; }
  static void* tail(mg_ctx* c) { return c->tail64; }
  static double* xs(Level& L, int q) { return L.xs64[q]; }
};
template <> struct Bufs<float> {
  static constexpr int prec = 1;
  static float* x(Level& L) { return L.x32; }
  static float* b(Level& L) { return L.b32; }
  static float* t(Level& L) { return L.t32; }
  static float* r(Level& L) { return L.r32; }
  static const float* kap(Level& L) { return L.kap32; }
  static const StencilParams<float>& st(Level& L) { return L.st32; }
  static const CsrOp<float>* csr(Level& L) { return &L.csr32; }
  static void* tail(mg_ctx* c) { return c->tail32; }
  static float* xs(Level& L, int q) { return L.xs32[q]; }
};

// Descriptor of the tail levels l0..L-1 of a hierarchy: per level (index
// l, absolute) its cells nl[l], operator st[l] and device coefficients
// kap[l] (OP_KAPPA); the coarsest factor Lc (m x m, device); r0buf: the
// device vector that holds level l0's residual when the LDS cannot (the
// level's node count).  Sets D.lds_bytes; fails when the levels exceed the
// tail's LDS budget.
template <typename T>
mg_status fill_tail_desc(const mg_options& o, int L, int l0, bool kappa, int m, const double* Lc,
                         const int* nl, const StencilParams<T>* st, const T* const* kap,
                         T* r0buf, TailDesc<T>& D) {
  D = TailDesc<T>{};
  D.nlev = L - l0;
  D.dim = o.dim;
  D.kind = st[l0].kind;
  D.smoother = o.smoother == MG_SMOOTH_JACOBI ? 0 : (o.smoother == MG_SMOOTH_GS ? 2 : 1);
  D.nu_pre = o.nu_pre;
  D.nu_post = o.nu_post;
  D.omega = (T)o.omega;
  D.m = m;
  D.L = Lc;
  // LDS layout (16-byte aligned pieces): per level iterate, spare,
  // right-hand side, residual (and cells), then the coarsest solve's
  // work vector; offsets of level vectors in elements of T
  long off = 0;
  auto take = [&](long bytes) {
    const long at = off;
    off += (bytes + 15) / 16 * 16;
    return at;
  };
  // the first level's residual goes to device memory when all else fits
  // the LDS only without it
  const bool r0_global =
      tail_lds_bytes(o.dim, o.n, L, l0, kappa, (int)sizeof(T), false) > kTailLdsBytes;
  D.r0 = r0_global ? r0buf : nullptr;
  for (int q = 0; q < D.nlev; ++q) {
    const int l = l0 + q;
    const Geo g = make_geo(o.dim, nl[l]);
    const long vb = g.nodes * (long)sizeof(T);
    TailLevel<T>& tl = D.lv[q];
    tl.n = g.n;
    tl.ox = (int)(take(vb) / sizeof(T));
    tl.ot = (int)(take(vb) / sizeof(T));
    tl.ob = (int)(take(vb) / sizeof(T));
    tl.orr = (q == 0 && r0_global) ? 0 : (int)(take(vb) / sizeof(T));
    tl.ok = kappa ? (int)(take(ipow(g.n, o.dim) * (long)sizeof(T)) / sizeof(T)) : 0;
    tl.kappa = kap[l];
    tl.wc = st[l].wc;
    tl.w1 = st[l].w1;
    tl.w2 = st[l].w2;
    tl.s = st[l].s;
    tl.wf = st[l].wf;
  }
  D.oy = (int)take((long)m * sizeof(double));
  if (off > kTailLdsBytes) return fail(MG_E_ARG, "internal: tail levels exceed the LDS budget");
  D.lds_bytes = (int)off;
  return MG_OK;
}

template <typename T>
mg_status build_tail(mg_ctx* c, hipStream_t s) {
  const int l0 = c->tail0;
  TailDesc<T> D{};
  if (l0 >= 0) {
    std::vector<int> nl(c->L);
    std::vector<StencilParams<T>> st(c->L);
    std::vector<const T*> kap(c->L);
    for (int l = 0; l < c->L; ++l) {
      nl[l] = c->lv[l].g.n;
      st[l] = Bufs<T>::st(c->lv[l]);
      kap[l] = Bufs<T>::kap(c->lv[l]);
    }
    mg_status r = fill_tail_desc<T>(c->o, c->L, l0, c->kappa, c->m, c->Lc, nl.data(), st.data(),
                                    kap.data(), Bufs<T>::r(c->lv[l0]), D);
    if (r != MG_OK) return r;
  }
  c->tail_lds[Bufs<T>::prec] = D.lds_bytes;
  HIP_TRY(hipMemcpyAsync(Bufs<T>::tail(c), &D, sizeof D, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MG_OK;
}

// ---------------------------------------------------------------------------
// recorded ops of one cycle
// ---------------------------------------------------------------------------
using Sink = std::function<void(const OpRec&)>;

template <typename T>
OpRec base_op(mg_ctx* c, int code, int l) {
  OpRec o;
  o.code = code;
  o.prec = Bufs<T>::prec;
  o.level = l;
  Level& Lv = c->lv[l];
  o.g = Lv.g;
  if (l + 1 < c->L) o.gc = c->lv[l + 1].g;
  const StencilParams<T>& st = Bufs<T>::st(Lv);
  o.opkind = st.kind;
  o.wc = st.wc;
  o.w1 = st.w1;
  o.w2 = st.w2;
  o.s = st.s;
  o.wf = st.wf;
  o.omega = (T)c->o.omega;
  o.m = c->m;
  o.item.kappa = Bufs<T>::kap(Lv);
  o.item.lay = b_split_half(c, l, Bufs<T>::prec);
  return o;
}

// Whether the red-black runs on level l keep the iterate colour-split (the
// level has split-iterate buffers of this precision).
template <typename T>
bool split_iterate(const mg_ctx* c, int l) {
  const Level& Lv = c->lv[l];
  return !c->csr && c->o.smoother == MG_SMOOTH_RBGS && !(c->o.flags & MG_FLAG_PAIR) &&
         use_split_x(Lv.g) && (std::is_same<T, double>::value ? (void*)Lv.xs64[0]
                                                               : (void*)Lv.xs32[0]) != nullptr;
}

template <typename T>
void emit_smooth(mg_ctx* c, const Sink& sink, int l, int kind, const T* xin, const T* b,
                 T* xout) {
  OpRec o = base_op<T>(c, c->csr ? OC_CSR_SMOOTH : OC_SMOOTH, l);
  o.sub = kind | ((xin == nullptr) << 4);
  o.item.a = xin;
  o.item.b = b;
  o.item.c = xout;
  if (c->csr) o.csr = Bufs<T>::csr(c->lv[l]);
  sink(o);
}

template <typename T>
void emit_residual(mg_ctx* c, const Sink& sink, int l, const T* x, const T* b, T* r,
                   double* partials, const int* split = nullptr) {
  OpRec o = base_op<T>(c, c->csr ? OC_CSR_RESID : OC_RESID, l);
  o.sub = partials != nullptr;
  o.item.a = x;
  o.item.b = b;
  o.item.c = r;
  if (split) {
    // x colour-split: even half in buffer split[0], odd half in split[1]
    Level& Lv = c->lv[l];
    o.sub |= XL_SPLIT << 5;
    o.item.a = Bufs<T>::xs(Lv, split[0]);
    o.item.a2 = Bufs<T>::xs(Lv, split[1]) + (Lv.g.nodes + 1) / 2;
  }
  o.item.partials = partials;
  if (c->csr) o.csr = Bufs<T>::csr(c->lv[l]);
  sink(o);
}

// Whether the residual of level l and its restriction run as one pass
// (k_resid_restrict3): 3D matrix-free levels k_sweep3 runs, constant or
// mass-shifted operator, not with MG_FLAG_NO_FUSE.
template <typename T>
bool fuse_resid_restrict(const mg_ctx* c, int l) {
  const Level& Lv = c->lv[l];
  return !c->csr && !(c->o.flags & MG_FLAG_NO_FUSE) && l + 1 < c->L && use_split_x(Lv.g) &&
         Bufs<T>::st(const_cast<Level&>(Lv)).kind != OP_KAPPA;
}

// b_{l+1} = R (b - A x) on level l (into bc_out, else the level's b): one
// pass where fuse_resid_restrict (plus the few coarse columns it leaves),
// else the residual into the level's r and the restriction.  split: x
// colour-split, even half in buffer split[0], odd half in split[1].
template <typename T>
void emit_resid_restrict(mg_ctx* c, const Sink& sink, int l, const T* x, const T* b,
                         const int* split, T* bc_out = nullptr) {
  Level& Lv = c->lv[l];
  T* const r = Bufs<T>::r(Lv);
  T* const bc = bc_out ? bc_out : Bufs<T>::b(c->lv[l + 1]);
  const long clay = b_split_half(c, l + 1, Bufs<T>::prec);  // the coarse b's layout
  if (fuse_resid_restrict<T>(c, l)) {
    OpRec o = base_op<T>(c, OC_RESID_RESTRICT, l);
    o.item.a = x;
    o.item.b = b;
    o.item.c = bc;
    o.item.e = r;
    o.item.flag = clay != 0;
    if (split) {
      o.sub = 1;
      o.item.a = Bufs<T>::xs(Lv, split[0]);
      o.item.a2 = Bufs<T>::xs(Lv, split[1]) + (Lv.g.nodes + 1) / 2;
    }
    sink(o);
    if (resid_restrict_xcols(Lv.g) > 0) {
      OpRec f = base_op<T>(c, OC_RESTRICT_XCOLS, l);
      f.item.lay = clay;
      f.item.a = r;
      f.item.c = bc;
      sink(f);
    }
    return;
  }
  emit_residual<T>(c, sink, l, x, b, r, nullptr, split);
  OpRec o = base_op<T>(c, OC_RESTRICT, l);
  o.item.lay = clay;
  o.item.a = r;
  o.item.c = bc;
  sink(o);
}

// Partial sums of ||b - A x||^2 on level l and, into xout, the first
// pre-smoothing step of the next cycle from x.
template <typename T>
void emit_head(mg_ctx* c, const Sink& sink, int l, const T* x, const T* b, T* xout,
               double* partials, bool in_split = false) {
  OpRec o = base_op<T>(c, c->csr ? OC_CSR_HEAD : OC_HEAD, l);
  o.sub = c->o.smoother == MG_SMOOTH_JACOBI ? SM_JACOBI : SM_RB0;
  o.item.a = x;
  o.item.b = b;
  o.item.c = xout;
  o.item.partials = partials;
  if (c->csr) o.csr = Bufs<T>::csr(c->lv[l]);
  if (split_iterate<T>(c, l)) {
    // the next cycle's smoothing run continues from the split halves
    Level& Lv = c->lv[l];
    const long lay = (Lv.g.nodes + 1) / 2;
    if (in_split) {
      // x split (halves in c->s0at); the updated colour 0 goes to the
      // even half of the other buffer, x itself stays where it is
      o.sub |= XL_SPLIT << 5;
      o.item.a = Bufs<T>::xs(Lv, c->s0at[0]);
      o.item.a2 = Bufs<T>::xs(Lv, c->s0at[1]) + lay;
      c->s0at[0] = 1 - c->s0at[0];
      o.item.c = Bufs<T>::xs(Lv, c->s0at[0]);
    } else {
      o.sub |= XL_TO_SPLIT << 5;
      o.item.c = Bufs<T>::xs(Lv, 0);
      o.item.c2 = Bufs<T>::xs(Lv, 0) + lay;
      c->s0at[0] = c->s0at[1] = 0;
    }
  }
  sink(o);
}

long residual_partials(mg_ctx* c, int l) {
  return c->csr ? csr_residual_blocks(c->lv[l].rows) : grid_blocks(c->lv[l].g);
}

void emit_reduce(mg_ctx* c, const Sink& sink, long count, double* out, double* part = nullptr) {
  OpRec o = base_op<double>(c, OC_REDUCE, 0);
  o.count = count;
  o.item.partials = part ? part : c->partials;
  o.item.scal = out;
  sink(o);
}

template <typename T>
void emit_fill(mg_ctx* c, const Sink& sink, int l, T* v) {
  OpRec o = base_op<T>(c, OC_FILL, l);
  o.count = c->lv[l].g.nodes;
  o.item.c = v;
  sink(o);
}

// A run of red-black half-sweeps (steps) on a level with colour-split
// iterate buffers xs[0..1]: the first step reads *cur (or x = 0) and writes
// both halves of xs[0] (from_split: the iterate is already split -- a fused
// step before the run, the head or the prolongation, has written it); each
// middle step reads the current even and odd halves and writes only the
// updated colour's half, into the buffer that does not hold that colour's
// current half; the last step writes the natural iterate where the
// ping-pong of natural steps would have left it (*cur after an even number
// of steps, else *spare) -- or, with end_split, stays split like a middle
// step.  state (in/out, or nullptr for a run of its own): the buffer
// holding the even / odd half.  Every node gets the arithmetic of the
// natural steps, so the result is bitwise theirs; the middle steps do not
// copy the other colour.
template <typename T>
void emit_split_run(mg_ctx* c, const Sink& sink, int l, const std::vector<int>& steps, T** cur,
                    T** spare, bool* zero, const T* b, bool from_split = false,
                    int* state = nullptr, bool end_split = false) {
  Level& Lv = c->lv[l];
  T* xs[2] = {Bufs<T>::xs(Lv, 0), Bufs<T>::xs(Lv, 1)};
  const long lay = (Lv.g.nodes + 1) / 2;  // start of the odd half
  int local[2] = {0, 0};
  int* at = state ? state : local;         // buffer holding the even / odd half
  if (steps.empty()) return;
  const size_t last = steps.size() - 1;
  const bool back = steps.size() % 2 == 0;
  for (size_t q = 0; q <= last; ++q) {
    const int col = steps[q] == SM_RB1 ? 1 : 0;  // parity of the updated nodes
    const bool first = q == 0 && !from_split;
    const bool z = first && *zero;
    const int xl =
        first ? XL_TO_SPLIT : (q == last && !end_split ? XL_TO_NATURAL : XL_SPLIT);
    OpRec o = base_op<T>(c, OC_SMOOTH, l);
    o.sub = steps[q] | ((z ? 1 : 0) << 4) | (xl << 5);
    o.item.b = b;
    if (first) {
      o.item.a = z ? nullptr : *cur;
      o.item.c = xs[0] + (col ? lay : 0);
      o.item.c2 = xs[0] + (col ? 0 : lay);
      at[0] = at[1] = 0;
    } else {
      o.item.a = xs[at[0]];
      o.item.a2 = xs[at[1]] + lay;
      if (xl == XL_TO_NATURAL) {
        o.item.c = back ? *cur : *spare;
      } else {
        const int dst = 1 - at[col];
        o.item.c = xs[dst] + (col ? lay : 0);
        at[col] = dst;
      }
    }
    sink(o);
  }
  if (!end_split && !back) std::swap(*cur, *spare);
  *zero = false;
}

// Smoothing on level l from *cur (or from 0 if *zero), ping-ponging between
// *cur and *spare; on return *cur holds the smoothed iterate.  With
// `skip`, the first step is not emitted: it has already been done, from
// *spare into *cur.  With MG_FLAG_PAIR, consecutive red-black half-sweeps
// on the large 3D stencil levels go out as pairs (one pass each, bitwise
// the same result).  state: the run is a split run whose halves are
// tracked there (see emit_split_run), ending split unless !end_split.
template <typename T>
void smooth_level(mg_ctx* c, const Sink& sink, int l, bool pre, T** cur, T** spare, bool* zero,
                  const T* b, bool skip = false, bool from_split = false,
                  int* state = nullptr, bool end_split = true) {
  const int nu = pre ? c->o.nu_pre : c->o.nu_post;
  if (c->o.smoother == MG_SMOOTH_GS) {
    // multicolour Gauss-Seidel: one in-place launch per colour, colours in
    // order for pre-smoothing and in reverse order for post-smoothing
    if (nu == 0) return;
    if (*zero) {
      emit_fill<T>(c, sink, l, *cur);
      *zero = false;
    }
    const int ncol = 1 << c->o.dim;
    for (int it = 0; it < nu; ++it)
      for (int q = 0; q < ncol; ++q)
        emit_smooth<T>(c, sink, l, SM_GS0 + (pre ? q : ncol - 1 - q), *cur, b, *cur);
    return;
  }
  std::vector<int> steps;
  for (int it = 0; it < nu; ++it) {
    if (c->o.smoother == MG_SMOOTH_JACOBI) {
      steps.push_back(SM_JACOBI);
    } else {
      steps.push_back(pre ? SM_RB0 : SM_RB1);
      steps.push_back(pre ? SM_RB1 : SM_RB0);
    }
  }
  if (skip && !steps.empty()) steps.erase(steps.begin());
  const bool pairs = !c->csr && c->o.smoother == MG_SMOOTH_RBGS &&
                     pair_sweeps(c->lv[l].g) && (c->o.flags & MG_FLAG_PAIR);
  if (state) {
    // the iterate is colour-split before the run (or starts it) and stays
    // split after it unless !end_split
    emit_split_run<T>(c, sink, l, steps, cur, spare, zero, b, from_split, state, end_split);
    return;
  }
  if (from_split) {
    emit_split_run<T>(c, sink, l, steps, cur, spare, zero, b, true);
    return;
  }
  if (!pairs && steps.size() >= 3 && split_iterate<T>(c, l)) {
    emit_split_run<T>(c, sink, l, steps, cur, spare, zero, b);
    return;
  }
  for (size_t q = 0; q < steps.size();) {
    if (pairs && q + 1 < steps.size()) {
      OpRec o = base_op<T>(c, OC_SMOOTH2, l);
      o.sub = steps[q] | ((*zero ? 1 : 0) << 4);
      o.item.a = *zero ? nullptr : *cur;
      o.item.b = b;
      o.item.c = *spare;
      sink(o);
      q += 2;
    } else {
      emit_smooth<T>(c, sink, l, steps[q], *zero ? nullptr : *cur, b, *spare);
      q += 1;
    }
    std::swap(*cur, *spare);
    *zero = false;
  }
}

// Coarse-level cycles that solve a level's coarse residual equation, per
// cycle kind (mg_cycle): V one V-cycle, W two W-cycles, F an F-cycle then a
// V-cycle; directly above the coarsest level one exact solve.
static_assert(MG_CYCLE_V == CYC_V && MG_CYCLE_W == CYC_W && MG_CYCLE_F == CYC_F,
              "cycle kinds of the tail kernel");
inline int cycle_subs(int kind) { return kind == MG_CYCLE_V ? 1 : 2; }
inline int cycle_sub(int kind, int i) {
  return kind == MG_CYCLE_W ? MG_CYCLE_W : (kind == MG_CYCLE_F && i == 0 ? MG_CYCLE_F : MG_CYCLE_V);
}

template <typename T>
bool fuse_prolongation(const mg_ctx* c, int l);

// One cycle of the context's kind (Algorithm 1 for the V-cycle) for
// A_0 x = b starting from x0 (or from 0 when x0_zero); the result is
// written back to x0.  Levels >= 1 and the spare level-0 buffer are
// internal.  Levels from c->tail0 on run in one workgroup per request (the
// tail kernel follows the same schedule).  head_done: the first level-0
// pre-smoothing step has already been applied to x0, its result is in
// spare0.  split0 (with c->s0on): the level-0 iterate stays colour-split
// through the cycle -- it starts in the halves c->s0at (after the head, or
// from 0), the residual and the fused prolongation read it split, and the
// result stays in the halves (recorded in c->s0u); x0 is not written.
// iru_u (FP32 cycles of iterative refinement): where the level-0 post-smoothing
// ends with a smoothing step that writes a natural iterate on a k_sweep3
// level, that step adds ir_scale(scal[1]) times its result to the FP64
// iterate iru_u instead of writing x0 (*iru_done is set then; x0 is not
// written).
template <typename T>
void emit_vcycle(mg_ctx* c, const Sink& sink, T* x0, T* spare0, const T* b0, bool x0_zero,
                 bool head_done = false, bool split0 = false, double* iru_u = nullptr,
                 bool* iru_done = nullptr) {
  if (iru_done) *iru_done = false;
  const int L = c->L;
  std::vector<T*> cur(L), spare(L);
  std::vector<const T*> bb(L);
  cur[0] = x0;
  spare[0] = spare0;
  bb[0] = b0;
  for (int l = 1; l < L; ++l) {
    cur[l] = Bufs<T>::x(c->lv[l]);
    spare[l] = Bufs<T>::t(c->lv[l]);
    bb[l] = Bufs<T>::b(c->lv[l]);
  }
  const int lt = c->tail0 >= 0 ? c->tail0 : L - 1;  // first level not cycled level by level
  if (head_done) std::swap(cur[0], spare[0]);
  // one visit of level l by a cycle of `kind`, its iterate starting at 0
  // when `zero`
  // level-0 post-smoothing ops are collected first (see iru_u)
  std::vector<OpRec> post0;
  const Sink collect0 = [&post0](const OpRec& o) { post0.push_back(o); };
  std::function<void(int, int, bool)> visit = [&](int l, int kind, bool zero) {
    if (l == lt) {
      if (c->tail0 >= 0) {
        OpRec o = base_op<T>(c, OC_TAIL, lt);
        o.count = c->tail_lds[Bufs<T>::prec];
        o.item.a = Bufs<T>::tail(c);
        o.item.b = bb[lt];
        o.item.c = cur[lt];
        o.item.flag = (zero ? 1 : 0) | (kind << 1);
        sink(o);
      } else {
        OpRec o = base_op<T>(c, OC_COARSE, L - 1);
        o.item.b = bb[L - 1];
        o.item.c = cur[L - 1];
        o.item.L = c->Lc;
        sink(o);
      }
      return;
    }
    bool z = zero;
    const bool s0 = l == 0 && split0;  // (head fusion: at least one pre-smoothing step)
    // Otherwise, on a level-0 visit that starts from a natural iterate or
    // from 0 (the FP32 cycles of refinement, the cycles of CG), the
    // iterate stays colour-split from the pre-smoothing through the
    // residual and the fused prolongation into the post-smoothing, whose
    // last step writes it natural: halves tracked in spat
    int spat[2] = {0, 0};
    const bool sp = l == 0 && !split0 && !head_done && c->o.smoother == MG_SMOOTH_RBGS &&
                    c->o.nu_pre >= 1 && split_iterate<T>(c, 0) && fuse_prolongation<T>(c, 0);
    int* const sat = s0 ? c->s0at : (sp ? spat : nullptr);
    smooth_level<T>(c, sink, l, true, &cur[l], &spare[l], &z, bb[l], l == 0 && head_done,
                    l == 0 && head_done && split_iterate<T>(c, 0), sat);
    if (z) emit_fill<T>(c, sink, l, cur[l]);  // no pre-smoothing: x = 0
    emit_resid_restrict<T>(c, sink, l, cur[l], bb[l], sat);
    if (l + 1 == L - 1) {
      visit(l + 1, kind, true);
    } else {
      for (int i = 0; i < cycle_subs(kind); ++i) visit(l + 1, cycle_sub(kind, i), i == 0);
    }
    // the prolongation fused into the first post-smoothing step where that
    // pays (bitwise the same as the separate launches)
    const bool fuse_pro = fuse_prolongation<T>(c, l);
    bool nz = false;
    if (fuse_pro) {
      OpRec o = base_op<T>(c, OC_SMOOTH_PRO, l);
      o.sub = c->o.smoother == MG_SMOOTH_JACOBI ? SM_JACOBI : SM_RB1;
      o.item.a = cur[l];
      o.item.e = cur[l + 1];
      o.item.b = bb[l];
      o.item.c = spare[l];
      const bool sx = split_iterate<T>(c, l);
      Level& Lv = c->lv[l];
      const long lay = (Lv.g.nodes + 1) / 2;
      if (sat) {
        // x split in the halves sat; x + P e changes every node, so both
        // halves go to the other buffers (colour 1 updated)
        o.sub |= XL_SPLIT_BOTH << 5;
        o.item.a = Bufs<T>::xs(Lv, sat[0]);
        o.item.a2 = Bufs<T>::xs(Lv, sat[1]) + lay;
        sat[0] = 1 - sat[0];
        sat[1] = 1 - sat[1];
        o.item.c = Bufs<T>::xs(Lv, sat[1]) + lay;
        o.item.c2 = Bufs<T>::xs(Lv, sat[0]);
      } else if (sx) {
        // colour 1 updated into the odd half, colour 0 copied to the even one
        o.sub |= XL_TO_SPLIT << 5;
        o.item.c = Bufs<T>::xs(Lv, 0) + lay;
        o.item.c2 = Bufs<T>::xs(Lv, 0);
      }
      sink(o);
      std::swap(cur[l], spare[l]);
      smooth_level<T>(c, l == 0 && iru_u ? collect0 : sink, l, false, &cur[l], &spare[l], &nz,
                      bb[l], true, sx || sat, sat, s0);
      if (s0) {
        c->s0u[0] = c->s0at[0];
        c->s0u[1] = c->s0at[1];
      }
    } else {
      OpRec pr = base_op<T>(c, OC_PROLONG, l);
      pr.item.a = cur[l + 1];
      pr.item.c = cur[l];
      sink(pr);
      smooth_level<T>(c, l == 0 && iru_u ? collect0 : sink, l, false, &cur[l], &spare[l], &nz,
                      bb[l]);
    }
    if (l == 0 && iru_u) {
      // the refinement update fused into the last step, where possible
      if (!post0.empty()) {
        OpRec& z = post0.back();
        const int kd = z.sub & 15, xl = (z.sub >> 5) & 7;
        if (std::is_same<T, float>::value && z.code == OC_SMOOTH && use_split_x(z.g) &&
            (kd == SM_JACOBI || kd == SM_RB0 || kd == SM_RB1) && !((z.sub >> 4) & 1) &&
            (xl == XL_NATURAL || xl == XL_TO_NATURAL)) {
          z.sub |= 1 << 8;
          z.item.c = iru_u;
          z.item.scal = c->scal + 1;
          *iru_done = true;
        }
      }
      for (const OpRec& o : post0) sink(o);
    }
  };
  visit(0, c->o.cycle, x0_zero);
  if (!split0 && !(iru_done && *iru_done) && cur[0] != x0) {
    OpRec o = base_op<T>(c, OC_COPY, 0);
    o.count = c->lv[0].g.nodes;
    o.item.a = cur[0];
    o.item.c = x0;
    sink(o);
  }
}

// Whether FP64 solves fuse the stopping residual of cycle k with the first
// pre-smoothing step of cycle k+1 (both read A and u_k once): needs a
// level-0 pre-smoothing step outside the tail.
bool head_fusion(const mg_ctx* c) {
  return !c->ir && c->o.nu_pre >= 1 && c->L >= 2 && c->tail0 != 0 &&
         c->o.smoother != MG_SMOOTH_GS &&
         !(c->o.flags & MG_FLAG_NO_FUSE);
}

// Whether the prolongation into level l is fused into its first
// post-smoothing step: the 3D stencil levels k_sweep3 runs; with per-cell
// kappa only in FP64 (the 192^3 kappa solve 12.65 -> 12.37 ms; in the FP32
// cycles the fused kappa kernel's register and LDS use cost about what the
// pass saves: 9.73 -> 9.77 ms).
template <typename T>
bool fuse_prolongation(const mg_ctx* c, int l) {
  return !c->csr && (!c->kappa || sizeof(T) == 8) && c->o.nu_post >= 1 &&
         c->o.smoother != MG_SMOOTH_GS &&
         pair_sweeps(c->lv[l].g) && !(c->o.flags & (MG_FLAG_PAIR | MG_FLAG_NO_FUSE));
}

// Whether an FP64 solve with head fusion keeps the finest iterate
// colour-split from cycle to cycle (see mg_ctx::s0on): the finest level has
// split iterates, and both its fused steps (head, prolongation) are there
// to read and write the halves.
bool split_persist(const mg_ctx* c) {
  return head_fusion(c) && split_iterate<double>(c, 0) && fuse_prolongation<double>(c, 0);
}

// Iteration kinds: IT_PLAIN = V-cycle, then residual norm;  IT_FUSED_FIRST =
// V-cycle, then the fused residual norm + next head (into the level-0
// spare);  IT_FUSED = the V-cycle without its head (taken from the spare),
// then the fused residual norm + next head.  In every kind u holds the new
// iterate and scal[0] its squared residual norm at the end.
enum IterKind { IT_PLAIN = 0, IT_FUSED_FIRST = 1, IT_FUSED = 2, IT_PCG_FIRST = 3, IT_PCG = 4 };

// One CG vector kernel on level-0 vectors (see kernels_pcg.hip).
void emit_pcg_op(mg_ctx* c, const Sink& sink, int sub, std::initializer_list<void*> vecs,
                 long count, int flag = 0) {
  OpRec o = base_op<double>(c, OC_PCG, 0);
  o.sub = sub;
  o.count = count;
  o.item.flag = flag;
  o.item.scal = c->scal;
  o.item.partials = c->partials;
  int q = 0;
  for (void* v : vecs) o.ext[q++] = v;
  sink(o);
}

// Conjugate gradients preconditioned by one V-cycle, one iteration (the
// steps in the order of the oracle's solve_pcg, with the preconditioner
// application of iteration k-1 moved to the front of iteration k so that
// the residual norm is the last value of an iteration):
//   z = B r;  beta = (z.r - z.r_old) / rz (0 first);  rz = z.r;
//   p = z + beta p (p = z first);  q = A p;  alpha = rz / p.q;
//   u += alpha p;  r_old = r;  r -= alpha q;  ||r||^2 into scal[0].
// B is the V-cycle from a zero guess on A z = r (FP64), or in FP32 on
// r / s scaled back by s = ir_scale(||r||^2).  r lives in its own vector:
// the cycle uses the level's residual buffer internally.
void emit_pcg_iteration(mg_ctx* c, const Sink& sink, double* u, bool first) {
  Level& L0 = c->lv[0];
  const long N = L0.g.nodes;
  double* S = c->scal;
  if (c->ir) {
    OpRec o = base_op<double>(c, OC_SCALE_CAST, 0);
    o.item.lay = b_split_half(c, 0, 1);  // the FP32 right-hand side it writes
    o.item.a = L0.rk64;
    o.item.c = L0.b32;
    o.item.scal = S + 0;
    sink(o);
    emit_vcycle<float>(c, sink, L0.x32, L0.t32, L0.b32, true);
    emit_pcg_op(c, sink, PO_ZSCALE, {L0.x32, L0.z64}, N);
  } else {
    emit_vcycle<double>(c, sink, L0.z64, L0.t64, L0.rk64, true);
  }
  const long PB = pcg_blocks(N);
  emit_pcg_op(c, sink, PO_DOTS2, {L0.z64, L0.rk64, L0.ro64}, N);
  emit_reduce(c, sink, PB, S + PCG_ZR, c->partials);
  emit_reduce(c, sink, PB, S + PCG_ZRO, c->partials + PB);
  emit_pcg_op(c, sink, PO_SCALARS, {}, 0, first);
  emit_pcg_op(c, sink, PO_DIR, {L0.z64, L0.p64}, N, first);
  OpRec a = base_op<double>(c, c->csr ? OC_CSR_APPLY_DOT : OC_APPLY_DOT, 0);
  a.item.a = L0.p64;
  a.item.c = L0.q64;
  a.item.partials = c->partials;
  if (c->csr) a.csr = Bufs<double>::csr(L0);
  sink(a);
  emit_reduce(c, sink, residual_partials(c, 0), S + PCG_PQ, c->partials);
  emit_pcg_op(c, sink, PO_UPDATE, {u, L0.p64, L0.rk64, L0.ro64, L0.q64}, N);
  emit_reduce(c, sink, PB, S + 0, c->partials);
}

// Iterative refinement: the partial sums of ||b - A u||^2 and the FP32
// cycle's right-hand side b32 = float(r / s), s = ir_scale(scal[1] =
// ||b||^2) -- in one residual pass on k_sweep3 levels (r is not stored;
// not with MG_FLAG_NO_FUSE), else r into r64 and a scaled-cast launch.
// Both give the same b32 bitwise.
void emit_ir_residual(mg_ctx* c, const Sink& sink, double* u, const double* b) {
  Level& L0 = c->lv[0];
  const long lay32 = b_split_half(c, 0, 1);  // layout of b32
  if (!c->csr && use_split_x(L0.g) && !(c->o.flags & MG_FLAG_NO_FUSE) &&
      b_split_half(c, 0, 0) == 0) {
    OpRec o = base_op<double>(c, OC_RESID, 0);
    o.sub = 1 | (1 << 9);  // with the partial sums; the scaled cast
    o.item.a = u;
    o.item.b = b;
    o.item.c = L0.b32;
    o.item.lay = lay32;
    o.item.scal = c->scal + 1;
    o.item.partials = c->partials;
    sink(o);
    return;
  }
  emit_residual<double>(c, sink, 0, u, b, L0.r64, c->partials);
  OpRec o = base_op<double>(c, OC_SCALE_CAST, 0);
  o.item.lay = lay32;
  o.item.a = L0.r64;
  o.item.c = L0.b32;
  o.item.scal = c->scal + 1;
  sink(o);
}

// u = 0, or for a warm start u's boundary entries = 0.
void emit_start(mg_ctx* c, const Sink& sink, double* u, bool warm) {
  if (!warm) {
    emit_fill<double>(c, sink, 0, u);
    return;
  }
  OpRec z = base_op<double>(c, OC_ZERO_BOUNDARY, 0);
  z.item.c = u;
  sink(z);
}

// Start of a CG solve: u = 0 (or the warm start), ||b||^2 into scal[1],
// r = b - A u (the vector kernels also stream boundary entries, which stay
// 0) with ||r||^2 into scal[0].
void emit_pcg_prologue(mg_ctx* c, const Sink& sink, double* u, const double* b, bool warm) {
  Level& L0 = c->lv[0];
  emit_start(c, sink, u, warm);
  OpRec o = base_op<double>(c, OC_NORM2, 0);
  o.item.a = b;
  o.item.partials = c->partials;
  sink(o);
  emit_reduce(c, sink, norm2_blocks(L0.g), c->scal + 1);
  emit_residual<double>(c, sink, 0, u, b, L0.rk64, c->partials);
  emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
}

void emit_iteration(mg_ctx* c, const Sink& sink, double* u, const double* b,
                    int kind = IT_PLAIN) {
  Level& L0 = c->lv[0];
  if (kind == IT_PCG_FIRST || kind == IT_PCG) {
    emit_pcg_iteration(c, sink, u, kind == IT_PCG_FIRST);
    return;
  }
  if (kind != IT_PLAIN) {
    if (c->s0on) {
      // the finest iterate stays split (the first cycle starts from 0)
      emit_vcycle<double>(c, sink, u, L0.t64, b, kind == IT_FUSED_FIRST, kind == IT_FUSED,
                          true);
      emit_head<double>(c, sink, 0, u, b, L0.t64, c->partials, true);
    } else {
      emit_vcycle<double>(c, sink, u, L0.t64, b, false, kind == IT_FUSED);
      emit_head<double>(c, sink, 0, u, b, L0.t64, c->partials);
    }
    emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
    return;
  }
  if (c->ir) {
    // c = V-cycle32(0, b32), u += s c (b32 = float(r / s) from the residual
    // of the previous iteration or the prologue, s = ir_scale(||b||^2)); the
    // update fused into the cycle's last level-0 step where that is a
    // k_sweep3 step (not with MG_FLAG_NO_FUSE)
    const bool nf = (c->o.flags & MG_FLAG_NO_FUSE) != 0;
    bool fused = false;
    emit_vcycle<float>(c, sink, L0.x32, L0.t32, L0.b32, true, false, false, nf ? nullptr : u,
                       &fused);
    if (!fused) {
      OpRec up = base_op<double>(c, OC_IR_UPDATE, 0);
      up.item.a = L0.x32;
      up.item.c = u;
      up.item.scal = c->scal + 1;
      sink(up);
    }
    emit_ir_residual(c, sink, u, b);
  } else {
    emit_vcycle<double>(c, sink, u, L0.t64, b, false);
    // r = b - A u and ||r||^2 into scal[0]
    emit_residual<double>(c, sink, 0, u, b, L0.r64, c->partials);
  }
  emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
}

// Start of a solve: u = 0 (or the warm start), ||b||^2 into scal[1]; for
// FP32 refinement and for a warm start also ||b - A u||^2 into scal[0] --
// for a warm-started solve with head fusion in one pass with the first
// smoothing step of the first cycle (into the level-0 spare, as at the end
// of an IT_FUSED_FIRST iteration), else with the residual in r64.
// norm_ready: the partial sums of ||b||^2 are already in c->partials.
void emit_prologue(mg_ctx* c, const Sink& sink, double* u, const double* b, bool warm = false,
                   bool fuse = false, bool norm_ready = false) {
  Level& L0 = c->lv[0];
  // (a solve whose finest iterate stays split from 0 writes u only after
  // its last cycle; mg_solve fills u itself when no cycle runs)
  if (warm || !c->s0on) emit_start(c, sink, u, warm);
  if (!norm_ready) {
    OpRec o = base_op<double>(c, OC_NORM2, 0);
    o.item.a = b;
    o.item.partials = c->partials;
    sink(o);
  }
  emit_reduce(c, sink, norm2_blocks(L0.g), c->scal + 1);
  if (warm && fuse) {
    emit_head<double>(c, sink, 0, u, b, L0.t64, c->partials);
    emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
  } else if (c->ir) {
    emit_ir_residual(c, sink, u, b);
    emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
  } else if (warm) {
    emit_residual<double>(c, sink, 0, u, b, L0.r64, c->partials);
    emit_reduce(c, sink, residual_partials(c, 0), c->scal + 0);
  }
}

// profiling hooks: bracket level-0 launches of the selected kernel class
enum ProfKind {
  PK_SMOOTH = 0, PK_RESID = 1, PK_RESTRICT = 2, PK_PROLONG = 3, PK_SMOOTH2 = 4, PK_SMOOTH_PRO = 5,
  PK_SMOOTH_IR = 6, PK_RESID_RESTRICT = 7, PK_SMOOTH_ZERO = 8
};

int prof_class(const OpRec& o) {
  switch (o.code) {
    case OC_SMOOTH:
      return (o.sub >> 8) & 1 ? PK_SMOOTH_IR : ((o.sub >> 4) & 1 ? PK_SMOOTH_ZERO : PK_SMOOTH);
    case OC_CSR_SMOOTH: return o.sub >> 4 ? PK_SMOOTH_ZERO : PK_SMOOTH;
    case OC_SMOOTH2: return PK_SMOOTH2;
    case OC_SMOOTH_PRO: return PK_SMOOTH_PRO;
    case OC_RESID:
    case OC_CSR_RESID:
    case OC_HEAD:
    case OC_CSR_HEAD:
    case OC_APPLY_DOT:
    case OC_CSR_APPLY_DOT: return PK_RESID;
    case OC_RESTRICT:
    case OC_RESTRICT_XCOLS: return PK_RESTRICT;
    case OC_RESID_RESTRICT: return PK_RESID_RESTRICT;
    case OC_PROLONG: return PK_PROLONG;
    default: return -1;
  }
}

hipEvent_t take_event(mg_ctx* c) {
  hipEvent_t e;
  if (!c->ev_pool.empty()) {
    e = c->ev_pool.back();
    c->ev_pool.pop_back();
  } else {
    hipEventCreate(&e);
  }
  return e;
}

void prof_collect(mg_ctx* c) {
  for (auto& pr : c->ev_pending) {
    float ms = 0.f;
    hipEventSynchronize(pr.second);
    hipEventElapsedTime(&ms, pr.first, pr.second);
    c->prof_ms += ms;
    c->prof_launches += 1;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  c->ev_pending.clear();
  c->ev_pool.insert(c->ev_pool.end(), c->ev_spare.begin(), c->ev_spare.end());
  c->ev_spare.clear();
}

Sink launch_sink(mg_ctx* c, hipStream_t s) {
  return [c, s](const OpRec& o) {
    const bool prof = c->prof_on && o.level == 0 && prof_class(o) == c->prof_kernel;
    // ka, kb: the start and end of the step's kernel, recorded by its launch
    // (the measured time when the step is one kernel); a, b: events on the
    // stream around the whole step (the measured time otherwise)
    hipEvent_t a = nullptr, b = nullptr, ka = nullptr, kb = nullptr;
    if (prof) {
      a = take_event(c);
      b = take_event(c);
      ka = take_event(c);
      kb = take_event(c);
      hipEventRecord(a, s);
      g_kernel_events = KernelEvents{ka, kb, 0};
    }
    const OpRec* p = &o;
    launch_ops(&p, 1, s);
    if (prof) {
      const int kernels = g_kernel_events.launches;
      g_kernel_events = KernelEvents{};
      hipEventRecord(b, s);
      if (kernels == 1) std::swap(a, ka), std::swap(b, kb);
      c->ev_pending.emplace_back(a, b);
      c->ev_spare.push_back(ka);
      c->ev_spare.push_back(kb);
    }
  };
}

void drop_graph(mg_ctx* c, int kind, int slot) {
  if (c->gexec[kind][slot]) hipGraphExecDestroy(c->gexec[kind][slot]);
  c->gexec[kind][slot] = nullptr;
  c->gkey[kind][slot][0] = c->gkey[kind][slot][1] = c->gkey[kind][slot][2] = nullptr;
}

void drop_graphs(mg_ctx* c) {
  for (int k = 0; k < mg_ctx::kIterKinds; ++k)
    for (int q = 0; q < mg_ctx::kGraphSlots; ++q) drop_graph(c, k, q);
}

// Run one iteration of the given kind: replay the cached graph (captured on
// first use for these buffers) or launch eagerly.
mg_status run_iteration(mg_ctx* c, double* u, const double* b, hipStream_t s, int kind) {
  const bool eager = (c->o.flags & MG_FLAG_NO_GRAPH) || c->prof_on;
  if (eager) {
    emit_iteration(c, launch_sink(c, s), u, b, kind);
    HIP_TRY(hipGetLastError());
    return MG_OK;
  }
  const int scode = c->s0on ? 1 + c->s0at[0] + 2 * c->s0at[1] : 0;
  const void* key[3] = {u, b, reinterpret_cast<const void*>((intptr_t)scode)};
  int slot = -1;
  for (int q = 0; q < mg_ctx::kGraphSlots; ++q)
    if (c->gexec[kind][q] && memcmp(key, c->gkey[kind][q], sizeof key) == 0) slot = q;
  if (slot < 0) {
    // replace the slot used less recently
    slot = (c->glast[kind] + 1) % mg_ctx::kGraphSlots;
    drop_graph(c, kind, slot);
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    emit_iteration(c, launch_sink(c, c->cap), u, b, kind);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(c->cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(MG_E_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                  hipGetErrorString(ee));
    }
    hipError_t ie = hipGraphInstantiate(&c->gexec[kind][slot], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      c->gexec[kind][slot] = nullptr;
      return fail(MG_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    }
    memcpy(c->gkey[kind][slot], key, sizeof key);
    // the split state the iteration leaves (capturing emitted it)
    c->gstate[kind][slot][0] = c->s0at[0] + 2 * c->s0at[1];
    c->gstate[kind][slot][1] = c->s0u[0] + 2 * c->s0u[1];
  }
  c->glast[kind] = slot;
  HIP_TRY(hipGraphLaunch(c->gexec[kind][slot], s));
  c->s0at[0] = c->gstate[kind][slot][0] & 1;
  c->s0at[1] = c->gstate[kind][slot][0] >> 1;
  c->s0u[0] = c->gstate[kind][slot][1] & 1;
  c->s0u[1] = c->gstate[kind][slot][1] >> 1;
  return MG_OK;
}

mg_status read_scalar(mg_ctx* c, int idx, double* out, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(c->pinned + idx, c->scal + idx, sizeof(double), hipMemcpyDeviceToHost,
                         s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = c->pinned[idx];
  return MG_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
StencilParams<T> params_of(const OpRec& o) {
  return StencilParams<T>{o.opkind, (T)o.wc, (T)o.w1, (T)o.w2, (T)o.s, (T)o.wf};
}

template <typename T>
void launch_typed(const OpRec& o, const Batch& B, hipStream_t s) {
  const Item& it = B.it[0];
  switch (o.code) {
    case OC_SMOOTH:
      launch_smooth<T>(o.g, params_of<T>(o), o.sub & 15, ((o.sub >> 4) & 1) != 0, (T)o.omega, B,
                       s, (o.sub >> 5) & 7, ((o.sub >> 8) & 1) != 0);
      break;
    case OC_RESID:
      launch_residual<T>(o.g, params_of<T>(o), (o.sub & 1) != 0, B, s, (o.sub >> 5) & 7,
                         ((o.sub >> 9) & 1) != 0);
      break;
    case OC_RESTRICT: launch_restrict<T>(o.g, o.gc, B, s); break;
    case OC_RESID_RESTRICT: launch_resid_restrict<T>(o.g, params_of<T>(o), o.sub == 1, B, s); break;
    case OC_RESTRICT_XCOLS: launch_restrict_xcols<T>(o.g, B, s); break;
    case OC_PROLONG: launch_prolong_add<T>(o.g, o.gc, B, s); break;
    case OC_COARSE: launch_coarse_solve<T>(o.g, o.m, B, s); break;
    case OC_NORM2: launch_norm2_partial<T>(o.g, B, s); break;
    case OC_TAIL: launch_tail<T>(o.g.dim, o.opkind, (int)o.count, B, s); break;
    case OC_FILL: launch_fill<T>((T*)it.c, o.count, T(0), s); break;
    case OC_COPY: launch_copy<T>((const T*)it.a, (T*)it.c, o.count, s); break;
    case OC_CSR_SMOOTH:
      launch_csr_smooth<T>(o.g, *(const CsrOp<T>*)o.csr, o.sub & 15,
                           (o.sub >> 4) ? nullptr : (const T*)it.a, (const T*)it.b, (T*)it.c,
                           (T)o.omega, s);
      break;
    case OC_CSR_RESID:
      launch_csr_residual<T>(o.g, *(const CsrOp<T>*)o.csr, (const T*)it.a, (const T*)it.b,
                             (T*)it.c, it.partials, s);
      break;
    case OC_HEAD:
      launch_head<T>(o.g, params_of<T>(o), o.sub & 15, (T)o.omega, B, s, (o.sub >> 5) & 7);
      break;
    case OC_SMOOTH2:
      launch_smooth_pair<T>(o.g, params_of<T>(o), o.sub & 15, (o.sub >> 4) != 0, B, s);
      break;
    case OC_SMOOTH_PRO:
      launch_smooth_prolong<T>(o.g, params_of<T>(o), o.sub & 15, (T)o.omega, B, s,
                               (o.sub >> 5) & 7);
      break;
    case OC_APPLY_DOT: launch_apply_dot<T>(o.g, params_of<T>(o), B, s); break;
    case OC_CSR_APPLY_DOT:
      launch_csr_apply_dot<T>(o.g, *(const CsrOp<T>*)o.csr, (const T*)it.a, (T*)it.c,
                              it.partials, s);
      break;
    case OC_CSR_HEAD:
      launch_csr_head<T>(o.g, *(const CsrOp<T>*)o.csr, o.sub, (const T*)it.a, (const T*)it.b,
                         (T*)it.c, (T)o.omega, it.partials, s);
      break;
    default: break;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// op fusion interface (used by the serving scheduler)
// ---------------------------------------------------------------------------
namespace mg {

bool batchable(const OpRec& a) {
  return a.code != OC_FILL && a.code != OC_COPY && a.code != OC_CSR_SMOOTH &&
         a.code != OC_CSR_RESID && a.code != OC_CSR_HEAD && a.code != OC_CSR_APPLY_DOT &&
         a.code != OC_PCG && a.code != OC_ZERO_BOUNDARY;
}

bool same_key(const OpRec& a, const OpRec& b) {
  return a.code == b.code && a.prec == b.prec && a.sub == b.sub && a.g.dim == b.g.dim &&
         a.g.n == b.g.n && a.g.s3 == b.g.s3 && a.gc.n == b.gc.n && a.opkind == b.opkind && a.wc == b.wc &&
         a.w1 == b.w1 && a.w2 == b.w2 && a.s == b.s && a.wf == b.wf && a.omega == b.omega &&
         a.m == b.m && a.item.lay == b.item.lay &&
         a.count == b.count && batchable(a) && batchable(b);
}

void launch_pcg(const OpRec& o, hipStream_t s) {
  double* const* v = reinterpret_cast<double* const*>(o.ext);
  double* S = o.item.scal;
  double* part = o.item.partials;
  switch (o.sub) {
    case PO_DOTS2:
      launch_pcg_dots2(v[0], v[1], v[2], o.count, part, part + pcg_blocks(o.count), s);
      break;
    case PO_SCALARS: launch_pcg_scalars(S, o.item.flag, s); break;
    case PO_DIR: launch_pcg_dir(v[0], v[1], S, o.count, o.item.flag, s); break;
    case PO_UPDATE: launch_pcg_update(v[0], v[1], v[2], v[3], v[4], S, o.count, part, s); break;
    case PO_ZSCALE:
      launch_pcg_zscale(reinterpret_cast<const float*>(o.ext[0]), v[1], S, o.count, s);
      break;
    default: break;
  }
}

void launch_ops(const OpRec* const* ops, int n, hipStream_t s) {
  Batch B{};
  B.count = n;
  for (int q = 0; q < n; ++q) B.it[q] = ops[q]->item;
  const OpRec& o = *ops[0];
  switch (o.code) {
    case OC_REDUCE: launch_reduce_final(o.count, B, s); return;
    case OC_SCALE_CAST: launch_scale_cast(o.g, B, s); return;
    case OC_IR_UPDATE: launch_ir_update(o.g, B, s); return;
    case OC_PCG: launch_pcg(o, s); return;
    case OC_ZERO_BOUNDARY: launch_zero_boundary(o.g, (double*)o.item.c, s); return;
    default: break;
  }
  if (o.prec == 0)
    launch_typed<double>(o, B, s);
  else
    launch_typed<float>(o, B, s);
}

void record_iteration(mg_ctx* c, double* u, const double* b, std::vector<OpRec>& out) {
  emit_iteration(c, [&out](const OpRec& o) { out.push_back(o); }, u, b);
}

void record_prologue(mg_ctx* c, double* u, const double* b, std::vector<OpRec>& out) {
  emit_prologue(c, [&out](const OpRec& o) { out.push_back(o); }, u, b);
}

size_t plan_bytes(const mg_options& o, bool has_kappa) { return plan(o, has_kappa, nullptr, nullptr); }

}  // namespace mg

namespace {

// Whether mg_solve runs the whole solve in one workgroup (k_tail_solve):
// FP64 cycles with the matrix-free operator on a hierarchy the tail holds
// from its finest level on, no CG and no warm start; MG_FLAG_NO_FUSE keeps
// the cycle-by-cycle iteration (one tail launch and one residual norm per
// cycle, read by the host).
bool whole_tail_solve(const mg_ctx* c) {
  return c->tail0 == 0 && !c->ir && !c->csr && !c->prof_on &&
         !(c->o.flags & (MG_FLAG_PCG | MG_FLAG_WARM | MG_FLAG_NO_FUSE));
}

// Status, cycle count and history from the results of k_tail_solve (res:
// host copy of kTailSolveHead + max_iter + 1 doubles).
mg_status tail_solve_result(const double* res, int max_iter, double tol, int* iters,
                            double* hist) {
  const int status = (int)res[0];
  const int k = (int)res[1];
  *iters = k;
  if (hist) {
    hist[0] = 1.0;
    for (int q = 1; q <= k && q <= max_iter; ++q) hist[q] = res[kTailSolveHead + q];
  }
  switch (status) {
    case TS_OK: return MG_OK;
    case TS_NONFINITE_B: return fail(MG_E_NONFINITE, "b holds NaN or Inf");
    case TS_DIVERGED:
      return fail(MG_E_DIVERGED, "relative residual %g after %d cycles", res[kTailSolveHead + k],
                  k);
    default: return fail(MG_E_MAXIT, "no convergence to %g in %d cycles", tol, max_iter);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* mg_last_error(void) { return g_err.c_str(); }

void mg_options_default(mg_options* o) {
  if (!o) return;
  o->dim = 3;
  o->n = 64;
  o->levels = 6;
  o->op = MG_OP_STENCIL;
  o->smoother = MG_SMOOTH_RBGS;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->omega = 2.0 / 3.0;
  o->precision = MG_PREC_FP64;
  o->max_iter = 100;
  o->flags = 0;
  o->cycle = MG_CYCLE_V;
  o->sigma = 0.0;
}

size_t mg_footprint_bytes(const mg_options* o) {
  std::string why;
  if (!valid_options(o, why)) {
    fail(MG_E_ARG, "%s", why.c_str());
    return 0;
  }
  // with or without per-cell kappa (the split iterates exist only without)
  return std::max(plan(*o, true, nullptr, nullptr), plan(*o, false, nullptr, nullptr));
}

mg_status mg_setup(const mg_options* o, const double* kappa_dev, void* stream, mg_ctx** out) {
  if (!out) return fail(MG_E_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_options(o, why)) return fail(MG_E_ARG, "%s", why.c_str());
  if (o->sigma > 0.0 && kappa_dev && o->op == MG_OP_STENCIL)
    return fail(MG_E_ARG, "the matrix-free operator with per-cell kappa has no mass term "
                          "(sigma > 0 needs kappa = 1 or MG_OP_CSR)");
  hipStream_t s = as_stream(stream);
  mg_ctx* c = new mg_ctx();
  c->o = *o;
  c->L = o->levels;
  c->kappa = kappa_dev != nullptr;
  c->ir = o->precision == MG_PREC_FP32_IR;
  c->csr = o->op == MG_OP_CSR;
  c->tail0 = tail_start(*o, c->kappa);
  c->lv.resize(c->L);
  auto bail = [&](mg_status st) {
    mg_destroy(c);
    return st;
  };
  const size_t bytes = plan(*o, c->kappa, nullptr, nullptr);
  if (hipMalloc(&c->arena, bytes) != hipSuccess) {
    c->arena = nullptr;
    (void)hipGetLastError();
    return bail(fail(MG_E_NOMEM, "hipMalloc of %zu bytes failed", bytes));
  }
  c->arena_bytes = bytes;
  plan(*o, c->kappa, c->arena, c);
  c->npinned = std::max(8, kTailSolveHead + o->max_iter + 1);
  if (hipHostMalloc(&c->pinned, c->npinned * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    c->pinned = nullptr;
    return bail(fail(MG_E_HIP, "hipHostMalloc failed"));
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->cap = nullptr;
    return bail(fail(MG_E_HIP, "hipStreamCreate failed"));
  }
  if (hipMemsetAsync(c->arena, 0, bytes, s) != hipSuccess)
    return bail(fail(MG_E_HIP, "hipMemsetAsync failed"));
  if (c->kappa) {
    const long cells0 = ipow(o->n, o->dim);
    launch_count_bad_kappa(kappa_dev, cells0, c->ibuf, c->ibuf + 1, s);
    int bad[2] = {0, 0};
    if (hipMemcpyAsync(bad, c->ibuf, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(MG_E_HIP, "kappa check failed: %s", hipGetErrorString(hipGetLastError())));
    if (bad[1]) return bail(fail(MG_E_NONFINITE, "kappa has %d non-finite entries", bad[1]));
    if (bad[0]) return bail(fail(MG_E_ARG, "kappa has %d entries <= 0", bad[0]));
    if (hipMemcpyAsync(c->lv[0].kap64, kappa_dev, cells0 * sizeof(double),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return bail(fail(MG_E_HIP, "kappa copy failed"));
    for (int l = 1; l < c->L; ++l)
      launch_kappa_coarsen(o->dim, c->lv[l - 1].g.n, c->lv[l - 1].kap64, c->lv[l].kap64, s);
    if (c->ir)
      for (int l = 0; l < c->L; ++l)
        launch_cast_f32(c->lv[l].kap64, c->lv[l].kap32, ipow(c->lv[l].g.n, o->dim), s);
  }
  for (int l = 0; l < c->L; ++l) set_stencil(c, l);
  if (c->csr) {
    for (int l = 0; l < c->L; ++l) {
      mg_status st = build_csr(c, l, s);
      if (st != MG_OK) return bail(st);
    }
  }
  mg_status st = coarse_factor(c, s);
  if (st != MG_OK) return bail(st);
  st = build_tail<double>(c, s);
  if (st == MG_OK && c->ir) st = build_tail<float>(c, s);
  if (st != MG_OK) return bail(st);
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return bail(fail(MG_E_HIP, "setup kernels failed"));
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  if (c->cap) hipStreamSynchronize(c->cap);
  drop_graphs(c);
  for (auto& pr : c->ev_pending) {
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  for (hipEvent_t e : c->ev_spare) hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->pinned) hipHostFree(c->pinned);
  if (c->arena) {
    hipDeviceSynchronize();
    hipFree(c->arena);
  }
  delete c;
}

mg_status mg_level_info(const mg_ctx* c, int level, int* n_l, size_t* nodes) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  if (level < 0 || level >= c->L) return fail(MG_E_ARG, "level %d out of range", level);
  if (n_l) *n_l = c->lv[level].g.n;
  if (nodes) *nodes = (size_t)c->lv[level].g.nodes;
  return MG_OK;
}

mg_status mg_solve(mg_ctx* c, const double* b, double* u, double tol, int* iters, double* hist,
                   void* stream) {
  if (!c || !b || !u || !iters) return fail(MG_E_ARG, "NULL argument");
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be > 0");
  if ((const void*)b == (const void*)u) return fail(MG_E_ARG, "u must not alias b");
  hipStream_t s = as_stream(stream);
  *iters = 0;
  if (hist) hist[0] = 1.0;
  c->natural = false;
  c->b0_split = split_b0(c->o);
  const bool pcg = (c->o.flags & MG_FLAG_PCG) != 0;
  const bool warm = (c->o.flags & MG_FLAG_WARM) != 0;
  if (whole_tail_solve(c)) {
    // every cycle, the norm and the stopping test in one launch; one read
    Batch B{};
    B.count = 1;
    B.it[0].a = c->tail64;
    B.it[0].b = b;
    B.it[0].c = u;
    B.it[0].scal = c->tres;
    B.it[0].flag = c->o.cycle << 1;
    launch_tail_solve(c->o.dim, c->lv[0].st64.kind, c->tail_lds[0], B, tol, c->o.max_iter, s);
    HIP_TRY(hipGetLastError());
    const int nres = kTailSolveHead + c->o.max_iter + 1;
    HIP_TRY(hipMemcpyAsync(c->pinned, c->tres, nres * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return tail_solve_result(c->pinned, c->o.max_iter, tol, iters, hist);
  }
  const bool fuse = head_fusion(c);
  c->s0on = fuse && !pcg && split_persist(c);
  c->s0at[0] = c->s0at[1] = c->s0u[0] = c->s0u[1] = 0;
  const double* bc = b;  // b as the cycles read it
  if (c->b0_split) {
    // the level-0 right-hand side colour-split (each half-sweep then reads
    // its colour's half), with the partial sums of ||b||^2 in the same pass
    launch_split_norm(c->lv[0].g, b, c->lv[0].b64, b_split_half(c, 0, 0), c->partials, s);
    bc = c->lv[0].b64;
  }
  if (pcg)
    emit_pcg_prologue(c, launch_sink(c, s), u, b, warm);
  else
    emit_prologue(c, launch_sink(c, s), u, bc, warm, fuse, c->b0_split);
  HIP_TRY(hipGetLastError());
  double nb2 = 0.0;
  mg_status st = read_scalar(c, 1, &nb2, s);
  if (st != MG_OK) return st;
  if (!std::isfinite(nb2)) return fail(MG_E_NONFINITE, "b holds NaN or Inf");
  if (nb2 == 0.0) {
    if (warm || c->s0on) {
      emit_fill<double>(c, launch_sink(c, s), 0, u);
      HIP_TRY(hipGetLastError());
    }
    return MG_OK;
  }
  const double nb = std::sqrt(nb2);
  if (warm) {
    double r2 = 0.0;
    st = read_scalar(c, 0, &r2, s);
    if (st != MG_OK) return st;
    const double rho0 = std::sqrt(r2) / nb;
    if (!std::isfinite(rho0)) return fail(MG_E_NONFINITE, "the initial u holds NaN or Inf");
    if (hist) hist[0] = rho0;
    if (rho0 <= tol) return MG_OK;
  }
  // a split finest iterate reaches u after the last cycle
  auto finish = [&](mg_status result) -> mg_status {
    if (c->s0on && *iters > 0) {
      Level& L0 = c->lv[0];
      Batch B{};
      B.count = 1;
      B.it[0].a = L0.xs64[c->s0u[0]];
      B.it[0].a2 = L0.xs64[c->s0u[1]] + (L0.g.nodes + 1) / 2;
      B.it[0].c = u;
      launch_unsplit<double>(L0.g, B, s);
      HIP_TRY(hipGetLastError());
    }
    return result;
  };
  for (int k = 1; k <= c->o.max_iter; ++k) {
    const int kind = pcg ? (k == 1 ? IT_PCG_FIRST : IT_PCG)
                         : (!fuse ? IT_PLAIN : (k == 1 && !warm ? IT_FUSED_FIRST : IT_FUSED));
    st = run_iteration(c, u, bc, s, kind);
    if (st != MG_OK) return st;
    double n2 = 0.0;
    st = read_scalar(c, 0, &n2, s);
    if (st != MG_OK) return st;
    if (c->prof_on) prof_collect(c);
    const double rho = std::sqrt(n2) / nb;
    *iters = k;
    if (hist) hist[k] = rho;
    if (!std::isfinite(rho) || rho > 1e3)
      return finish(fail(MG_E_DIVERGED, "relative residual %g after %d cycles", rho, k));
    if (rho <= tol) return finish(MG_OK);
  }
  return finish(fail(MG_E_MAXIT, "no convergence to %g in %d cycles", tol, c->o.max_iter));
}

mg_status mg_cn_rhs(mg_ctx* c, const double* u, double* guess, const double* g0, double c0,
                    const double* g1, double c1, const double* F, double cf, double* b,
                    void* stream) {
  if (!c || !u || !b) return fail(MG_E_ARG, "NULL argument");
  if (c->kappa) return fail(MG_E_ARG, "mg_cn_rhs needs a context with kappa = 1");
  if ((const double*)b == u || b == guess || (const double*)b == g0 ||
      (const double*)b == g1 || (const double*)b == F)
    return fail(MG_E_ARG, "b must not alias an input");
  if ((const double*)guess == u) return fail(MG_E_ARG, "guess must not alias u");
  if (!(std::isfinite(c0) && std::isfinite(c1) && std::isfinite(cf)))
    return fail(MG_E_ARG, "c0, c1 and cf must be finite");
  const Level& L0 = c->lv[0];
  const int dim = c->o.dim;
  const double h = 1.0 / L0.g.n, sg = c->o.sigma;
  CnWeights w{};
  for (int cls = 0; cls <= dim; ++cls) {
    const double wm = mass_weight(dim, h, cls), wk = stiff_weight(dim, h, cls);
    w.wb[cls] = sg * wm - wk;
    w.wa[cls] = sg * wm + wk;
  }
  w.c0 = c0;
  w.c1 = c1;
  w.cf = cf;
  hipStream_t s = as_stream(stream);
  launch_zero_boundary(L0.g, b, s);
  launch_cn_rhs(L0.g, w, u, guess, g0, g1, F, b, s);
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_mass(mg_ctx* c, const double* f, double* F, void* stream) {
  if (!c || !f || !F) return fail(MG_E_ARG, "NULL argument");
  if ((const double*)F == f) return fail(MG_E_ARG, "F must not alias f");
  const Level& L0 = c->lv[0];
  const int dim = c->o.dim;
  const double h = 1.0 / L0.g.n;
  // the node kernel of the right-hand side with x0 = f on every node and
  // the mass weights: F = M f
  CnWeights w{};
  for (int cls = 0; cls <= dim; ++cls) w.wb[cls] = mass_weight(dim, h, cls);
  w.c0 = 1.0;
  hipStream_t s = as_stream(stream);
  launch_zero_boundary(L0.g, F, s);
  launch_cn_rhs_nodes(L0.g, w, f, f, F, s);
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

}  // extern "C"

// ---- single steps -----------------------------------------------------------
namespace {
mg_status check_step(mg_ctx* c, int level, int prec, bool need_next) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  c->natural = true;  // caller buffers: natural layout throughout
  if (level < 0 || level >= c->L || (need_next && level >= c->L - 1))
    return fail(MG_E_ARG, "level %d out of range", level);
  if (prec != MG_PREC_FP64 && prec != MG_PREC_FP32_IR) return fail(MG_E_ARG, "bad precision");
  if (prec == MG_PREC_FP32_IR && !c->ir)
    return fail(MG_E_STATE, "FP32 operators exist only in MG_PREC_FP32_IR contexts");
  return MG_OK;
}

template <typename F>
mg_status typed(int prec, F f) {
  if (prec == MG_PREC_FP64)
    f(double(0));
  else
    f(float(0));
  HIP_TRY(hipGetLastError());
  return MG_OK;
}
}  // namespace

extern "C" {

mg_status mg_apply_residual(mg_ctx* c, int level, int prec, const void* x, const void* b, void* r,
                            void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!x || !b || !r) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    emit_fill<T>(c, sink, level, (T*)r);
    emit_residual<T>(c, sink, level, (const T*)x, (const T*)b, (T*)r, nullptr);
  });
}

mg_status mg_apply_smooth(mg_ctx* c, int level, int prec, int step, const void* x_in,
                          const void* b, void* x_out, void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!b || !x_out) return fail(MG_E_ARG, "NULL vector");
  const int ncol = 1 << c->o.dim;
  if (step < 0 || step > 4 + ncol) return fail(MG_E_ARG, "step must be 0..%d", 4 + ncol);
  if (step >= 5 && c->csr && c->o.smoother != MG_SMOOTH_GS)
    return fail(MG_E_STATE, "CSR colour steps need rows blocked by colour (MG_SMOOTH_GS)");
  if (step >= 5 && x_in == x_out) return fail(MG_E_ARG, "x_out must not alias x_in");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    T* out = (T*)x_out;
    const T* in = (const T*)x_in;
    const T* bb = (const T*)b;
    emit_fill<T>(c, sink, level, out);
    if (step >= 5) {
      // Gauss-Seidel update of colour step - 5 on a copy of x_in
      if (in) {
        OpRec o = base_op<T>(c, OC_COPY, level);
        o.count = c->lv[level].g.nodes;
        o.item.a = in;
        o.item.c = out;
        sink(o);
      }
      emit_smooth<T>(c, sink, level, SM_GS0 + step - 5, out, bb, out);
      return;
    }
    if (step <= 2) {
      emit_smooth<T>(c, sink, level, step, in, bb, out);
      return;
    }
    // full red-black sweep through the level's spare buffer
    T* tmp = Bufs<T>::t(c->lv[level]);
    const int k1 = step == 3 ? SM_RB0 : SM_RB1, k2 = step == 3 ? SM_RB1 : SM_RB0;
    emit_smooth<T>(c, sink, level, k1, in, bb, tmp);
    emit_smooth<T>(c, sink, level, k2, tmp, bb, out);
  });
}

mg_status mg_apply_restrict(mg_ctx* c, int level, int prec, const void* r, void* bc,
                            void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!r || !bc) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    emit_fill<T>(c, sink, level + 1, (T*)bc);
    OpRec o = base_op<T>(c, OC_RESTRICT, level);
    o.item.lay = b_split_half(c, level + 1, Bufs<T>::prec);
    o.item.a = r;
    o.item.c = bc;
    sink(o);
  });
}

mg_status mg_apply_residual_restrict(mg_ctx* c, int level, int prec, const void* x, const void* b,
                                     void* bc, void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!x || !b || !bc) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    // (natural layouts: check_step set c->natural)
    emit_fill<T>(c, sink, level + 1, (T*)bc);
    emit_resid_restrict<T>(c, sink, level, (const T*)x, (const T*)b, nullptr, (T*)bc);
  });
}

mg_status mg_apply_prolong_add(mg_ctx* c, int level, int prec, const void* e, void* x,
                               void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!e || !x) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    OpRec o = base_op<T>(c, OC_PROLONG, level);
    o.item.a = e;
    o.item.c = x;
    sink(o);
  });
}

mg_status mg_apply_coarse_solve(mg_ctx* c, int prec, const void* bc, void* xc, void* stream) {
  mg_status st = check_step(c, c ? c->L - 1 : 0, prec, false);
  if (st != MG_OK) return st;
  if (!bc || !xc) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    emit_fill<T>(c, sink, c->L - 1, (T*)xc);
    OpRec o = base_op<T>(c, OC_COARSE, c->L - 1);
    o.item.b = bc;
    o.item.c = xc;
    o.item.L = c->Lc;
    sink(o);
  });
}

mg_status mg_vcycle(mg_ctx* c, int prec, void* x, const void* b, void* stream) {
  mg_status st = check_step(c, 0, prec, false);
  if (st != MG_OK) return st;
  if (!x || !b) return fail(MG_E_ARG, "NULL vector");
  const Sink sink = launch_sink(c, as_stream(stream));
  return typed(prec, [&](auto tag) {
    using T = decltype(tag);
    emit_vcycle<T>(c, sink, (T*)x, Bufs<T>::t(c->lv[0]), (const T*)b, false);
  });
}

mg_status mg_norm2(mg_ctx* c, int level, int prec, const void* v, double* out, void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!v || !out) return fail(MG_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  const Sink sink = launch_sink(c, s);
  st = typed(prec, [&](auto tag) {
    using T = decltype(tag);
    OpRec o = base_op<T>(c, OC_NORM2, level);
    o.item.a = v;
    o.item.partials = c->partials;
    sink(o);
    emit_reduce(c, sink, norm2_blocks(c->lv[level].g), c->scal + 2);
  });
  if (st != MG_OK) return st;
  return read_scalar(c, 2, out, s);
}

mg_status mg_profile_enable(mg_ctx* c, int kernel_id, int enable) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  if (kernel_id < 0 || kernel_id > 8) return fail(MG_E_ARG, "kernel_id must be 0..8");
  c->prof_kernel = kernel_id;
  c->prof_on = enable != 0;
  c->prof_launches = 0;
  c->prof_ms = 0.0;
  return MG_OK;
}

mg_status mg_profile_read(mg_ctx* c, long* launches, double* total_ms) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  prof_collect(c);
  if (launches) *launches = c->prof_launches;
  if (total_ms) *total_ms = c->prof_ms;
  return MG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the solve that allocates nothing (mg_solve_noalloc)
// ---------------------------------------------------------------------------
namespace {

// Device scratch of mg_solve_noalloc, one copy per GPU for the life of the
// process.  Host code never passes `scratch` itself to a kernel or a copy:
// it uses the device address hipGetSymbolAddress returns for the current
// device (noalloc_scratch).  Layout (bytes):
constexpr long kNaDesc = 0;                    // TailDesc<double>
constexpr long kNaRes = 4096;                  // results: status, cycles, history
constexpr int kNaMaxIter = 1000;               // max_iter accepted
constexpr long kNaBad = 12288;                 // two ints: kappa check counters
constexpr long kNaKappa = 12544;               // cell coefficients, every level
constexpr long kNaKappaCells = 8192;
constexpr long kNaR0 = kNaKappa + 8 * kNaKappaCells;  // finest residual (if not in LDS)
constexpr long kNaR0Nodes = 5120;
constexpr long kNaL = kNaR0 + 8 * kNaR0Nodes;  // coarsest Cholesky factor
constexpr int kNaMaxCoarse = 256;              // coarsest unknowns accepted
constexpr long kNaBytes = 1L << 20;
static_assert(sizeof(TailDesc<double>) <= kNaRes - kNaDesc, "descriptor slot");
static_assert((kTailSolveHead + kNaMaxIter + 1) * 8 <= kNaBad - kNaRes, "result slot");
static_assert(kNaL % 256 == 0 && kNaKappa % 256 == 0 && kNaR0 % 256 == 0, "alignment");
static_assert(kNaL + 8L * kNaMaxCoarse * kNaMaxCoarse <= kNaBytes, "scratch size");

__device__ __align__(256) char scratch[kNaBytes];

// Host state of mg_solve_noalloc, used under g_na_mu only: calls from
// several threads run one after the other, each to completion.
std::mutex g_na_mu;
char* g_na_ptr[64] = {};                        // device address per device
double g_na_L[kNaMaxCoarse * kNaMaxCoarse];     // coarsest factor (host)
double g_na_kc[4096];                           // coarsest cell coefficients (host)
double g_na_res[kTailSolveHead + kNaMaxIter + 1];
TailDesc<double> g_na_desc;

// The scratch array's device address on the current device (looked up once
// per device).
mg_status noalloc_scratch(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MG_E_ARG, "device %d out of range", dev);
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_na_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_na_ptr[dev];
  return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_solve_noalloc(const mg_options* o, const double* kappa_dev, const double* b,
                           double* u, double tol, int* iters, double* hist, void* stream) {
  if (!b || !u || !iters) return fail(MG_E_ARG, "NULL argument");
  std::string why;
  if (!valid_options(o, why)) return fail(MG_E_ARG, "%s", why.c_str());
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be > 0");
  if ((const void*)b == (const void*)u) return fail(MG_E_ARG, "u must not alias b");
  if (o->precision != MG_PREC_FP64 || o->op != MG_OP_STENCIL || o->flags != 0)
    return fail(MG_E_ARG, "the no-allocation solve takes FP64, the matrix-free operator and "
                          "no flags");
  if (o->max_iter > kNaMaxIter)
    return fail(MG_E_ARG, "max_iter %d above the no-allocation limit %d", o->max_iter,
                kNaMaxIter);
  const bool kappa = kappa_dev != nullptr;
  if (kappa && o->sigma > 0.0)
    return fail(MG_E_ARG, "the matrix-free operator with per-cell kappa has no mass term");
  if (tail_start(*o, kappa) != 0)
    return fail(MG_E_ARG, "the no-allocation solve needs a hierarchy one workgroup holds "
                          "(finest level at most %d unknowns, its vectors within %d bytes "
                          "of LDS)", kTailMaxUnknowns, kTailLdsBytes);
  const int L = o->levels, dim = o->dim;
  const int nc = o->n >> (L - 1);
  const int m = (int)ipow(nc - 1, dim);
  if (m > kNaMaxCoarse)
    return fail(MG_E_ARG, "coarsest level has %d unknowns (the no-allocation solve takes at "
                          "most %d): use more levels", m, kNaMaxCoarse);
  long cells = 0;
  for (int l = 0; l < L; ++l) cells += ipow(o->n >> l, dim);
  if ((kappa && cells > kNaKappaCells) || ipow(o->n + 1L, dim) > kNaR0Nodes ||
      ipow(nc, dim) > 4096)
    return fail(MG_E_ARG, "internal: hierarchy exceeds the no-allocation scratch");
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lock(g_na_mu);
  char* base = nullptr;
  mg_status st = noalloc_scratch(&base);
  if (st != MG_OK) return st;
  double* kap[kTailMaxLevels] = {};
  const double* kc_host = nullptr;
  if (kappa) {
    int* bad = reinterpret_cast<int*>(base + kNaBad);
    int badh[2] = {0, 0};
    launch_fill<double>(reinterpret_cast<double*>(bad), 1, 0.0, s);  // both counters = 0
    launch_count_bad_kappa(kappa_dev, ipow(o->n, dim), bad, bad + 1, s);
    HIP_TRY(hipMemcpyAsync(badh, bad, sizeof badh, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (badh[1]) return fail(MG_E_NONFINITE, "kappa has %d non-finite entries", badh[1]);
    if (badh[0]) return fail(MG_E_ARG, "kappa has %d entries <= 0", badh[0]);
    double* k = reinterpret_cast<double*>(base + kNaKappa);
    for (int l = 0; l < L; ++l) {
      kap[l] = k;
      k += ipow(o->n >> l, dim);
    }
    HIP_TRY(hipMemcpyAsync(kap[0], kappa_dev, ipow(o->n, dim) * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    for (int l = 1; l < L; ++l) launch_kappa_coarsen(dim, o->n >> (l - 1), kap[l - 1], kap[l], s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(g_na_kc, kap[L - 1], ipow(nc, dim) * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    kc_host = g_na_kc;
  }
  st = coarse_cholesky(dim, nc, kc_host, o->sigma, m, g_na_L);
  if (st != MG_OK) return st;
  double* Ld = reinterpret_cast<double*>(base + kNaL);
  HIP_TRY(hipMemcpyAsync(Ld, g_na_L, (size_t)m * m * sizeof(double), hipMemcpyHostToDevice, s));
  int nl[kTailMaxLevels];
  StencilParams<double> stp[kTailMaxLevels];
  const int kind = kappa ? OP_KAPPA : (dim == 3 && o->sigma > 0.0 ? OP_MASS : OP_CONST);
  for (int l = 0; l < L; ++l) {
    nl[l] = o->n >> l;
    stp[l] = stencil_of(dim, nl[l], o->sigma, kind);
  }
  st = fill_tail_desc<double>(*o, L, 0, kappa, m, Ld, nl, stp, kap,
                              reinterpret_cast<double*>(base + kNaR0), g_na_desc);
  if (st != MG_OK) return st;
  HIP_TRY(hipMemcpyAsync(base + kNaDesc, &g_na_desc, sizeof g_na_desc, hipMemcpyHostToDevice, s));
  Batch B{};
  B.count = 1;
  B.it[0].a = base + kNaDesc;
  B.it[0].b = b;
  B.it[0].c = u;
  B.it[0].scal = reinterpret_cast<double*>(base + kNaRes);
  B.it[0].flag = o->cycle << 1;
  launch_tail_solve(dim, kind, g_na_desc.lds_bytes, B, tol, o->max_iter, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(g_na_res, base + kNaRes,
                         (kTailSolveHead + o->max_iter + 1) * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return tail_solve_result(g_na_res, o->max_iter, tol, iters, hist);
}

}  // extern "C"
