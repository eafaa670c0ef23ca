// Host runtime of the Q1 multigrid library: option validation, the device
// arena, the level hierarchy (Sec. 5.1), the V-cycle driver (Algorithm 1,
// Sec. 5.3), the outer cycle iteration (Sec. 5.5.1), the FP32-inner /
// FP64-outer refinement loop, HIP graph replay of whole cycles and the
// C ABI declared in mg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <utility>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mg.h"
#include "mg_internal.h"

using namespace mg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_err;

mg_status fail(mg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(MG_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                             \
  } while (0)

constexpr int kCoarseMax = kCoarseMaxUnknowns;
constexpr size_t kAlign = 256;

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Level {
  Geo g;
  // FP64 vectors (x and b of level 0 are the caller's)
  double *x64 = nullptr, *b64 = nullptr, *t64 = nullptr, *r64 = nullptr;
  // FP32 vectors (FP32_IR contexts)
  float *x32 = nullptr, *b32 = nullptr, *t32 = nullptr, *r32 = nullptr;
  // coefficients per cell
  double* kap64 = nullptr;
  float* kap32 = nullptr;
  // CSR
  int *rowptr = nullptr, *col = nullptr, *rowmap = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  int rows = 0;
  long nnz = 0;
  int coff[3] = {0, 0, 0};
  StencilOp<double> st64{};
  StencilOp<float> st32{};
  CsrOp<double> csr64{};
  CsrOp<float> csr32{};
};

struct mg_ctx {
  mg_options o{};
  int L = 0;
  bool kappa = false;
  bool ir = false;
  bool csr = false;
  std::vector<Level> lv;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  double* Lc = nullptr;  // coarsest Cholesky factor, row major
  int m = 0;
  double* partials = nullptr;
  long npart = 0;
  double* scal = nullptr;      // device scalars: [0] residual norm^2, [1] ||b||^2
  int* ibuf = nullptr;         // device ints (setup checks)
  double* pinned = nullptr;    // host pinned scalars
  hipStream_t cap = nullptr;   // private stream for graph capture
  hipGraphExec_t gexec = nullptr;
  const void* gkey[3] = {nullptr, nullptr, nullptr};
  // profiling
  int prof_kernel = -1;
  bool prof_on = false;
  long prof_launches = 0;
  double prof_ms = 0.0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
};

namespace {

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

bool valid_options(const mg_options* o, std::string& why) {
  char buf[256];
  if (!o) { why = "options is NULL"; return false; }
  if (o->dim != 2 && o->dim != 3) { why = "dim must be 2 or 3"; return false; }
  if (o->n < 2) { why = "n must be >= 2"; return false; }
  if (o->levels < 1 || o->levels > 30) { why = "levels must be in 1..30"; return false; }
  if (o->n % (1 << (o->levels - 1)) != 0 || (o->n >> (o->levels - 1)) < 2) {
    snprintf(buf, sizeof buf, "n = %d needs to be divisible by 2^(levels-1) with n >> (levels-1) >= 2", o->n);
    why = buf;
    return false;
  }
  if (o->op != MG_OP_STENCIL && o->op != MG_OP_CSR) { why = "op must be MG_OP_STENCIL or MG_OP_CSR"; return false; }
  if (o->smoother != MG_SMOOTH_JACOBI && o->smoother != MG_SMOOTH_RBGS) { why = "unknown smoother"; return false; }
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post > 64) { why = "nu_pre/nu_post out of range"; return false; }
  if (o->smoother == MG_SMOOTH_JACOBI && !(o->omega > 0.0 && o->omega <= 1.0)) { why = "omega must be in (0, 1]"; return false; }
  if (o->precision != MG_PREC_FP64 && o->precision != MG_PREC_FP32_IR) { why = "unknown precision"; return false; }
  if (o->max_iter < 1) { why = "max_iter must be >= 1"; return false; }
  const long nc = o->n >> (o->levels - 1);
  long m = 1;
  for (int d = 0; d < o->dim; ++d) m *= (nc - 1);
  if (m > kCoarseMax) {
    snprintf(buf, sizeof buf, "coarsest level has %ld unknowns (max %d): use more levels", m, kCoarseMax);
    why = buf;
    return false;
  }
  const long nodes = o->dim == 3 ? (long)(o->n + 1) * (o->n + 1) * (o->n + 1) : (long)(o->n + 1) * (o->n + 1);
  if (nodes >= (1L << 31)) { why = "grid too large for 32-bit node indices"; return false; }
  if (o->op == MG_OP_CSR) {
    long nnz = 1;
    for (int d = 0; d < o->dim; ++d) nnz *= (3L * o->n - 5);
    if (nnz >= (1L << 31)) { why = "CSR matrix too large for 32-bit offsets"; return false; }
  }
  return true;
}

long ipow(long b, int e) {
  long r = 1;
  while (e--) r *= b;
  return r;
}

long csr_nnz(int dim, int n) { return ipow(3L * n - 5, dim); }

// Lay out every buffer of a context; with base == nullptr only sizes.
size_t plan(const mg_options& o, bool has_kappa, char* base, mg_ctx* c) {
  Planner P(base);
  const bool ir = o.precision == MG_PREC_FP32_IR;
  const bool csr = o.op == MG_OP_CSR;
  long maxpart = 1;
  for (int l = 0; l < o.levels; ++l) {
    const int nl = o.n >> l;
    const Geo g = make_geo(o.dim, nl);
    Level tmp;
    Level& L = c ? c->lv[l] : tmp;
    L.g = g;
    if (l > 0) {
      L.x64 = P.take<double>(g.nodes);
      L.b64 = P.take<double>(g.nodes);
    }
    L.t64 = P.take<double>(g.nodes);
    L.r64 = P.take<double>(g.nodes);
    if (ir) {
      L.x32 = P.take<float>(g.nodes);
      L.b32 = P.take<float>(g.nodes);
      L.t32 = P.take<float>(g.nodes);
      L.r32 = P.take<float>(g.nodes);
    }
    const long cells = ipow(nl, o.dim);
    if (has_kappa) {
      L.kap64 = P.take<double>(cells);
      if (ir) L.kap32 = P.take<float>(cells);
    }
    const long rows = ipow(nl - 1, o.dim);
    if (csr) {
      const long nnz = csr_nnz(o.dim, nl);
      L.rows = (int)rows;
      L.nnz = nnz;
      L.rowptr = P.take<int>(rows + 1);
      L.col = P.take<int>(nnz);
      L.rowmap = P.take<int>(rows);
      L.val64 = P.take<double>(nnz);
      if (ir) L.val32 = P.take<float>(nnz);
      maxpart = std::max(maxpart, csr_residual_blocks((int)rows));
    }
    maxpart = std::max(maxpart, grid_blocks(g));
  }
  const long nc = o.n >> (o.levels - 1);
  const int m = (int)ipow(nc - 1, o.dim);
  double* Lc = P.take<double>((size_t)m * m);
  double* part = P.take<double>(maxpart);
  double* scal = P.take<double>(8);
  int* ibuf = P.take<int>(8);
  if (c) {
    c->Lc = Lc;
    c->m = m;
    c->partials = part;
    c->npart = maxpart;
    c->scal = scal;
    c->ibuf = ibuf;
  }
  return (P.off + kAlign - 1) / kAlign * kAlign;
}

// Entry of the rediscretised Q1 matrix between node (i,j,k) and its
// neighbour at offset d, from the cell coefficients kap (nullptr = 1):
// the sum over the cells containing both nodes of kappa_c times the element
// matrix entry, which depends only on the number of nonzero components of d.
double q1_entry(int dim, int n, const std::vector<double>* kap, int i, int j, int k, int dx,
                int dy, int dz) {
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
          ks += (*kap)[cell];
        }
      }
  return dim == 3 ? (h / 12.0) * f3[cls] * ks : (1.0 / 6.0) * f2[cls] * ks;
}

// Dense coarsest matrix and its Cholesky factor (row major, lower).
mg_status coarse_factor(mg_ctx* c, hipStream_t s) {
  const Level& Lv = c->lv[c->L - 1];
  const int dim = c->o.dim, n = Lv.g.n, mi = n - 1, m = c->m;
  std::vector<double> kap;
  if (c->kappa) {
    kap.resize(ipow(n, dim));
    HIP_TRY(hipMemcpyAsync(kap.data(), Lv.kap64, kap.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<double> A((size_t)m * m, 0.0);
  for (int q = 0; q < m; ++q) {
    const int i = q % mi + 1, j = (q / mi) % mi + 1, k = dim == 3 ? q / (mi * mi) + 1 : 0;
    for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int qi = i + dx, qj = j + dy, qk = k + dz;
          if (qi < 1 || qi > mi || qj < 1 || qj > mi) continue;
          if (dim == 3 && (qk < 1 || qk > mi)) continue;
          const int q2 = (qi - 1) + mi * (qj - 1) + (dim == 3 ? mi * mi * (qk - 1) : 0);
          A[(size_t)q * m + q2] = q1_entry(dim, n, c->kappa ? &kap : nullptr, i, j, k, dx, dy, dz);
        }
  }
  // Cholesky A = L L^T (lower, row major), in place.
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
  HIP_TRY(hipMemcpyAsync(c->Lc, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MG_OK;
}

// Rows of level l ordered by colour (colour 0 first), lexicographic within a
// colour; row lengths from the number of unknown neighbours per direction.
mg_status build_csr(mg_ctx* c, int l, hipStream_t s) {
  Level& Lv = c->lv[l];
  const int dim = c->o.dim, n = Lv.g.n;
  const int rows = Lv.rows;
  std::vector<int> rowmap(rows), rowptr(rows + 1);
  rowptr[0] = 0;
  int idx = 0;
  auto cnt = [&](int i) { return 1 + (i > 1) + (i < n - 1); };
  for (int colour = 0; colour < 2; ++colour) {
    if (colour == 1) Lv.coff[1] = idx;
    for (int k = (dim == 3 ? 1 : 0); k <= (dim == 3 ? n - 1 : 0); ++k)
      for (int j = 1; j <= n - 1; ++j)
        for (int i = 1; i <= n - 1; ++i) {
          if (((i + j + k) & 1) != colour) continue;
          rowmap[idx] = (int)(i + j * Lv.g.sy + (long)k * Lv.g.sz);
          const int len = cnt(i) * cnt(j) * (dim == 3 ? cnt(k) : 1);
          rowptr[idx + 1] = rowptr[idx] + len;
          ++idx;
        }
  }
  Lv.coff[0] = 0;
  Lv.coff[2] = rows;
  if (idx != rows || rowptr[rows] != Lv.nnz)
    return fail(MG_E_ARG, "internal: CSR layout mismatch on level %d", l);
  HIP_TRY(hipMemcpyAsync(Lv.rowmap, rowmap.data(), rows * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(Lv.rowptr, rowptr.data(), (rows + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  const double selem = dim == 3 ? (1.0 / n) / 12.0 : 1.0 / 6.0;
  launch_csr_build<double>(Lv.g, Lv.kap64, selem, rows, Lv.rowmap, Lv.rowptr, Lv.col, Lv.val64, s);
  if (Lv.val32)
    launch_csr_build<float>(Lv.g, Lv.kap64, selem, rows, Lv.rowmap, Lv.rowptr, Lv.col, Lv.val32, s);
  HIP_TRY(hipGetLastError());
  // the host vectors must stay alive until the copies finish
  HIP_TRY(hipStreamSynchronize(s));
  auto fill = [&](auto& op, auto* val) {
    op.rowptr = Lv.rowptr;
    op.col = Lv.col;
    op.val = val;
    op.rowmap = Lv.rowmap;
    op.rows = rows;
    for (int q = 0; q < 3; ++q) op.coff[q] = Lv.coff[q];
  };
  fill(Lv.csr64, Lv.val64);
  if (Lv.val32) fill(Lv.csr32, Lv.val32);
  return MG_OK;
}

void set_stencil(mg_ctx* c, int l) {
  Level& Lv = c->lv[l];
  const double h = 1.0 / Lv.g.n;
  double wc, w1, w2, s;
  if (c->o.dim == 2) {
    wc = 8.0 / 3.0;
    w1 = -1.0 / 3.0;
    w2 = -1.0 / 3.0;
    s = 1.0 / 6.0;
  } else {
    wc = 8.0 * h / 3.0;
    w1 = -h / 6.0;
    w2 = -h / 12.0;
    s = h / 12.0;
  }
  const int kind = c->kappa ? OP_KAPPA : OP_CONST;
  Lv.st64 = StencilOp<double>{kind, Lv.kap64, wc, w1, w2, s};
  Lv.st32 = StencilOp<float>{kind, Lv.kap32, (float)wc, (float)w1, (float)w2, (float)s};
}

// ---------------------------------------------------------------------------
// typed access to per-level buffers and operators
// ---------------------------------------------------------------------------
template <typename T> struct Bufs;
template <> struct Bufs<double> {
  static double* x(Level& L) { return L.x64; }
  static double* b(Level& L) { return L.b64; }
  static double* t(Level& L) { return L.t64; }
  static double* r(Level& L) { return L.r64; }
  static const StencilOp<double>& st(Level& L) { return L.st64; }
  static const CsrOp<double>& csr(Level& L) { return L.csr64; }
};
template <> struct Bufs<float> {
  static float* x(Level& L) { return L.x32; }
  static float* b(Level& L) { return L.b32; }
  static float* t(Level& L) { return L.t32; }
  static float* r(Level& L) { return L.r32; }
  static const StencilOp<float>& st(Level& L) { return L.st32; }
  static const CsrOp<float>& csr(Level& L) { return L.csr32; }
};

// profiling hooks: bracket level-0 launches of the selected kernel class
enum ProfKind { PK_SMOOTH = 0, PK_RESID = 1, PK_RESTRICT = 2, PK_PROLONG = 3 };

struct ProfScope {
  mg_ctx* c;
  hipStream_t s;
  bool on;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(mg_ctx* ctx, int kind, int level, hipStream_t st)
      : c(ctx), s(st), on(ctx->prof_on && level == 0 && kind == ctx->prof_kernel) {
    if (!on) return;
    for (int q = 0; q < 2; ++q) {
      hipEvent_t e;
      if (!c->ev_pool.empty()) {
        e = c->ev_pool.back();
        c->ev_pool.pop_back();
      } else {
        hipEventCreate(&e);
      }
      (q == 0 ? a : b) = e;
    }
    hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!on) return;
    hipEventRecord(b, s);
    c->ev_pending.emplace_back(a, b);
  }
};

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
}

template <typename T>
void op_smooth(mg_ctx* c, int l, int kind, const T* xin, const T* b, T* xout, hipStream_t s) {
  Level& Lv = c->lv[l];
  ProfScope ps(c, PK_SMOOTH, l, s);
  if (c->csr)
    launch_csr_smooth<T>(Lv.g, Bufs<T>::csr(Lv), kind, xin, b, xout, (T)c->o.omega, s);
  else
    launch_smooth<T>(Lv.g, Bufs<T>::st(Lv), kind, xin, b, xout, (T)c->o.omega, s);
}

template <typename T>
void op_residual(mg_ctx* c, int l, const T* x, const T* b, T* r, double* partials,
                 hipStream_t s) {
  Level& Lv = c->lv[l];
  ProfScope ps(c, PK_RESID, l, s);
  if (c->csr)
    launch_csr_residual<T>(Lv.g, Bufs<T>::csr(Lv), x, b, r, partials, s);
  else
    launch_residual<T>(Lv.g, Bufs<T>::st(Lv), x, b, r, partials, s);
}

template <typename T>
long residual_blocks(mg_ctx* c, int l) {
  return c->csr ? csr_residual_blocks(c->lv[l].rows) : grid_blocks(c->lv[l].g);
}

template <typename T>
void op_resid_restrict(mg_ctx* c, int l, const T* x, const T* b, T* bc, hipStream_t s) {
  Level& Lv = c->lv[l];
  T* r = Bufs<T>::r(Lv);
  ProfScope ps(c, PK_RESTRICT, l, s);
  if (c->csr)
    launch_csr_residual<T>(Lv.g, Bufs<T>::csr(Lv), x, b, r, nullptr, s);
  else
    launch_residual<T>(Lv.g, Bufs<T>::st(Lv), x, b, r, nullptr, s);
  launch_restrict<T>(Lv.g, c->lv[l + 1].g, r, bc, s);
}

// Smoothing on level l from *cur (or from 0 if *zero), ping-ponging between
// *cur and *spare; on return *cur holds the smoothed iterate.
template <typename T>
void smooth_level(mg_ctx* c, int l, bool pre, T** cur, T** spare, bool* zero, const T* b,
                  hipStream_t s) {
  const int nu = pre ? c->o.nu_pre : c->o.nu_post;
  for (int it = 0; it < nu; ++it) {
    if (c->o.smoother == MG_SMOOTH_JACOBI) {
      op_smooth<T>(c, l, SM_JACOBI, *zero ? nullptr : *cur, b, *spare, s);
      std::swap(*cur, *spare);
      *zero = false;
    } else {
      const int first = pre ? SM_RB0 : SM_RB1;
      const int second = pre ? SM_RB1 : SM_RB0;
      for (int kind : {first, second}) {
        op_smooth<T>(c, l, kind, *zero ? nullptr : *cur, b, *spare, s);
        std::swap(*cur, *spare);
        *zero = false;
      }
    }
  }
}

// One V-cycle (Algorithm 1) for A_0 x = b starting from x0 (or from 0 when
// x0_zero); the result is written back to x0.  Levels >= 1 and the spare
// level-0 buffer are internal.
template <typename T>
void enqueue_vcycle(mg_ctx* c, T* x0, T* spare0, const T* b0, bool x0_zero, hipStream_t s) {
  const int L = c->L;
  if (L == 1) {
    launch_coarse_solve<T>(c->lv[0].g, c->Lc, c->m, b0, x0, s);
    return;
  }
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
  for (int l = 0; l < L - 1; ++l) {
    bool zero = (l > 0) || x0_zero;
    smooth_level<T>(c, l, true, &cur[l], &spare[l], &zero, bb[l], s);
    if (zero) {  // no pre-smoothing: materialise x = 0
      launch_fill<T>(cur[l], c->lv[l].g.nodes, T(0), s);
    }
    op_resid_restrict<T>(c, l, cur[l], bb[l], Bufs<T>::b(c->lv[l + 1]), s);
  }
  launch_coarse_solve<T>(c->lv[L - 1].g, c->Lc, c->m, bb[L - 1], cur[L - 1], s);
  for (int l = L - 2; l >= 0; --l) {
    {
      ProfScope ps(c, PK_PROLONG, l, s);
      launch_prolong_add<T>(c->lv[l].g, c->lv[l + 1].g, cur[l + 1], cur[l], s);
    }
    bool zero = false;
    smooth_level<T>(c, l, false, &cur[l], &spare[l], &zero, bb[l], s);
  }
  if (cur[0] != x0) launch_copy<T>(cur[0], x0, c->lv[0].g.nodes, s);
}

// FP64 iteration body: one V-cycle on u, then r = b - A u and ||r||^2.
void enqueue_cycle64(mg_ctx* c, double* u, const double* b, hipStream_t s) {
  Level& L0 = c->lv[0];
  enqueue_vcycle<double>(c, u, L0.t64, b, false, s);
  op_residual<double>(c, 0, u, b, L0.r64, c->partials, s);
  launch_reduce_final(c->partials, residual_blocks<double>(c, 0), c->scal + 0, s);
}

// FP32-IR iteration body: b32 = float(r/||r||), c = V-cycle32(0, b32),
// u += ||r|| c, r = b - A u, ||r||^2.
void enqueue_cycle_ir(mg_ctx* c, double* u, const double* b, hipStream_t s) {
  Level& L0 = c->lv[0];
  launch_scale_cast(L0.g, L0.r64, c->scal + 0, L0.b32, s);
  enqueue_vcycle<float>(c, L0.x32, L0.t32, L0.b32, true, s);
  launch_ir_update(L0.g, u, L0.x32, c->scal + 0, s);
  op_residual<double>(c, 0, u, b, L0.r64, c->partials, s);
  launch_reduce_final(c->partials, residual_blocks<double>(c, 0), c->scal + 0, s);
}

void drop_graph(mg_ctx* c) {
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gkey[0] = c->gkey[1] = c->gkey[2] = nullptr;
}

// Run one iteration body: replay the cached graph (captured on first use
// for these buffers) or launch eagerly.
mg_status run_iteration(mg_ctx* c, double* u, const double* b, hipStream_t s) {
  const bool eager = (c->o.flags & MG_FLAG_NO_GRAPH) || c->prof_on;
  auto body = [&](hipStream_t st) {
    if (c->ir)
      enqueue_cycle_ir(c, u, b, st);
    else
      enqueue_cycle64(c, u, b, st);
  };
  if (eager) {
    body(s);
    HIP_TRY(hipGetLastError());
    return MG_OK;
  }
  const void* key[3] = {u, b, (const void*)(long)c->ir};
  if (!c->gexec || memcmp(key, c->gkey, sizeof key) != 0) {
    drop_graph(c);
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    body(c->cap);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(c->cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(MG_E_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                  hipGetErrorString(ee));
    }
    hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      c->gexec = nullptr;
      return fail(MG_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    }
    memcpy(c->gkey, key, sizeof key);
  }
  HIP_TRY(hipGraphLaunch(c->gexec, s));
  return MG_OK;
}

mg_status read_scalar(mg_ctx* c, int idx, double* out, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(c->pinned + idx, c->scal + idx, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = c->pinned[idx];
  return MG_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

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
}

size_t mg_footprint_bytes(const mg_options* o) {
  std::string why;
  if (!valid_options(o, why)) {
    fail(MG_E_ARG, "%s", why.c_str());
    return 0;
  }
  // the footprint with a coefficient is the larger one
  return plan(*o, true, nullptr, nullptr);
}

mg_status mg_setup(const mg_options* o, const double* kappa_dev, void* stream, mg_ctx** out) {
  if (!out) return fail(MG_E_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_options(o, why)) return fail(MG_E_ARG, "%s", why.c_str());
  hipStream_t s = as_stream(stream);
  mg_ctx* c = new mg_ctx();
  c->o = *o;
  c->L = o->levels;
  c->kappa = kappa_dev != nullptr;
  c->ir = o->precision == MG_PREC_FP32_IR;
  c->csr = o->op == MG_OP_CSR;
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
  if (hipHostMalloc(&c->pinned, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
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
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return bail(fail(MG_E_HIP, "setup kernels failed"));
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  if (c->cap) hipStreamSynchronize(c->cap);
  drop_graph(c);
  for (auto& pr : c->ev_pending) {
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
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
  Level& L0 = c->lv[0];
  *iters = 0;
  if (hist) hist[0] = 1.0;
  launch_fill<double>(u, L0.g.nodes, 0.0, s);
  launch_norm2_partial<double>(L0.g, b, c->partials, s);
  launch_reduce_final(c->partials, grid_blocks(L0.g), c->scal + 1, s);
  HIP_TRY(hipGetLastError());
  double nb2 = 0.0;
  mg_status st = read_scalar(c, 1, &nb2, s);
  if (st != MG_OK) return st;
  if (!std::isfinite(nb2)) return fail(MG_E_NONFINITE, "b holds NaN or Inf");
  if (nb2 == 0.0) return MG_OK;
  const double nb = std::sqrt(nb2);
  if (c->ir) {
    // r = b - A 0 = b and ||r||^2, the state every refinement step expects
    op_residual<double>(c, 0, u, b, L0.r64, c->partials, s);
    launch_reduce_final(c->partials, residual_blocks<double>(c, 0), c->scal + 0, s);
    HIP_TRY(hipGetLastError());
  }
  for (int k = 1; k <= c->o.max_iter; ++k) {
    st = run_iteration(c, u, b, s);
    if (st != MG_OK) return st;
    double n2 = 0.0;
    st = read_scalar(c, 0, &n2, s);
    if (st != MG_OK) return st;
    if (c->prof_on) prof_collect(c);
    const double rho = std::sqrt(n2) / nb;
    *iters = k;
    if (hist) hist[k] = rho;
    if (!std::isfinite(rho) || rho > 1e3)
      return fail(MG_E_DIVERGED, "relative residual %g after %d cycles", rho, k);
    if (rho <= tol) return MG_OK;
  }
  return fail(MG_E_MAXIT, "no convergence to %g in %d cycles", tol, c->o.max_iter);
}

// ---- single steps -----------------------------------------------------------
namespace {
mg_status check_step(mg_ctx* c, int level, int prec, bool need_next) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  if (level < 0 || level >= c->L || (need_next && level >= c->L - 1))
    return fail(MG_E_ARG, "level %d out of range", level);
  if (prec != MG_PREC_FP64 && prec != MG_PREC_FP32_IR) return fail(MG_E_ARG, "bad precision");
  if (prec == MG_PREC_FP32_IR && !c->ir)
    return fail(MG_E_STATE, "FP32 operators exist only in MG_PREC_FP32_IR contexts");
  return MG_OK;
}
}  // namespace

mg_status mg_apply_residual(mg_ctx* c, int level, int prec, const void* x, const void* b, void* r,
                            void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!x || !b || !r) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  if (prec == MG_PREC_FP64) {
    launch_fill<double>((double*)r, c->lv[level].g.nodes, 0.0, s);
    op_residual<double>(c, level, (const double*)x, (const double*)b, (double*)r, nullptr, s);
  } else {
    launch_fill<float>((float*)r, c->lv[level].g.nodes, 0.f, s);
    op_residual<float>(c, level, (const float*)x, (const float*)b, (float*)r, nullptr, s);
  }
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_smooth(mg_ctx* c, int level, int prec, int step, const void* x_in,
                          const void* b, void* x_out, void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!b || !x_out) return fail(MG_E_ARG, "NULL vector");
  if (step < 0 || step > 4) return fail(MG_E_ARG, "step must be 0..4");
  hipStream_t s = as_stream(stream);
  Level& Lv = c->lv[level];
  auto run = [&](auto tag) {
    using T = decltype(tag);
    T* out = (T*)x_out;
    const T* in = (const T*)x_in;
    const T* bb = (const T*)b;
    launch_fill<T>(out, Lv.g.nodes, T(0), s);
    if (step <= 2) {
      op_smooth<T>(c, level, step, in, bb, out, s);
      return;
    }
    // full red-black sweep through the level's spare buffer
    T* tmp = Bufs<T>::t(Lv);
    const int k1 = step == 3 ? SM_RB0 : SM_RB1, k2 = step == 3 ? SM_RB1 : SM_RB0;
    op_smooth<T>(c, level, k1, in, bb, tmp, s);
    op_smooth<T>(c, level, k2, tmp, bb, out, s);
  };
  if (prec == MG_PREC_FP64) run(double(0)); else run(float(0));
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_restrict(mg_ctx* c, int level, int prec, const void* r, void* bc,
                            void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!r || !bc) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  const Geo& gf = c->lv[level].g;
  const Geo& gc = c->lv[level + 1].g;
  if (prec == MG_PREC_FP64) {
    launch_fill<double>((double*)bc, gc.nodes, 0.0, s);
    launch_restrict<double>(gf, gc, (const double*)r, (double*)bc, s);
  } else {
    launch_fill<float>((float*)bc, gc.nodes, 0.f, s);
    launch_restrict<float>(gf, gc, (const float*)r, (float*)bc, s);
  }
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_residual_restrict(mg_ctx* c, int level, int prec, const void* x, const void* b,
                                     void* bc, void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!x || !b || !bc) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  const Geo& gc = c->lv[level + 1].g;
  if (prec == MG_PREC_FP64) {
    launch_fill<double>((double*)bc, gc.nodes, 0.0, s);
    op_resid_restrict<double>(c, level, (const double*)x, (const double*)b, (double*)bc, s);
  } else {
    launch_fill<float>((float*)bc, gc.nodes, 0.f, s);
    op_resid_restrict<float>(c, level, (const float*)x, (const float*)b, (float*)bc, s);
  }
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_prolong_add(mg_ctx* c, int level, int prec, const void* e, void* x,
                               void* stream) {
  mg_status st = check_step(c, level, prec, true);
  if (st != MG_OK) return st;
  if (!e || !x) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  const Geo& gf = c->lv[level].g;
  const Geo& gc = c->lv[level + 1].g;
  if (prec == MG_PREC_FP64)
    launch_prolong_add<double>(gf, gc, (const double*)e, (double*)x, s);
  else
    launch_prolong_add<float>(gf, gc, (const float*)e, (float*)x, s);
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_apply_coarse_solve(mg_ctx* c, int prec, const void* bc, void* xc, void* stream) {
  mg_status st = check_step(c, c ? c->L - 1 : 0, prec, false);
  if (st != MG_OK) return st;
  if (!bc || !xc) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  const Geo& g = c->lv[c->L - 1].g;
  if (prec == MG_PREC_FP64) {
    launch_fill<double>((double*)xc, g.nodes, 0.0, s);
    launch_coarse_solve<double>(g, c->Lc, c->m, (const double*)bc, (double*)xc, s);
  } else {
    launch_fill<float>((float*)xc, g.nodes, 0.f, s);
    launch_coarse_solve<float>(g, c->Lc, c->m, (const float*)bc, (float*)xc, s);
  }
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_vcycle(mg_ctx* c, int prec, void* x, const void* b, void* stream) {
  mg_status st = check_step(c, 0, prec, false);
  if (st != MG_OK) return st;
  if (!x || !b) return fail(MG_E_ARG, "NULL vector");
  hipStream_t s = as_stream(stream);
  Level& L0 = c->lv[0];
  if (prec == MG_PREC_FP64)
    enqueue_vcycle<double>(c, (double*)x, L0.t64, (const double*)b, false, s);
  else
    enqueue_vcycle<float>(c, (float*)x, L0.t32, (const float*)b, false, s);
  HIP_TRY(hipGetLastError());
  return MG_OK;
}

mg_status mg_norm2(mg_ctx* c, int level, int prec, const void* v, double* out, void* stream) {
  mg_status st = check_step(c, level, prec, false);
  if (st != MG_OK) return st;
  if (!v || !out) return fail(MG_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  const Geo& g = c->lv[level].g;
  if (prec == MG_PREC_FP64)
    launch_norm2_partial<double>(g, (const double*)v, c->partials, s);
  else
    launch_norm2_partial<float>(g, (const float*)v, c->partials, s);
  launch_reduce_final(c->partials, grid_blocks(g), c->scal + 2, s);
  HIP_TRY(hipGetLastError());
  return read_scalar(c, 2, out, s);
}

mg_status mg_profile_enable(mg_ctx* c, int kernel_id, int enable) {
  if (!c) return fail(MG_E_ARG, "ctx is NULL");
  if (kernel_id < 0 || kernel_id > 3) return fail(MG_E_ARG, "kernel_id must be 0..3");
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
