// Internal definitions shared by the solver runtime and the serving
// scheduler: the context (level hierarchy and its device buffers) and the
// recorded form of one kernel launch of a V-cycle ("op"), which the
// scheduler fuses across requests.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/mg.h"
#include "mg_internal.h"

namespace mg {

struct Level {
  Geo g;
  // FP64 vectors (x and b of level 0 are the caller's)
  double *x64 = nullptr, *b64 = nullptr, *t64 = nullptr, *r64 = nullptr;
  // preconditioned CG on level 0 (MG_FLAG_PCG): direction, A times it,
  // preconditioned residual, residual and previous residual
  double *p64 = nullptr, *q64 = nullptr, *z64 = nullptr, *rk64 = nullptr, *ro64 = nullptr;
  // FP32 vectors (FP32_IR contexts)
  float *x32 = nullptr, *b32 = nullptr, *t32 = nullptr, *r32 = nullptr;
  // two colour-split iterates (even half, then odd half from (nodes+1)/2),
  // zero on the boundary, on levels whose red-black runs keep x split
  double* xs64[2] = {nullptr, nullptr};
  float* xs32[2] = {nullptr, nullptr};
  // coefficients per cell
  double* kap64 = nullptr;
  float* kap32 = nullptr;
  // CSR
  int *rowptr = nullptr, *col = nullptr, *rowmap = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  int rows = 0;
  long nnz = 0;
  int coff[9] = {};
  StencilParams<double> st64{};
  StencilParams<float> st32{};
  CsrOp<double> csr64{};
  CsrOp<float> csr32{};
};

enum OpCode {
  OC_SMOOTH = 0,
  OC_RESID,
  OC_RESTRICT,
  OC_PROLONG,
  OC_COARSE,
  OC_NORM2,
  OC_REDUCE,
  OC_SCALE_CAST,
  OC_IR_UPDATE,
  OC_TAIL,
  OC_FILL,
  OC_COPY,
  OC_CSR_SMOOTH,
  OC_CSR_RESID,
  OC_HEAD,      // residual partial sums + first smoothing step (sub: kind)
  OC_CSR_HEAD,
  OC_SMOOTH2,        // two red-black half-sweeps in one pass (sub: first kind | zero << 4)
  OC_SMOOTH_PRO,     // x + P e then one smoothing step (sub: kind), item.e = e
  OC_APPLY_DOT,      // q = A x with partials of x.q
  OC_CSR_APPLY_DOT,
  OC_PCG,            // CG vector kernel (sub: PcgOp), pointers in ext[]
  OC_ZERO_BOUNDARY,  // c = 0 on the boundary nodes (FP64)
  OC_RESID_RESTRICT,  // b_c = R (b - A x) in one pass (sub: x colour-split)
  OC_RESTRICT_XCOLS,  // the coarse columns OC_RESID_RESTRICT leaves
};

// CG vector kernels (OpRec::sub of OC_PCG)
enum PcgOp { PO_DOTS2 = 0, PO_SCALARS, PO_DIR, PO_UPDATE, PO_ZSCALE };

// One kernel launch of a cycle for one request.  Ops with equal keys (all
// fields but `item`, `level` and `csr`) can run as one batched launch.
struct OpRec {
  int code = 0;
  int prec = 0;     // 0 double, 1 float
  // OC_SMOOTH: kind | zero << 4 | XLayout << 5 | IRU << 8;
  // OC_RESID: norm | XLayout << 5 | scaled cast << 9
  int sub = 0;
  int level = 0;    // level index within its context (profiling)
  Geo g{}, gc{};    // level geometry and the next coarser one
  int opkind = 0;   // OP_CONST / OP_KAPPA / OP_MASS
  double wc = 0, w1 = 0, w2 = 0, s = 0, wf = 0, omega = 0;
  int m = 0;        // coarsest unknowns
  long count = 0;   // OC_REDUCE: partials; OC_FILL / OC_COPY: elements
  Item item{};
  const void* csr = nullptr;  // CsrOp<T>* (CSR ops, not batchable)
  void* ext[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // OC_PCG operands
};

bool same_key(const OpRec& a, const OpRec& b);
bool batchable(const OpRec& a);
// Launch ops[0..n) (equal keys, n <= kMaxBatch) as one batched launch.
void launch_ops(const OpRec* const* ops, int n, hipStream_t s);

}  // namespace mg

struct mg_ctx {
  mg_options o{};
  int L = 0;
  bool kappa = false;
  bool ir = false;
  bool csr = false;
  int tail0 = -1;  // first level cycled by the one-workgroup tail kernel (-1: none)
  // ops emitted for the single-step entry points (caller buffers in the
  // natural layout) keep every right-hand side in the natural layout
  bool natural = false;
  // mg_solve keeps a colour-split copy of the caller's FP64 b (level 0)
  bool b0_split = false;
  // FP64 mg_solve with head fusion on a split-iterate finest level keeps
  // the finest iterate colour-split from cycle to cycle (s0on): s0at[h] is
  // the split buffer holding the even (h = 0) / odd (h = 1) half of the
  // current iterate, s0u where the last cycle's result lives (the head of
  // the next cycle writes the new even half elsewhere); the caller's u is
  // written from the halves once, after the last cycle
  bool s0on = false;
  int s0at[2] = {0, 0};
  int s0u[2] = {0, 0};
  std::vector<mg::Level> lv;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  double* Lc = nullptr;  // coarsest Cholesky factor, row major
  int m = 0;
  double* partials = nullptr;
  long npart = 0;
  double* scal = nullptr;       // device scalars: [0] residual norm^2, [1] ||b||^2, [2] scratch
  int* ibuf = nullptr;          // device ints (setup checks)
  double* tres = nullptr;       // results of a one-workgroup whole solve (status,
                                // cycles, history), kTailSolveHead + max_iter + 1
  int npinned = 0;              // doubles at `pinned`
  void* tail64 = nullptr;       // TailDesc<double> (device)
  void* tail32 = nullptr;       // TailDesc<float> (device)
  int tail_lds[2] = {0, 0};     // dynamic LDS bytes of the tail launch (FP64, FP32)
  double* pinned = nullptr;     // host pinned scalars
  hipStream_t cap = nullptr;    // private stream for graph capture
  // one cached graph per iteration kind (plain, first fused, steady fused,
  // first CG, steady CG), valid for the (u, b) it was captured with
  static constexpr int kIterKinds = 5;
  // four cached graphs per iteration kind, keyed by the (u, b) buffers and
  // the split state the iteration starts from (a split finest iterate
  // alternates between two states), so that solves alternating between two
  // solution buffers replay their graphs
  static constexpr int kGraphSlots = 4;
  hipGraphExec_t gexec[kIterKinds][kGraphSlots] = {};
  const void* gkey[kIterKinds][kGraphSlots][3] = {};
  int gstate[kIterKinds][kGraphSlots][2] = {};  // s0at, s0u after the iteration (codes)
  int glast[kIterKinds] = {};  // most recently used slot
  // profiling
  int prof_kernel = -1;
  bool prof_on = false;
  long prof_launches = 0;
  double prof_ms = 0.0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<hipEvent_t> ev_spare;  // recorded but not read; back to ev_pool
};

namespace mg {

// Ops of one iteration of mg_solve for the context (u, b: level-0 FP64
// vectors), in launch order.
void record_iteration(mg_ctx* c, double* u, const double* b, std::vector<OpRec>& out);
// Ops that prepare a solve: u = 0, ||b||^2 into scal[1], and for FP32-IR
// r = b with ||r||^2 in scal[0].
void record_prologue(mg_ctx* c, double* u, const double* b, std::vector<OpRec>& out);
size_t plan_bytes(const mg_options& o, bool has_kappa);

}  // namespace mg
