/*
 * mg.h -- C ABI of the Q1 geometric-multigrid library for MI355X (gfx950).
 *
 * The library solves A u = b, where A = K + sigma M is the conforming Q1
 * finite element stiffness matrix K of -div(kappa grad u) plus sigma >= 0
 * times the mass matrix M (sigma = 0: the Poisson-type problem; sigma =
 * 2/dt: the Crank-Nicolson step of the heat equation, Sec. 6.2) on the unit
 * square (dim = 2) or unit cube (dim = 3), n cells per direction,
 * homogeneous Dirichlet data on the unknowns, with the multigrid V-cycle of
 * the paper's Algorithm 1 (Sec. 5.3) on a hierarchy of nested uniformly
 * refined meshes (Sec. 5.1).  One GPU holds the whole hierarchy.
 *
 * Layouts (all arrays x fastest):
 *   node vectors  (n_l+1)^dim entries, all nodes of level l including the
 *                 boundary; boundary entries of vectors the library writes
 *                 are 0, boundary entries of inputs are ignored;
 *   cell arrays   n^dim entries (coefficient kappa per cell).
 * Level 0 is the finest mesh (n cells), level l has n_l = n / 2^l cells.
 *
 * Memory: "device" pointers are HIP device memory owned by the caller
 * (allocated by any allocator, e.g. PyTorch); "host" pointers are ordinary
 * host memory.  The library never frees caller memory.  A context owns one
 * device allocation (its arena) for the hierarchy.
 *
 * Streams: every call that takes `stream` (a hipStream_t, NULL = the null
 * stream) enqueues its device work on that stream.  Calls that return
 * results to the host (mg_solve, mg_norm2) synchronise that stream.
 *
 * Errors: every call returns an mg_status; on failure mg_last_error()
 * returns a message for the calling thread.  A context is not thread safe;
 * distinct contexts are.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

typedef enum {
  MG_OK = 0,
  MG_E_ARG = 1,        /* invalid argument or option */
  MG_E_NOMEM = 2,      /* device allocation failed / budget exceeded */
  MG_E_HIP = 3,        /* a HIP runtime call failed */
  MG_E_NOT_SPD = 4,    /* coarsest matrix has a non-positive Cholesky pivot */
  MG_E_MAXIT = 5,      /* max_iter cycles done without reaching tol */
  MG_E_DIVERGED = 6,   /* residual grew above 1e3 ||b|| or became NaN */
  MG_E_NONFINITE = 7,  /* NaN or Inf in an input */
  MG_E_STATE = 8       /* call not valid in the current state */
} mg_status;

typedef enum { MG_OP_STENCIL = 0, MG_OP_CSR = 1 } mg_opfmt;
/* Smoothers (Eq. (1), Sec. 5.3): damped Jacobi; red-black Gauss-Seidel
 * with the unknowns of one colour (sum of node coordinates mod 2) updated
 * simultaneously; multicolour Gauss-Seidel with the 2^dim colours
 * sum_d (x_d mod 2) 2^d, whose unknowns are pairwise uncoupled, so one
 * in-place pass per colour is an exact Gauss-Seidel sweep in the
 * colour-sorted numbering (colours in order for pre-, in reverse order for
 * post-smoothing).  MG_SMOOTH_GS runs on node kernels and CSR rows blocked
 * by its colours, without the fused head and prolongation steps, and not
 * in the server. */
typedef enum { MG_SMOOTH_JACOBI = 0, MG_SMOOTH_RBGS = 1, MG_SMOOTH_GS = 2 } mg_smoother;
typedef enum { MG_PREC_FP64 = 0, MG_PREC_FP32_IR = 1 } mg_precision;
/* Cycle shape: how the coarse residual equation of a level is solved --
 * by one coarse cycle (V, Algorithm 1), by two (W), or by an F-cycle
 * followed by a V-cycle (F); directly above the coarsest level always
 * exactly, once.  The paper mentions other cycle shapes besides the V-cycle
 * (Sec. 5.3). */
typedef enum { MG_CYCLE_V = 0, MG_CYCLE_W = 1, MG_CYCLE_F = 2 } mg_cycle;

/* Flags (mg_options.flags). */
#define MG_FLAG_NO_GRAPH 1   /* launch kernels one by one instead of replaying
                                one captured HIP graph per cycle */
#define MG_FLAG_NO_TAIL 2    /* cycle every level with grid-wide launches, also
                                the small coarse levels that otherwise run
                                inside one workgroup */
#define MG_FLAG_NO_FUSE 4    /* launch the fused steps separately (same
                                results bitwise): the stopping residual of an
                                FP64 cycle, otherwise computed in one pass
                                with the next cycle's first pre-smoothing
                                step, and on 3D stencil levels with n >= 32
                                (coarse levels of a graph-replayed solve:
                                n >= 96; per-cell kappa: FP64 only) the
                                prolongation, otherwise done while the first
                                post-smoothing step stages x */
#define MG_FLAG_PAIR 16      /* on 3D stencil levels with n >= 32 (coarse
                                levels of a graph-replayed solve: n >= 96),
                                launch
                                consecutive red-black half-sweeps as one pass
                                each (x, b and the result cross HBM once per
                                pair; a halo of width 2 is recomputed in
                                LDS).  Same results bitwise; slower than
                                separate half-sweeps on MI355X, whose
                                half-sweep is HBM-bound while the pair is
                                bound by LDS traffic and occupancy. */
#define MG_FLAG_PCG 8        /* mg_solve runs conjugate gradients
                                preconditioned by one V-cycle per iteration
                                (multigrid as a Krylov preconditioner,
                                Sec. 1) instead of the plain cycle iteration
                                (Sec. 5.5.1); needs a symmetric cycle
                                (nu_pre == nu_post).  In FP32_IR contexts the
                                preconditioning cycle runs in FP32 on
                                r / s, s the power of two with
                                s / 2 <= ||r|| < s.  Iterations and the history then
                                count CG iterations, with the recursively
                                updated residual.  V- or W-cycles only (the
                                F-cycle is not symmetric).  Not for the
                                server. */
#define MG_FLAG_NO_SPLIT 64  /* keep every vector in the natural layout.
                                By default the right-hand sides of the 3D
                                matrix-free levels with even n whose vectors
                                reach 64 MB are stored colour-split --
                                even-indexed nodes first, then odd-indexed
                                ones, which for even n are the two red-black
                                colours -- so a half-sweep reads its colour's
                                half only (mg_solve without CG keeps a split
                                copy of an FP64 b); with red-black smoothing
                                and no kappa the iterate is also kept split
                                between the first and the last half-sweep of
                                each smoothing run (two more vectors per such
                                level), so the middle half-sweeps write only
                                the colour they update.  Same results
                                bitwise. */
#define MG_FLAG_WARM 32      /* mg_solve starts from the u it is given (a
                                warm start, e.g. the previous time step)
                                instead of u = 0: it sets u's boundary
                                entries to 0, computes hist[0] = ||b - A u|| /
                                ||b|| and returns after 0 iterations if that
                                already meets tol.  Not for the server. */

typedef struct {
  int dim;          /* 2 or 3 */
  int n;            /* cells per direction on the finest level, >= 2 */
  int levels;       /* >= 1; n divisible by 2^(levels-1); n >> (levels-1) >= 2 */
  int op;           /* mg_opfmt: matrix-free stencil or CSR matrices */
  int smoother;     /* mg_smoother */
  int nu_pre;       /* pre-smoothing sweeps per level, >= 0 */
  int nu_post;      /* post-smoothing sweeps per level, >= 0 */
  double omega;     /* Jacobi damping, 0 < omega <= 1 (ignored for RBGS) */
  int precision;    /* mg_precision */
  int max_iter;     /* maximum number of cycles / refinement steps, >= 1 */
  int flags;        /* MG_FLAG_* */
  int cycle;        /* mg_cycle */
  double sigma;     /* mass shift: A = K + sigma M on every level, finite,
                       >= 0.  With sigma > 0 a matrix-free stencil context
                       takes no kappa (kappa = 1), MG_FLAG_PAIR is refused,
                       and the server refuses the request. */
} mg_options;

/* Fill *o with the defaults: 3D, n = 64, levels = 6, stencil, red-black,
 * V(2,2), omega = 2/3, FP64, max_iter = 100, flags = 0, V-cycle,
 * sigma = 0. */
void mg_options_default(mg_options* o);

/* Device bytes that mg_setup(o, ...) allocates for its arena: the larger of
 * the footprints with and without a kappa_dev, so an upper bound either
 * way; 0 if the options are invalid. */
size_t mg_footprint_bytes(const mg_options* o);

/* Build the level hierarchy (Sec. 5.1): coefficients per level, operators
 * (stencil data or CSR matrices with rows blocked by colour, Sec. 4.2.6),
 * and the FP64 Cholesky factor of the coarsest matrix.
 *   kappa_dev  device, n^dim cell coefficients (kappa > 0, finite), or NULL
 *              for kappa = 1 (the Poisson problem).  Copied; the caller may
 *              free it after the call returns.
 *   stream     hipStream_t used for setup work (synchronised before return).
 *   out        receives the new context.
 * Coarse coefficients are the geometric mean of the 2^dim children.
 * Errors: MG_E_ARG (options, kappa <= 0), MG_E_NONFINITE (kappa), MG_E_NOMEM,
 * MG_E_NOT_SPD, MG_E_HIP. */
mg_status mg_setup(const mg_options* o, const double* kappa_dev, void* stream,
                   mg_ctx** out);

/* Solve A u = b to a relative residual ||b - A u||_2 / ||b||_2 <= tol
 * (2-norm over the unknowns), starting from u = 0 (or from the given u with
 * MG_FLAG_WARM), one V(nu_pre, nu_post) cycle per iteration (Sec. 5.5.1).
 * With MG_PREC_FP32_IR each iteration is
 * one FP32 V-cycle from 0 on float(r / s), r the FP64 residual and s the
 * power of two with s / 2 <= ||b|| < s (exact scaling), followed by the FP64
 * update u += s c and residual.
 *   b_dev      device, (n+1)^dim doubles; boundary entries ignored.
 *   u_dev      device, (n+1)^dim doubles, output (and with MG_FLAG_WARM
 *              the initial iterate on its unknowns); boundary entries set
 *              to 0.  Must not alias b_dev.
 *   tol        > 0.
 *   iters      host, out: cycles done.
 *   hist_host  host, out, room for max_iter + 1 doubles (or NULL):
 *              hist[0] = 1 (warm start: the relative residual of the
 *              initial u), hist[k] = relative residual after cycle k.
 * Returns MG_OK, or MG_E_MAXIT / MG_E_DIVERGED with u, iters and hist
 * holding the last iterate; b = 0 gives u = 0, iters = 0, MG_OK.
 * MG_E_NONFINITE if b holds NaN/Inf.  Host-synchronous. */
mg_status mg_solve(mg_ctx* ctx, const double* b_dev, double* u_dev, double tol,
                   int* iters, double* hist_host, void* stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. tight serving loops or harnesses that forbid it): the
 * whole mg_solve of a small hierarchy without a context, taking every
 * buffer beyond b and u from a fixed device scratch array of 1 MiB that the
 * library holds per GPU until the process ends.  The options are those of
 * mg_setup, restricted to MG_PREC_FP64, MG_OP_STENCIL, flags = 0 and
 * max_iter <= 1000, on a hierarchy that one workgroup's LDS holds whole
 * (2D n <= 64, 3D n <= 16, e.g. the 2D 64^2 / 5-level problem) whose
 * coarsest level has at most 256 unknowns.  Arguments and results as for
 * mg_setup (kappa_dev: device, n^dim cells, or NULL) followed by mg_solve
 * (b_dev, u_dev, tol, iters, hist_host); the cycles are those of mg_solve,
 * which gives the same iterates.  Calls made from several host threads of
 * a process run one after the other, each to completion on its stream
 * (host-synchronous); the scratch keeps the last call's contents, so calls
 * from separate processes on one GPU do not share it.  Errors: MG_E_ARG
 * (options or sizes outside these limits, kappa <= 0), MG_E_NONFINITE,
 * MG_E_NOT_SPD, MG_E_MAXIT / MG_E_DIVERGED (u, iters, hist valid),
 * MG_E_HIP. */
mg_status mg_solve_noalloc(const mg_options* o, const double* kappa_dev,
                           const double* b_dev, double* u_dev, double tol,
                           int* iters, double* hist_host, void* stream);

/* Right-hand side of one Crank-Nicolson step of the heat equation (the
 * model problem of Sec. 6.2) for a context with A = K + sigma M, sigma =
 * 2/dt (kappa = 1): on the unknowns
 *   b = (sigma M - K) x0 - (sigma M + K) x1 + cf F,
 * the Crank-Nicolson equation M (u' - u)/dt + K (u' + u)/2 = (F + F')/2
 * times 2/dt with the Dirichlet values of u' moved to the right-hand side.
 *   u_dev      device, (n+1)^dim doubles: the solution at t_n on the
 *              unknowns, e.g. the previous mg_solve output; boundary entries
 *              ignored (they must be finite).
 *   guess_dev  device, (n+1)^dim doubles or NULL, in/out: on entry the
 *              solution at t_{n-1}; on return 2 u - guess on the unknowns,
 *              the linear extrapolation of the solution to t_{n+1}, a start
 *              for the next solve (MG_FLAG_WARM).  May not alias u.
 *   g0_dev     device, (n+1)^dim doubles or NULL (= 0): x0 takes c0 * g0 on
 *              the boundary nodes (the Dirichlet data at t_n); interior
 *              entries ignored.
 *   g1_dev     device, (n+1)^dim doubles or NULL: x1 = c1 * g1 on the
 *              boundary nodes, 0 inside (the Dirichlet data at t_{n+1}).
 *   F_dev      device, (n+1)^dim doubles or NULL: a load vector on the
 *              unknowns (boundary entries ignored), scaled by cf -- e.g. the
 *              load of a source profile from mg_apply_mass and cf =
 *              lambda(t_n) + lambda(t_{n+1}) for a source lambda(t) f(x).
 *   b_dev      device, (n+1)^dim doubles, out: boundary entries set to 0.
 * The same array may serve as g0 and g1 (time-separable Dirichlet data); b
 * must not alias any input.  FP64 in every context.  Errors: MG_E_ARG (NULL
 * u or b, aliasing, non-finite scalars, a context with per-cell kappa).
 * Stream-ordered, no synchronisation. */
mg_status mg_cn_rhs(mg_ctx* ctx, const double* u_dev, double* guess_dev,
                    const double* g0_dev, double c0, const double* g1_dev,
                    double c1, const double* F_dev, double cf, double* b_dev,
                    void* stream);

/* Load vector of nodal data: F = M f on the unknowns of level 0, with M the
 * Q1 mass matrix over all nodes -- the Galerkin load of the Q1 interpolant
 * of f (Sec. 2).
 *   f_dev   device, (n+1)^dim doubles, every node (boundary included).
 *   F_dev   device, (n+1)^dim doubles, out: boundary entries set to 0; must
 *           not alias f.
 * FP64.  Errors: MG_E_ARG.  Stream-ordered, no synchronisation. */
mg_status mg_apply_mass(mg_ctx* ctx, const double* f_dev, double* F_dev,
                        void* stream);

/* Release a context and its device memory (NULL is ignored). */
void mg_destroy(mg_ctx* ctx);

/* Message describing the last error of the calling thread ("" if none). */
const char* mg_last_error(void);

/* Number of levels and the cells per direction of level l. */
mg_status mg_level_info(const mg_ctx* ctx, int level, int* n_l, size_t* nodes);

/* ---------------------------------------------------------------------
 * Single steps of the cycle on caller buffers, for testing and profiling.
 * `prec` selects the element type of every vector argument: MG_PREC_FP64
 * (double) or MG_PREC_FP32_IR (float; the level's FP32 operator).  FP32
 * operators exist only in contexts set up with MG_PREC_FP32_IR.  All
 * vectors are device node vectors of level `level` unless stated otherwise;
 * outputs must not alias inputs.  Iterate and correction inputs (x, e) are
 * read on the boundary too and must hold 0 there (the eliminated Dirichlet
 * values); boundary entries of right-hand sides and residuals are ignored.
 * Each call is stream-ordered and returns without synchronising.  The
 * steps use the context's internal buffers, so they must not overlap with
 * another call on the same context.
 * ------------------------------------------------------------------- */

/* r = b - A_l x on the unknowns (Sec. 5.3, "restriction" input); r's
 * boundary entries are set to 0. */
mg_status mg_apply_residual(mg_ctx* ctx, int level, int prec, const void* x,
                            const void* b, void* r, void* stream);

/* One smoothing step (Eq. (1), Algorithm 1 pre-/post-smoothing):
 *   step 0: damped Jacobi sweep      x_out = x + omega D^-1 (b - A x)
 *   step 1: red-black half-sweep on colour 0 (sum of node coordinates even)
 *   step 2: red-black half-sweep on colour 1
 *   step 3: full red-black sweep, colour 0 then 1 (pre-smoothing order)
 *   step 4: full red-black sweep, colour 1 then 0 (post-smoothing order)
 *   step 5 + c, c < 2^dim: multicolour Gauss-Seidel update of the unknowns
 *           of colour c (MG_SMOOTH_GS numbering), the others copied; on
 *           CSR operators only in MG_SMOOTH_GS contexts (MG_E_STATE)
 * A half-sweep updates every node of its colour from the values of x at the
 * start of the half-sweep and copies the other colour.  x_in may be NULL to
 * mean x = 0.  x_out's boundary entries are set to 0. */
mg_status mg_apply_smooth(mg_ctx* ctx, int level, int prec, int step,
                          const void* x_in, const void* b, void* x_out,
                          void* stream);

/* b_coarse = P^T r (level -> level+1, Sec. 5.4): weights 1, 1/2, 1/4, 1/8,
 * no 2^-dim scaling.  r is a node vector of `level` (boundary entries
 * ignored), b_coarse a node vector of level+1. */
mg_status mg_apply_restrict(mg_ctx* ctx, int level, int prec, const void* r,
                            void* b_coarse, void* stream);

/* b_coarse = P^T (b - A_l x) (Algorithm 1: residual, then its restriction,
 * Sec. 5.4).  On 3D matrix-free levels with n >= 32 (coarse levels of a
 * context without MG_FLAG_NO_GRAPH: n >= 96) and the constant or
 * mass-shifted operator one pass, the fine residual not stored (the
 * context's residual buffer of the level serves as scratch), unless the
 * context was set up with MG_FLAG_NO_FUSE; elsewhere the residual and the
 * restriction.  b_coarse: (n_l/2+1)^dim elements, boundary entries set to
 * 0. */
mg_status mg_apply_residual_restrict(mg_ctx* ctx, int level, int prec,
                                     const void* x, const void* b,
                                     void* b_coarse, void* stream);

/* x_fine += P e_coarse (multilinear interpolation, level+1 -> level). */
mg_status mg_apply_prolong_add(mg_ctx* ctx, int level, int prec,
                               const void* e_coarse, void* x_fine,
                               void* stream);

/* x_c = A_c^-1 b_c on the coarsest level by the FP64 Cholesky factor
 * (Algorithm 1, exact coarsest solve); FP32 vectors are cast to FP64 and
 * back. */
mg_status mg_apply_coarse_solve(mg_ctx* ctx, int prec, const void* b_c,
                                void* x_c, void* stream);

/* One V-cycle on level 0: x <- V-cycle(x, b) in place, in precision prec
 * (FP32 only in FP32_IR contexts). */
mg_status mg_vcycle(mg_ctx* ctx, int prec, void* x, const void* b,
                    void* stream);

/* Squared 2-norm over the unknowns of a level node vector, summed in a
 * fixed order (run-to-run bitwise reproducible).  Host-synchronous. */
mg_status mg_norm2(mg_ctx* ctx, int level, int prec, const void* v,
                   double* out_host, void* stream);

/* ---------------------------------------------------------------------
 * Kernel timing: while enabled, mg_solve launches kernels one by one and
 * times every launch of the kernels matching `kernel_id` on level 0 with
 * HIP events: the start and end of the kernel itself, recorded by its
 * launch (hipExtLaunchKernelGGL), or, for a step of more than one kernel,
 * events on the launch stream around the step.  mg_profile_read returns
 * the number of such launches and their summed duration in milliseconds.
 *   kernel_id: 0 = smoothing sweep (Jacobi sweep or red-black half-sweep)
 *              that reads the iterate,
 *              1 = residual (with or without norm), 2 = restriction,
 *              3 = prolongation + add, 4 = pair of red-black half-sweeps
 *              in one pass, 5 = prolongation fused into a smoothing step,
 *              6 = last FP32 smoothing step of an iterative-refinement
 *              cycle, with the update of u fused in, 7 = residual and
 *              restriction in one pass, 8 = smoothing step from x = 0
 *              (the iterate is not read)
 * ------------------------------------------------------------------- */
mg_status mg_profile_enable(mg_ctx* ctx, int kernel_id, int enable);
mg_status mg_profile_read(mg_ctx* ctx, long* launches, double* total_ms);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of independent solves on one GPU.
 *
 * A server owns a scheduler thread and a HIP stream.  Requests (any
 * matrix-free options; right-hand side and optional coefficient given in
 * host memory) queue in arrival order and are admitted while fewer than
 * max_slots are in flight and their footprint (mg_footprint_bytes plus
 * their b and u vectors) fits the remaining HBM budget; a context of the
 * same shape and precision left by a finished Poisson request is reused.
 * In flight, every request advances one kernel launch of its V-cycle per
 * scheduler step, and the steps of all requests with the same kernel,
 * level shape and precision are fused into one batched launch.  Each
 * request's result is bitwise the same whether it runs alone or fused.
 * ------------------------------------------------------------------- */
typedef struct mg_server mg_server;

typedef struct {
  uint64_t submitted, admitted, completed, failed;
  uint64_t launches;          /* batched launches issued */
  uint64_t fused_ops;         /* per-request ops carried by those launches */
  uint64_t steps;             /* scheduler steps with work */
  double busy_s;              /* wall time with requests in flight */
  size_t hbm_in_use, hbm_peak;
  int in_flight, queued;
} mg_server_stats;

/* Start a server on the current device.
 *   hbm_budget  device bytes the in-flight requests may hold (> 0).
 *   max_slots   requests in flight at most, 1..1024. */
mg_status mg_server_create(size_t hbm_budget, int max_slots, mg_server** out);

/* Queue one solve.  o: matrix-free options (op = MG_OP_STENCIL);
 *   b_host     host, (n+1)^dim doubles, copied before the call returns;
 *   kappa_host host, n^dim cell coefficients, copied, or NULL (Poisson);
 *   u_host     host, (n+1)^dim doubles, written before the request is
 *              reported done; must stay valid until then;
 *   tol        > 0;  id: out, request id (increasing from 1).
 * MG_E_ARG for invalid options, MG_E_NOMEM if the request can never fit the
 * budget, MG_E_STATE after the server stopped. */
mg_status mg_server_submit(mg_server* srv, const mg_options* o, const double* b_host,
                           const double* kappa_host, double* u_host, double tol,
                           uint64_t* id);

/* Collect up to `max` finished requests (non-blocking): their ids, cycle
 * counts, statuses and, if hist is not NULL, final relative residuals, and
 * (if t_us is not NULL) submit -> done latencies in microseconds.  Returns
 * the number in *n_done. */
mg_status mg_server_poll(mg_server* srv, uint64_t* ids, int* iters, int* status,
                         double* final_rel_residual, double* latency_us, int max,
                         int* n_done);

/* Block until no request is queued or in flight (or timeout_s elapsed:
 * MG_E_STATE). */
mg_status mg_server_drain(mg_server* srv, double timeout_s);

mg_status mg_server_get_stats(mg_server* srv, mg_server_stats* out);

/* Stop the scheduler (finishing in-flight work) and free everything. */
void mg_server_destroy(mg_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
