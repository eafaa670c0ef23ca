// Serving scheduler: continuous batching of independent multigrid solves on
// one GPU (the serving part of the C ABI in mg.h).
//
// Requests queue in arrival order and are admitted while slots and HBM
// budget allow.  Every admitted request holds a context (its hierarchy and
// vectors stay resident until it finishes; Poisson contexts are pooled by
// shape) and the recorded kernel launches of its prologue and of one
// iteration.  Requests are spread over a few streams (lanes), so that the
// small kernels of different lanes can run side by side.  Each scheduler
// step takes, lane by lane, the next launch of every request that is not
// waiting for a norm read-back, groups launches with the same kernel, level
// shape and precision, and issues each group as one batched launch on the
// lane's stream (a lane's lone runnable request queues the rest of its
// iteration at once).  A new request goes to the lane that runs most
// requests of its shape, and a request about to start an iteration while
// another of its shape in its lane is inside one waits (at most 1 ms) for
// that one, so that their iterations proceed as batched launches.  A request that finishes an iteration (or its
// prologue) copies its norms to pinned host memory behind an event and
// waits for that event alone; the other requests keep the GPU busy
// meanwhile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mg_ctx.h"

namespace mg {
mg_status fail(mg_status st, const char* fmt, ...);
}

using namespace mg;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

long ipow_l(long b, int e) {
  long r = 1;
  while (e--) r *= b;
  return r;
}

struct Slot {  // a context plus device b and u of its finest level
  mg_ctx* ctx = nullptr;
  double* b = nullptr;
  double* u = nullptr;
  double* host = nullptr;  // pinned staging of b in and u out
  size_t bytes = 0;
  mg_options o{};
  bool poisson = true;
};

struct Request {
  uint64_t id = 0;
  mg_options o{};
  std::vector<double> b, kappa;
  double* u_host = nullptr;
  double tol = 0;
  double t_submit = 0;
  size_t bytes = 0;
  // in flight
  Slot slot;
  std::vector<OpRec> pro, it;
  int phase = 0;  // 0 prologue, 1 iterations
  size_t pc = 0;
  int k = 0;
  double nb = 0;
  double rho = 1.0;
  bool waiting = false;
  int lane = 0;  // the stream its launches and read-backs go to
  hipEvent_t ev = nullptr;
  double* pin = nullptr;  // 2 pinned doubles: ||r||^2, ||b||^2
  // b: host copy to the pinned staging (copy thread), then one DMA; u: DMA
  // to the staging, then host copy to u_host (copy thread)
  enum { STAGE_IN, RUN, COPY_OUT, HOST_OUT } stage = STAGE_IN;
  std::atomic<bool> host_done{false};
  int final_status = 0;
};

struct CopyJob {
  void* dst;
  const void* src;
  size_t bytes;
  std::atomic<bool>* done;
};

struct Done {
  uint64_t id;
  int iters;
  int status;
  double rho;
  double latency_us;
};

}  // namespace

struct mg_server {
  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, cv_idle;
  bool stop = false;
  uint64_t next_id = 1;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<Done> done;
  mg_server_stats st{};
  // scheduler-thread state
  std::list<std::unique_ptr<Request>> active;
  std::vector<Slot> pool;  // idle Poisson contexts
  size_t in_use = 0;       // bytes of active requests and pooled contexts
  std::vector<double*> pinned_free;
  double busy_since = -1;
  // Requests are spread over kLanes streams; launches are batched within a
  // lane, and the lanes' small kernels can run side by side on the GPU.
  // `stream` serves admissions and result copies.
  static constexpr int kLanes = 4;
  hipStream_t lanes[kLanes] = {};
  static constexpr int kStepsAhead = 8;
  // how many more active requests than the least loaded lane a lane may
  // hold and still be chosen for a request of a shape it runs
  static constexpr int kLaneSlack = 4;
  hipEvent_t step_ev[kLanes][kStepsAhead] = {};
  // per shape in a lane: a request of that shape, the smallest position
  // of those inside an iteration (scheduler scratch)
  std::vector<std::pair<const Request*, size_t>> lag;
  int step_head[kLanes] = {};
  // host copies between pageable request memory and the pinned staging run
  // on their own threads, so the scheduler keeps launching meanwhile
  static constexpr int kCopyThreads = 2;
  std::thread copiers[kCopyThreads];
  std::mutex copy_mu;
  std::condition_variable copy_cv;
  std::deque<CopyJob> copy_jobs;
  bool copy_stop = false;
};

namespace {

size_t request_bytes(const mg_options& o) {
  const size_t nodes = (size_t)ipow_l(o.n + 1L, o.dim);
  return mg_footprint_bytes(&o) + 2 * nodes * sizeof(double);
}

bool same_shape(const mg_options& a, const mg_options& b) {
  return a.dim == b.dim && a.n == b.n && a.levels == b.levels && a.op == b.op &&
         a.smoother == b.smoother && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post &&
         a.omega == b.omega && a.precision == b.precision && a.flags == b.flags;
}

void free_slot(Slot& s) {
  if (s.ctx) mg_destroy(s.ctx);
  if (s.b) hipFree(s.b);
  if (s.u) hipFree(s.u);
  if (s.host) hipHostFree(s.host);
  s = Slot{};
}

void copier(mg_server* S) {
  for (;;) {
    CopyJob j;
    {
      std::unique_lock<std::mutex> lk(S->copy_mu);
      S->copy_cv.wait(lk, [&] { return S->copy_stop || !S->copy_jobs.empty(); });
      if (S->copy_jobs.empty()) return;  // stopping
      j = S->copy_jobs.front();
      S->copy_jobs.pop_front();
    }
    std::memcpy(j.dst, j.src, j.bytes);
    j.done->store(true, std::memory_order_release);
    S->cv.notify_all();  // wake the scheduler
  }
}

void post_copy(mg_server* S, void* dst, const void* src, size_t bytes, std::atomic<bool>* done) {
  done->store(false, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(S->copy_mu);
    S->copy_jobs.push_back(CopyJob{dst, src, bytes, done});
  }
  S->copy_cv.notify_one();
}

// Get a context for r: a pooled one of the same shape or a new one.
mg_status acquire_slot(mg_server* S, Request& r) {
  if (r.kappa.empty()) {
    for (size_t q = 0; q < S->pool.size(); ++q) {
      if (same_shape(S->pool[q].o, r.o)) {
        r.slot = S->pool[q];
        S->pool.erase(S->pool.begin() + q);
        return MG_OK;
      }
    }
  }
  Slot s;
  s.o = r.o;
  s.poisson = r.kappa.empty();
  s.bytes = r.bytes;
  const size_t nodes = (size_t)ipow_l(r.o.n + 1L, r.o.dim);
  if (hipMalloc(&s.b, nodes * sizeof(double)) != hipSuccess ||
      hipMalloc(&s.u, nodes * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&s.host, nodes * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    free_slot(s);
    return fail(MG_E_NOMEM, "device allocation for a request failed");
  }
  double* kdev = nullptr;
  if (!s.poisson) {
    if (hipMalloc(&kdev, r.kappa.size() * sizeof(double)) != hipSuccess ||
        hipMemcpyAsync(kdev, r.kappa.data(), r.kappa.size() * sizeof(double),
                       hipMemcpyHostToDevice, S->stream) != hipSuccess) {
      (void)hipGetLastError();
      if (kdev) hipFree(kdev);
      free_slot(s);
      return fail(MG_E_NOMEM, "device allocation for a coefficient failed");
    }
  }
  mg_status st = mg_setup(&r.o, kdev, S->stream, &s.ctx);
  if (kdev) hipFree(kdev);
  if (st != MG_OK) {
    free_slot(s);
    return st;
  }
  r.slot = s;
  return MG_OK;
}

void release_slot(mg_server* S, Request& r) {
  if (r.slot.poisson && r.slot.ctx) {
    S->pool.push_back(r.slot);  // its bytes stay counted in in_use
  } else {
    S->in_use -= r.slot.bytes;
    free_slot(r.slot);
  }
  r.slot = Slot{};
}

// Make room for `need` bytes by freeing pooled contexts (oldest first).
bool make_room(mg_server* S, size_t need) {
  while (S->in_use + need > S->budget && !S->pool.empty()) {
    S->in_use -= S->pool.front().bytes;
    free_slot(S->pool.front());
    S->pool.erase(S->pool.begin());
  }
  return S->in_use + need <= S->budget;
}

// Report r done (its u, if any, is already in u_host) and free what it holds.
void finish(mg_server* S, Request& r, int status) {
  const double t = now_s();
  if (r.ev) hipEventDestroy(r.ev);
  r.ev = nullptr;
  if (r.pin) S->pinned_free.push_back(r.pin);
  r.pin = nullptr;
  release_slot(S, r);
  std::lock_guard<std::mutex> lk(S->mu);
  S->st.hbm_in_use = S->in_use;
  S->done.push_back(Done{r.id, r.k, status, r.rho, (t - r.t_submit) * 1e6});
  if (status == MG_OK) ++S->st.completed; else ++S->st.failed;
}

// Whether two requests run the same launches (equal kernels, level shapes
// and precision), so that their launches can be batched.
bool same_ops(const Request& a, const Request& b) {
  return same_shape(a.o, b.o) && a.slot.poisson == b.slot.poisson;
}

// The lane for a new request: among the lanes whose load (active
// requests) is within kLaneSlack of the least loaded one, the one running
// the most requests of its shape (their launches batch with its own), the
// less loaded on a tie.  The slack keeps one shape from piling up on one
// stream while the others idle.
int pick_lane(mg_server* S, const Request& r) {
  int load[mg_server::kLanes] = {}, same[mg_server::kLanes] = {};
  for (auto& a : S->active) {
    ++load[a->lane];
    if (same_ops(*a, r)) ++same[a->lane];
  }
  const int lo = *std::min_element(load, load + mg_server::kLanes);
  int best = -1;
  for (int q = 0; q < mg_server::kLanes; ++q) {
    if (load[q] > lo + mg_server::kLaneSlack) continue;
    if (best < 0 || same[q] > same[best] || (same[q] == same[best] && load[q] < load[best]))
      best = q;
  }
  return best;
}

// Admit queued requests in arrival order while slots and budget allow.
void admit(mg_server* S) {
  for (;;) {
    std::unique_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->queue.empty() || (int)S->active.size() >= S->max_slots) return;
      Request& head = *S->queue.front();
      bool pooled = false;
      if (head.kappa.empty())
        for (auto& p : S->pool) pooled |= same_shape(p.o, head.o);
      if (!pooled && !make_room(S, head.bytes)) return;  // head-of-line waits for memory
      r = std::move(S->queue.front());
      S->queue.pop_front();
      if (!pooled) S->in_use += r->bytes;
      S->st.hbm_in_use = S->in_use;
      S->st.hbm_peak = std::max(S->st.hbm_peak, S->in_use);
    }
    bool pooled = false;
    if (r->kappa.empty())
      for (auto& p : S->pool) pooled |= same_shape(p.o, r->o);
    mg_status st = acquire_slot(S, *r);
    if (st != MG_OK) {
      if (!pooled) S->in_use -= r->bytes;
      r->k = 0;
      finish(S, *r, st);
      continue;
    }
    std::vector<double>().swap(r->kappa);
    record_prologue(r->slot.ctx, r->slot.u, r->slot.b, r->pro);
    record_iteration(r->slot.ctx, r->slot.u, r->slot.b, r->it);
    if (!S->pinned_free.empty()) {
      r->pin = S->pinned_free.back();
      S->pinned_free.pop_back();
    } else if (hipHostMalloc(&r->pin, 2 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      r->pin = nullptr;
      finish(S, *r, MG_E_HIP);
      continue;
    }
    hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    r->lane = pick_lane(S, *r);
    // b goes to the slot's pinned staging on a copy thread, then by DMA
    r->stage = Request::STAGE_IN;
    const size_t nodes = (size_t)ipow_l(r->o.n + 1L, r->o.dim);
    post_copy(S, r->slot.host, r->b.data(), nodes * sizeof(double), &r->host_done);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      ++S->st.admitted;
    }
    S->active.push_back(std::move(r));
  }
}

// A request reached the end of its prologue or of an iteration: evaluate
// the norms it read back.
void after_readback(mg_server* S, std::list<std::unique_ptr<Request>>::iterator itr) {
  Request& r = **itr;
  r.waiting = false;
  r.pc = 0;
  int st = -1;
  if (r.phase == 0) {
    const double nb2 = r.pin[1];
    if (!std::isfinite(nb2)) st = MG_E_NONFINITE;
    else if (nb2 == 0.0) st = MG_OK;  // u = 0 already
    else {
      r.nb = std::sqrt(nb2);
      r.phase = 1;
    }
  } else {
    r.k += 1;
    r.rho = std::sqrt(r.pin[0]) / r.nb;
    if (!std::isfinite(r.rho) || r.rho > 1e3) st = MG_E_DIVERGED;
    else if (r.rho <= r.tol) st = MG_OK;
    else if (r.k >= r.o.max_iter) st = MG_E_MAXIT;
  }
  if (st >= 0) {
    // u to the pinned staging by DMA, then to u_host on a copy thread
    r.final_status = st;
    const size_t nodes = (size_t)ipow_l(r.o.n + 1L, r.o.dim);
    if (r.slot.u && r.u_host) {
      hipStream_t ls = S->lanes[r.lane];
      hipMemcpyAsync(r.slot.host, r.slot.u, nodes * sizeof(double), hipMemcpyDeviceToHost, ls);
      hipEventRecord(r.ev, ls);
      r.stage = Request::COPY_OUT;
    } else {
      finish(S, r, st);
      S->active.erase(itr);
    }
  }
}

// Advance the requests whose copies have landed: staged b goes to the
// device, u staged from the device goes to u_host, a request whose u is in
// u_host is done.
void progress_copies(mg_server* S) {
  for (auto itr = S->active.begin(); itr != S->active.end();) {
    auto nxt = std::next(itr);
    Request& r = **itr;
    const size_t bytes = (size_t)ipow_l(r.o.n + 1L, r.o.dim) * sizeof(double);
    if (r.stage == Request::STAGE_IN && r.host_done.load(std::memory_order_acquire)) {
      // (the request's launches follow on the same stream)
      hipMemcpyAsync(r.slot.b, r.slot.host, bytes, hipMemcpyHostToDevice, S->lanes[r.lane]);
      std::vector<double>().swap(r.b);
      r.stage = Request::RUN;
    } else if (r.stage == Request::COPY_OUT && hipEventQuery(r.ev) == hipSuccess) {
      r.stage = Request::HOST_OUT;
      post_copy(S, r.u_host, r.slot.host, bytes, &r.host_done);
    } else if (r.stage == Request::HOST_OUT && r.host_done.load(std::memory_order_acquire)) {
      finish(S, r, r.final_status);
      S->active.erase(itr);
    }
    itr = nxt;
  }
}

// One scheduler step of one lane: the next launch of each of its runnable
// requests, equal launches batched.
void step_lane(mg_server* S, int lane, std::vector<const OpRec*>& ops,
               std::vector<Request*>& owners, std::vector<std::vector<const OpRec*>>& groups) {
  hipStream_t stream = S->lanes[lane];
  ops.clear();
  owners.clear();
  // Laggard first: among the runnable requests of one shape in this lane
  // inside their iterations, only those at the smallest position advance,
  // so a request that starts an iteration (or fell behind) catches up
  // with the others of its shape, and from then on they run as batched
  // launches.  The requests at the smallest position always advance.
  auto& lag = S->lag;
  lag.clear();
  for (auto& rp : S->active) {
    const Request& r = *rp;
    if (r.stage != Request::RUN || r.waiting || r.lane != lane || r.phase != 1) continue;
    bool found = false;
    for (auto& g : lag)
      if (same_ops(*g.first, r)) {
        g.second = std::min(g.second, r.pc);
        found = true;
        break;
      }
    if (!found) lag.emplace_back(&r, r.pc);
  }
  bool deferred = false;
  for (auto& rp : S->active) {
    Request& r = *rp;
    if (r.stage != Request::RUN || r.waiting || r.lane != lane) continue;
    if (r.phase == 1) {
      bool behind = false;
      for (auto& g : lag)
        if (same_ops(*g.first, r)) {
          behind = r.pc > g.second;
          break;
        }
      if (behind) {
        deferred = true;
        continue;
      }
    }
    const std::vector<OpRec>& list = r.phase == 0 ? r.pro : r.it;
    ops.push_back(&list[r.pc]);
    owners.push_back(&r);
  }
  if (ops.empty()) return;
  if (ops.size() == 1 && !deferred) {
    // a lone runnable request has nothing to be batched with: queue the
    // rest of its list at once rather than one launch per step, which
    // would leave the GPU waiting for the scheduler between its small
    // kernels
    Request* r = owners[0];
    const std::vector<OpRec>& list = r->phase == 0 ? r->pro : r->it;
    hipEvent_t& slot_ev = S->step_ev[lane][S->step_head[lane]];
    if (slot_ev) hipEventSynchronize(slot_ev);
    const size_t n = list.size() - r->pc;
    for (size_t q = r->pc; q < list.size(); ++q) {
      const OpRec* one = &list[q];
      launch_ops(&one, 1, stream);
    }
    if (!slot_ev) hipEventCreateWithFlags(&slot_ev, hipEventDisableTiming);
    hipEventRecord(slot_ev, stream);
    S->step_head[lane] = (S->step_head[lane] + 1) % mg_server::kStepsAhead;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.launches += n;
      S->st.fused_ops += n;
      S->st.steps += 1;
    }
    r->pc = list.size();
    hipMemcpyAsync(r->pin, r->slot.ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                   stream);
    hipEventRecord(r->ev, stream);
    r->waiting = true;
    return;
  }
  // group equal launches (first-come order), at most kMaxBatch per group
  groups.clear();
  for (const OpRec* o : ops) {
    bool placed = false;
    if (batchable(*o)) {
      for (auto& g : groups)
        if ((int)g.size() < kMaxBatch && same_key(*g[0], *o)) {
          g.push_back(o);
          placed = true;
          break;
        }
    }
    if (!placed) groups.push_back({o});
  }
  // at most kStepsAhead steps queued on the GPU, so that a read-back is
  // never stuck behind a long queue
  hipEvent_t& slot_ev = S->step_ev[lane][S->step_head[lane]];
  if (slot_ev) hipEventSynchronize(slot_ev);
  for (auto& g : groups) launch_ops(g.data(), (int)g.size(), stream);
  if (!slot_ev) hipEventCreateWithFlags(&slot_ev, hipEventDisableTiming);
  hipEventRecord(slot_ev, stream);
  S->step_head[lane] = (S->step_head[lane] + 1) % mg_server::kStepsAhead;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.launches += groups.size();
    S->st.fused_ops += ops.size();
    S->st.steps += 1;
  }
  // advance; requests at the end of a list read their norms back
  for (Request* r : owners) {
    const std::vector<OpRec>& list = r->phase == 0 ? r->pro : r->it;
    if (++r->pc < list.size()) continue;
    hipMemcpyAsync(r->pin, r->slot.ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                   stream);
    hipEventRecord(r->ev, stream);
    r->waiting = true;
  }
}

void scheduler(mg_server* S) {
  hipSetDevice(S->device);
  std::vector<const OpRec*> ops;
  std::vector<Request*> owners;
  std::vector<std::vector<const OpRec*>> groups;
  for (;;) {
    admit(S);
    // read-backs that have landed
    for (auto itr = S->active.begin(); itr != S->active.end();) {
      auto nxt = std::next(itr);
      if ((*itr)->stage == Request::RUN && (*itr)->waiting &&
          hipEventQuery((*itr)->ev) == hipSuccess)
        after_readback(S, itr);
      itr = nxt;
    }
    progress_copies(S);
    int runnable = 0;
    bool host_wait = false;
    Request* gpu_wait = nullptr;
    for (auto& rp : S->active) {
      Request& r = *rp;
      runnable += r.stage == Request::RUN && !r.waiting;
      host_wait |= r.stage == Request::STAGE_IN || r.stage == Request::HOST_OUT;
      if (!gpu_wait && ((r.stage == Request::RUN && r.waiting) || r.stage == Request::COPY_OUT))
        gpu_wait = &r;
    }
    if (runnable == 0) {
      if (host_wait) {
        // nothing to launch: a copy thread will wake us (or the timeout)
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
      if (gpu_wait) {
        // nothing to launch: block on the oldest outstanding read-back or copy
        hipEventSynchronize(gpu_wait->ev);
        continue;
      }
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->busy_since >= 0) {
        S->st.busy_s += now_s() - S->busy_since;
        S->busy_since = -1;
      }
      S->st.in_flight = 0;
      S->st.queued = (int)S->queue.size();
      S->cv_idle.notify_all();
      if (S->stop && S->queue.empty()) return;
      S->cv.wait_for(lk, std::chrono::milliseconds(50),
                     [&] { return S->stop || !S->queue.empty(); });
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->busy_since < 0) S->busy_since = now_s();
      S->st.in_flight = (int)S->active.size();
      S->st.queued = (int)S->queue.size();
    }
    for (int lane = 0; lane < mg_server::kLanes; ++lane)
      step_lane(S, lane, ops, owners, groups);
  }
}


}  // namespace

extern "C" {

mg_status mg_server_create(size_t hbm_budget, int max_slots, mg_server** out) {
  if (!out) return fail(MG_E_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget == 0) return fail(MG_E_ARG, "hbm_budget must be > 0");
  if (max_slots < 1 || max_slots > 1024) return fail(MG_E_ARG, "max_slots must be in 1..1024");
  mg_server* S = new mg_server();
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  bool ok = hipGetDevice(&S->device) == hipSuccess &&
            hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
  for (int q = 0; ok && q < mg_server::kLanes; ++q)
    ok = hipStreamCreateWithFlags(&S->lanes[q], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    for (hipStream_t l : S->lanes)
      if (l) hipStreamDestroy(l);
    if (S->stream) hipStreamDestroy(S->stream);
    delete S;
    return fail(MG_E_HIP, "could not create the server streams");
  }
  for (auto& t : S->copiers) t = std::thread(copier, S);
  S->th = std::thread(scheduler, S);
  *out = S;
  return MG_OK;
}

mg_status mg_server_submit(mg_server* S, const mg_options* o, const double* b_host,
                           const double* kappa_host, double* u_host, double tol, uint64_t* id) {
  if (!S || !o || !b_host || !u_host || !id) return fail(MG_E_ARG, "NULL argument");
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be > 0");
  if (o->op != MG_OP_STENCIL) return fail(MG_E_ARG, "serving takes matrix-free requests");
  if (o->flags & MG_FLAG_PCG) return fail(MG_E_ARG, "serving runs the cycle iteration, not CG");
  if (o->flags & MG_FLAG_WARM) return fail(MG_E_ARG, "served solves start from u = 0");
  if (o->sigma != 0.0) return fail(MG_E_ARG, "the server solves sigma = 0 problems only");
  if (o->smoother == MG_SMOOTH_GS) return fail(MG_E_ARG, "the server runs Jacobi or red-black smoothing");
  if (mg_footprint_bytes(o) == 0) return MG_E_ARG;  // message set by mg_footprint_bytes
  auto r = std::make_unique<Request>();
  r->o = *o;
  r->o.flags |= MG_FLAG_NO_GRAPH;
  r->bytes = request_bytes(r->o);
  if (r->bytes > S->budget) return fail(MG_E_NOMEM, "request needs %zu bytes > budget", r->bytes);
  const size_t nodes = (size_t)ipow_l(o->n + 1L, o->dim);
  r->b.assign(b_host, b_host + nodes);
  if (kappa_host) r->kappa.assign(kappa_host, kappa_host + ipow_l(o->n, o->dim));
  r->u_host = u_host;
  r->tol = tol;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(MG_E_STATE, "server stopped");
    r->id = S->next_id++;
    *id = r->id;
    S->queue.push_back(std::move(r));
    ++S->st.submitted;
  }
  S->cv.notify_all();
  return MG_OK;
}

mg_status mg_server_poll(mg_server* S, uint64_t* ids, int* iters, int* status, double* rho,
                         double* latency_us, int max, int* n_done) {
  if (!S || !n_done || max < 0) return fail(MG_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(S->mu);
  const int n = std::min<int>(max, (int)S->done.size());
  for (int q = 0; q < n; ++q) {
    const Done& d = S->done[q];
    if (ids) ids[q] = d.id;
    if (iters) iters[q] = d.iters;
    if (status) status[q] = d.status;
    if (rho) rho[q] = d.rho;
    if (latency_us) latency_us[q] = d.latency_us;
  }
  S->done.erase(S->done.begin(), S->done.begin() + n);
  *n_done = n;
  return MG_OK;
}

mg_status mg_server_drain(mg_server* S, double timeout_s) {
  if (!S) return fail(MG_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  const bool ok = S->cv_idle.wait_for(
      lk, std::chrono::duration<double>(timeout_s),
      [&] { return S->queue.empty() && S->st.in_flight == 0 &&
                   S->st.completed + S->st.failed == S->st.submitted; });
  return ok ? MG_OK : fail(MG_E_STATE, "drain timed out");
}

mg_status mg_server_get_stats(mg_server* S, mg_server_stats* out) {
  if (!S || !out) return fail(MG_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  return MG_OK;
}

void mg_server_destroy(mg_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  {
    std::lock_guard<std::mutex> lk(S->copy_mu);
    S->copy_stop = true;
  }
  S->copy_cv.notify_all();
  for (auto& t : S->copiers)
    if (t.joinable()) t.join();
  for (auto& p : S->pool) free_slot(p);
  for (double* p : S->pinned_free) hipHostFree(p);
  for (auto& lane : S->step_ev)
    for (hipEvent_t e : lane)
      if (e) hipEventDestroy(e);
  for (hipStream_t l : S->lanes)
    if (l) hipStreamDestroy(l);
  if (S->stream) hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
