// Serving loop over the solver (not part of the paper): continuous batching of
// requests of different d, n and kind on one GPU.
//
// * Memory: the budget is split into a request arena and a plan reserve (by
//   default a quarter of the budget).  The arena is allocated once, at creation, and
//   each admitted request's scratch (apply workspace, phase tables, solver
//   vectors) is carved from it with a first-fit free list, so no hipMalloc /
//   hipFree happens while requests run; a request waits in the queue until
//   its scratch fits.
// * Resident factors: plans are cached by (grid, potential samples) -- the
//   shift is a per-request argument of the tasks -- and the cache is held
//   within the plan reserve: plans that no queued or running request uses are
//   evicted least recently used first, and a submit whose plan cannot fit
//   even then returns TS_ERR_BUSY.
// * Scheduling: requests advance one unit at a time (an apply, a refinement
//   sweep, a few PCG iterations, a few split steps; ts_tasks.h) on a pool of
//   non-blocking streams.  Each free stream takes the next unit of the most
//   urgent admitted request, urgency being the submit time plus the request's
//   estimated GPU time (earliest expected completion first): a short request
//   that arrives behind long ones overtakes them at their next unit boundary,
//   while a long request is not starved by a stream of short ones, whose
//   urgency lies later than its own once they arrive late enough.  At most one
//   request per stream is in flight, so the kernels of a few requests overlap
//   on the device instead of every admitted request sharing it.
// * A request computes exactly what the plain entry points compute: the same
//   task code, deterministic kernels, no dependence on the schedule.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"
#include "ts_small.h"
#include "ts_tasks.h"

namespace ts {
namespace {

constexpr size_t kAlign = 256;

// First-fit allocator over one device block.
class Arena {
 public:
  bool init(size_t bytes) {
    size_ = round_up((int64_t)bytes, kAlign);
    if (hipMalloc(&base_, size_) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = size_;
    return true;
  }
  ~Arena() {
    if (base_) hipFree(base_);
  }
  size_t size() const { return size_; }
  void* alloc(size_t bytes) {
    bytes = round_up((int64_t)bytes, kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p, size_t bytes) {
    bytes = round_up((int64_t)bytes, kAlign);
    size_t off = (char*)p - base_;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

struct CachedPlan {
  ts_plan* plan = nullptr;
  size_t bytes = 0;
  int refs = 0;          // queued or running requests that use it
  uint64_t last_use = 0;
};

enum class RState : int { Waiting = 0, InFlight = 1, Ready = 2 };

struct Request {
  uint64_t ticket = 0;
  ts_request r{};
  std::vector<std::vector<double>> f;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double est = 0.0;       // estimated GPU seconds
  double urgency = 0.0;   // t_submit + est
  RState state = RState::Waiting;
  bool started = false;
  bool holds_stream = false;  // q->st is taken from the pool
  std::string key;
  ts_plan* plan = nullptr;
  size_t slot_bytes[kSlots] = {};
  size_t need = 0;
  void* block = nullptr;
  std::unique_ptr<ExecCtx> ctx;
  int host_slot = -1;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  std::unique_ptr<Task> task;
  int status = TS_OK;
  int iters = 0;
  double relres = 0.0;
  bool done = false;
};

std::string plan_key(const ts_request& r) {
  std::string k((const char*)&r.d, sizeof(r.d));
  k.append((const char*)r.n, sizeof(int64_t) * r.d);
  k.append((const char*)&r.L, sizeof(r.L));
  for (int i = 0; i < r.d; ++i) k.append((const char*)r.f[i], sizeof(double) * r.n[i]);
  return k;
}

// Rough GPU seconds of a request, for ordering only: per-point costs of an
// apply on this device (FP64 ~1.1e-10 s, FP32 about half, BF16 about a
// quarter; complex data twice the real cost), ~12 iterations for PCG and
// ~6 sweeps for refinement, plus a fixed launch cost per unit.
double estimate_seconds(const ts_request& r, int64_t N) {
  const double pt = r.prec == TS_PREC_FP64 ? 1.1e-10 : (r.prec == TS_PREC_FP32 ? 6e-11 : 3e-11);
  const double vec = 3e-11;  // FP64 stencil and vector updates per point and iteration
  double t;
  if (r.kind == TS_REQ_INVERSE) {
    if (r.V2) t = 12.0 * (pt + vec) * N;
    else if (r.prec == TS_PREC_FP64) t = pt * N;
    else t = 6.0 * (pt + vec) * N;
  } else {
    const double c = r.dtype == TS_C128 ? 2.0 : 1.0;
    const int steps = r.V2 ? std::max(1, (int)std::ceil(std::fabs(r.tau) / r.dt)) : 1;
    t = steps * c * pt * N;
  }
  return t + 1e-4;
}

}  // namespace
}  // namespace ts

struct ts_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ts::Request*> pending;  // submitted, waiting for memory
  std::vector<ts::Request*> active;
  std::unordered_map<uint64_t, std::unique_ptr<ts::Request>> all;
  std::map<std::string, ts::CachedPlan> plans;
  size_t plan_reserve = 0, plan_bytes = 0;
  uint64_t use_clock = 0;
  ts::Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<hipStream_t> free_streams;
  int max_active = 0;
  int device = 0;
  char* pinned = nullptr;
  std::vector<int> free_pinned;
  std::thread thr;
  bool stop = false;
  uint64_t next_ticket = 1;
  int outstanding = 0;
  std::chrono::steady_clock::time_point t0;
  double clock() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop();
  bool try_admit(ts::Request* q);
  int dispatch(ts::Request* q, hipStream_t st);
  void finish(ts::Request* q, int status);
  void release_plan(const std::string& key);
  bool evict_for(size_t bytes);
};

namespace ts {
namespace {

constexpr int kPinnedSlots = 4096;

// Scratch of a request in each context slot.
void request_needs(const ts_request& r, const ts_plan* p, size_t* b) {
  for (int i = 0; i < kSlots; ++i) b[i] = 0;
  if (r.kind == TS_REQ_INVERSE) {
    for (int i = 0; i < kSlots; ++i) b[i] = need_inverse(p, i);
    if (r.V2 || r.prec != TS_PREC_FP64) b[kSlotSolver] = need_solver(p, 5);  // PCG: r, z, p (x2), q
  } else {
    for (int i = 0; i < kSlots; ++i) b[i] = need_exp(p, i);
  }
}

int validate(const ts_request* r) {
  if (!r) return TS_ERR_INVALID;
  if (r->kind != TS_REQ_INVERSE && r->kind != TS_REQ_EXP) return TS_ERR_INVALID;
  if (r->d < 1 || r->d > TS_MAX_D || !r->in || !r->out) return TS_ERR_INVALID;
  for (int k = 0; k < r->d; ++k)
    if (!r->f[k] || r->n[k] < 1) return TS_ERR_INVALID;
  if (r->prec < TS_PREC_FP64 || r->prec > TS_PREC_BF16) return TS_ERR_INVALID;
  if (r->kind == TS_REQ_INVERSE) {
    if (r->dtype != TS_F64) return TS_ERR_INVALID;
    if ((r->V2 || r->prec != TS_PREC_FP64) && (!(r->rtol > 0) || r->maxit < 1)) return TS_ERR_INVALID;
  } else {
    if (r->dtype != TS_C128 && r->dtype != TS_C64) return TS_ERR_INVALID;
    if (r->V2 && !(r->dt > 0)) return TS_ERR_INVALID;
  }
  return TS_OK;
}

}  // namespace
}  // namespace ts

using namespace ts;

bool ts_server::try_admit(Request* q) {
  if (max_active > 0 && (int)active.size() >= max_active) return false;
  if (free_pinned.empty()) return false;
  void* block = arena.alloc(q->need);
  if (!block) return false;
  q->block = block;
  q->t_admit = clock();
  q->ctx.reset(new ExecCtx());
  q->ctx->growable = false;
  size_t off = 0;
  for (int i = 0; i < kSlots; ++i) {
    q->ctx->buf[i] = q->slot_bytes[i] ? (char*)block + off : nullptr;
    q->ctx->bytes[i] = q->slot_bytes[i];
    off += round_up((int64_t)q->slot_bytes[i], kAlign);
  }
  q->host_slot = free_pinned.back();
  free_pinned.pop_back();
  q->ctx->host = pinned + 256 * (size_t)q->host_slot;
  const ts_request& r = q->r;
  if (r.kind == TS_REQ_INVERSE) {
    if (r.V2) {
      q->task = make_pcg_task(q->plan, (const double*)r.V2, r.sigma, r.sigma, (const double*)r.in, (double*)r.out,
                              r.rtol, r.maxit, r.prec, *q->ctx);
    } else if (r.prec == TS_PREC_FP64) {
      q->task = make_inverse_task(q->plan, r.sigma, r.in, r.out, TS_F64, TS_PREC_FP64, *q->ctx);
    } else {
      q->task = make_refine_task(q->plan, r.sigma, (const double*)r.in, (double*)r.out, r.prec, r.rtol, r.maxit,
                                 *q->ctx);
    }
  } else {
    if (r.V2) {
      const int nsteps = std::max(1, (int)std::ceil(std::fabs(r.tau) / r.dt));
      q->task = make_split_task(q->plan, r.V2, r.out, r.tau / nsteps, nsteps, TS_STRANG_BAB, r.dtype, r.prec,
                                *q->ctx);
    } else {
      q->task = make_exp_task(q->plan, r.tau, r.in, r.out, r.dtype, r.prec, *q->ctx);
    }
  }
  q->state = RState::Ready;
  active.push_back(q);
  return true;
}

// Enqueue the request's next unit (its first: the set-up copies and start())
// on stream st and record its event.  Returns TS_OK if a unit is in flight,
// else the request has been finished (done or failed) and st is free again.
int ts_server::dispatch(Request* q, hipStream_t st) {
  const ts_request& r = q->r;
  int rc = TS_OK;
  bool done = false;
  q->st = st;
  if (!q->started) {
    q->started = true;
    if (r.kind == TS_REQ_INVERSE && r.V2) {
      if (hipMemsetAsync(r.out, 0, sizeof(double) * q->plan->N, st) != hipSuccess) rc = TS_ERR_DEVICE;
    } else if (r.kind == TS_REQ_EXP && r.V2 && r.in != r.out) {
      const size_t eb = r.dtype == TS_C128 ? 16 : 8;
      if (hipMemcpyAsync(r.out, r.in, eb * q->plan->N, hipMemcpyDeviceToDevice, st) != hipSuccess) rc = TS_ERR_DEVICE;
    }
    if (rc == TS_OK) rc = q->task->start(st);
  } else {
    rc = q->task->advance(st, &done);
  }
  if (rc == TS_OK && done) {
    q->iters = q->task->iters;
    q->relres = q->task->relres;
    finish(q, q->task->status);
    return q->status == TS_OK ? 1 : q->status;
  }
  if (rc == TS_OK && !q->ev && hipEventCreateWithFlags(&q->ev, hipEventDisableTiming) != hipSuccess) rc = TS_ERR_DEVICE;
  if (rc == TS_OK && hipEventRecord(q->ev, st) != hipSuccess) rc = TS_ERR_DEVICE;
  if (rc != TS_OK) {
    hipStreamSynchronize(st);  // let queued work drain before the scratch is reused
    finish(q, rc);
    return rc;
  }
  q->state = RState::InFlight;
  return TS_OK;
}

// Plan cache: drop one reference; keep the plan resident for later requests.
void ts_server::release_plan(const std::string& key) {
  auto it = plans.find(key);
  if (it != plans.end() && it->second.refs > 0) --it->second.refs;
}

// Evict unreferenced plans, least recently used first, until `bytes` more fit
// in the plan reserve.  Returns false if they cannot.
bool ts_server::evict_for(size_t bytes) {
  while (plan_bytes + bytes > plan_reserve) {
    auto victim = plans.end();
    for (auto it = plans.begin(); it != plans.end(); ++it)
      if (it->second.refs == 0 && (victim == plans.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == plans.end()) return false;
    plan_bytes -= victim->second.bytes;
    ts_destroy(victim->second.plan);
    plans.erase(victim);
  }
  return true;
}

// Called with mu held.
void ts_server::finish(Request* q, int status) {
  q->status = status;
  q->t_done = clock();
  if (q->holds_stream) free_streams.push_back(q->st);
  q->holds_stream = false;
  q->state = RState::Ready;
  release_plan(q->key);
  if (q->ev) {
    hipEventDestroy(q->ev);
    q->ev = nullptr;
  }
  q->task.reset();
  q->ctx.reset();
  if (q->block) arena.release(q->block, q->need);
  q->block = nullptr;
  if (q->host_slot >= 0) free_pinned.push_back(q->host_slot);
  q->host_slot = -1;
  q->done = true;
  active.erase(std::remove(active.begin(), active.end(), q), active.end());
  --outstanding;
  cv_done.notify_all();
}

void ts_server::loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  // one request at a time (max_active == 1) is a plain FIFO queue: arrival order
  const bool fifo = max_active == 1;
  auto more_urgent = [fifo](const Request* a, const Request* b) {
    if (fifo) return a->ticket < b->ticket;
    return a->urgency < b->urgency || (a->urgency == b->urgency && a->ticket < b->ticket);
  };
  for (;;) {
    if (stop && pending.empty() && active.empty()) break;
    bool progressed = false;
    // admission: most urgent first, first fit in the arena
    std::stable_sort(pending.begin(), pending.end(), more_urgent);
    for (auto it = pending.begin(); it != pending.end();) {
      if (try_admit(*it)) {
        it = pending.erase(it);
        progressed = true;
      } else {
        ++it;
      }
    }
    // completions: a request whose unit has finished gives its stream back
    for (Request* q : active) {
      if (q->state != RState::InFlight) continue;
      const hipError_t e = hipEventQuery(q->ev);
      if (e == hipErrorNotReady) continue;
      progressed = true;
      q->state = RState::Ready;
      free_streams.push_back(q->st);
      q->holds_stream = false;
      if (e != hipSuccess) q->status = TS_ERR_DEVICE;
    }
    for (Request* q : std::vector<Request*>(active))
      if (q->state == RState::Ready && q->status != TS_OK) finish(q, q->status);
    // dispatch: each free stream takes the next unit of the most urgent ready request
    if (!free_streams.empty()) {
      std::vector<Request*> ready;
      for (Request* q : active)
        if (q->state == RState::Ready) ready.push_back(q);
      std::sort(ready.begin(), ready.end(), more_urgent);
      for (Request* q : ready) {
        if (free_streams.empty()) break;
        hipStream_t st = free_streams.back();
        free_streams.pop_back();
        q->holds_stream = true;
        dispatch(q, st);
        progressed = true;
      }
    }
    if (!progressed) {
      cv_work.wait_for(lk, std::chrono::microseconds(50));
    } else {
      // let submit / poll in
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

extern "C" {

int ts_serve_create(size_t hbm_budget_bytes, size_t plan_reserve_bytes, int n_streams, int max_active,
                    ts_server** out) {
  if (plan_reserve_bytes == 0) plan_reserve_bytes = hbm_budget_bytes / 4;
  if (!out || n_streams < 1 || n_streams > 64 || max_active < 0 || plan_reserve_bytes >= hbm_budget_bytes ||
      hbm_budget_bytes - plan_reserve_bytes < kAlign) {
    set_error("bad argument");
    return TS_ERR_INVALID;
  }
  *out = nullptr;
  std::unique_ptr<ts_server> s(new ts_server());
  s->t0 = std::chrono::steady_clock::now();
  hipGetDevice(&s->device);
  s->plan_reserve = plan_reserve_bytes;
  if (!s->arena.init(hbm_budget_bytes - s->plan_reserve)) {
    set_error("arena allocation failed");
    return TS_ERR_NOMEM;
  }
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      set_error("stream creation failed");
      return TS_ERR_DEVICE;
    }
    s->streams.push_back(st);
    s->free_streams.push_back(st);
  }
  if (hipHostMalloc((void**)&s->pinned, 256 * (size_t)kPinnedSlots, hipHostMallocDefault) != hipSuccess) {
    set_error("pinned allocation failed");
    return TS_ERR_NOMEM;
  }
  for (int i = kPinnedSlots - 1; i >= 0; --i) s->free_pinned.push_back(i);
  s->max_active = max_active;
  ts_server* raw = s.get();
  s->thr = std::thread([raw] { raw->loop(); });
  *out = s.release();
  return TS_OK;
}

int ts_serve_submit(ts_server* s, const ts_request* req, uint64_t* ticket) {
  if (!s || !ticket) { set_error("null argument"); return TS_ERR_INVALID; }
  if (validate(req) != TS_OK) { set_error("malformed request"); return TS_ERR_INVALID; }
  std::unique_ptr<Request> q(new Request());
  q->r = *req;
  q->t_submit = s->clock();
  for (int k = 0; k < req->d; ++k) {
    q->f.emplace_back(req->f[k], req->f[k] + req->n[k]);
    q->r.f[k] = q->f.back().data();
  }
  // resident factors: build a missing plan outside the server lock (host work),
  // then hold it in the cache within the plan reserve
  q->key = plan_key(q->r);
  ts_plan* plan = nullptr;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->plans.find(q->key);
    if (it != s->plans.end()) {
      plan = it->second.plan;
      it->second.refs += 1;
      it->second.last_use = ++s->use_clock;
    }
  }
  if (!plan) {
    const double* fp[TS_MAX_D];
    for (int k = 0; k < req->d; ++k) fp[k] = q->r.f[k];
    int rc = ts_setup(req->d, req->n, req->L, fp, req->sigma, &plan);
    if (rc) return rc;
    const size_t pb = plan_device_bytes(plan);
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->plans.find(q->key);
    if (it != s->plans.end()) {  // built by another thread meanwhile
      ts_destroy(plan);
      plan = it->second.plan;
      it->second.refs += 1;
      it->second.last_use = ++s->use_clock;
    } else {
      if (pb > s->plan_reserve) {
        ts_destroy(plan);
        set_error("the request's factors (" + std::to_string(pb) + " bytes) exceed the plan reserve (" +
                  std::to_string(s->plan_reserve) + " bytes)");
        return TS_ERR_NOMEM;
      }
      if (!s->evict_for(pb)) {
        ts_destroy(plan);
        set_error("plan reserve held by running requests; resubmit later");
        return TS_ERR_BUSY;
      }
      CachedPlan cp;
      cp.plan = plan;
      cp.bytes = pb;
      cp.refs = 1;
      cp.last_use = ++s->use_clock;
      s->plans[q->key] = cp;
      s->plan_bytes += pb;
    }
  }
  auto unref = [&]() {
    std::lock_guard<std::mutex> g(s->mu);
    s->release_plan(q->key);
  };
  if (req->kind == TS_REQ_INVERSE && !(plan->lam_min + req->sigma > 0.0)) {
    unref();
    set_error("H1 + sigma is not positive definite");
    return TS_ERR_NOT_SPD;
  }
  q->plan = plan;
  request_needs(q->r, plan, q->slot_bytes);
  q->need = 0;
  for (int i = 0; i < kSlots; ++i) q->need += round_up((int64_t)q->slot_bytes[i], kAlign);
  if (q->need > s->arena.size()) {
    unref();
    set_error("request scratch (" + std::to_string(q->need) + " bytes) exceeds the server's arena (" +
              std::to_string(s->arena.size()) + " bytes)");
    return TS_ERR_NOMEM;
  }
  q->est = estimate_seconds(q->r, plan->N);
  q->urgency = q->t_submit + q->est;
  std::lock_guard<std::mutex> g(s->mu);
  q->ticket = s->next_ticket++;
  *ticket = q->ticket;
  s->pending.push_back(q.get());
  s->all[q->ticket] = std::move(q);
  ++s->outstanding;
  s->cv_work.notify_all();
  return TS_OK;
}

int ts_serve_poll(ts_server* s, uint64_t ticket, int* done, ts_result* res) {
  if (!s || !done) { set_error("null argument"); return TS_ERR_INVALID; }
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) { set_error("unknown ticket"); return TS_ERR_INVALID; }
  Request* q = it->second.get();
  *done = q->done ? 1 : 0;
  if (q->done && res) {
    res->status = q->status;
    res->iters = q->iters;
    res->relres = q->relres;
    res->t_submit = q->t_submit;
    res->t_admit = q->t_admit;
    res->t_done = q->t_done;
    res->tag = q->r.tag;
  }
  return TS_OK;
}

int ts_serve_drain(ts_server* s) {
  if (!s) { set_error("null argument"); return TS_ERR_INVALID; }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->outstanding == 0; });
  return TS_OK;
}

double ts_serve_clock(ts_server* s) { return s ? s->clock() : 0.0; }

int ts_serve_destroy(ts_server* s) {
  if (!s) return TS_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->thr.joinable()) s->thr.join();
  for (auto st : s->streams) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  for (auto& kv : s->plans) ts_destroy(kv.second.plan);
  if (s->pinned) hipHostFree(s->pinned);
  delete s;
  return TS_OK;
}

}  // extern "C"
