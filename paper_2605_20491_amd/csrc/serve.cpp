// Serving loop over the solver (not part of the paper): continuous batching of
// requests of different d, n and kind on one GPU.
//
// * Admission by memory: the server allocates one arena of device memory at
//   creation and carves each admitted request's scratch (apply workspace,
//   phase tables, solver vectors) from it with a first-fit free list, so no
//   hipMalloc / hipFree happens while requests run.  A request waits in the
//   queue until its scratch fits.
// * Resident factors: plans are cached by (grid, potential samples, sigma).
// * Concurrency: admitted requests run on a pool of non-blocking streams;
//   each advances one unit at a time (an apply, a refinement sweep, a few PCG
//   iterations, a few split steps; ts_tasks.h), so new requests join between
//   units and their kernels overlap on the device.
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

struct Request {
  uint64_t ticket = 0;
  ts_request r{};
  std::vector<std::vector<double>> f;
  double t_submit = 0, t_admit = 0, t_done = 0;
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
  k.append((const char*)&r.sigma, sizeof(r.sigma));
  for (int i = 0; i < r.d; ++i) k.append((const char*)r.f[i], sizeof(double) * r.n[i]);
  return k;
}

}  // namespace
}  // namespace ts

struct ts_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ts::Request*> pending;  // submitted, waiting for memory
  std::vector<ts::Request*> active;
  std::unordered_map<uint64_t, std::unique_ptr<ts::Request>> all;
  std::map<std::string, ts_plan*> plans;
  ts::Arena arena;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
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
  void finish(ts::Request* q, int status);
};

namespace ts {
namespace {

constexpr int kPinnedSlots = 4096;

// Scratch of a request in each context slot.
void request_needs(const ts_request& r, const ts_plan* p, size_t* b) {
  for (int i = 0; i < kSlots; ++i) b[i] = 0;
  if (r.kind == TS_REQ_INVERSE) {
    for (int i = 0; i < kSlots; ++i) b[i] = need_inverse(p, i);
    if (r.V2 || r.prec != TS_PREC_FP64) b[kSlotSolver] = need_solver(p, 4);
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
    if (r->prec == TS_PREC_FP64 && r->dtype != TS_C128) return TS_ERR_INVALID;
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
  q->st = streams[next_stream];
  next_stream = (next_stream + 1) % (int)streams.size();
  const ts_request& r = q->r;
  int rc = TS_OK;
  if (r.kind == TS_REQ_INVERSE) {
    if (r.V2) {
      if (hipMemsetAsync(r.out, 0, sizeof(double) * q->plan->N, q->st) != hipSuccess) rc = TS_ERR_DEVICE;
      q->task = make_pcg_task(q->plan, (const double*)r.V2, r.sigma, r.sigma, (const double*)r.in, (double*)r.out,
                              r.rtol, r.maxit, r.prec, *q->ctx);
    } else if (r.prec == TS_PREC_FP64) {
      q->task = make_inverse_task(q->plan, r.sigma, r.in, r.out, TS_F64, TS_PREC_FP64, *q->ctx);
    } else {
      q->task = make_refine_task(q->plan, (const double*)r.in, (double*)r.out, r.prec, r.rtol, r.maxit, *q->ctx);
    }
  } else {
    if (r.V2) {
      const int nsteps = std::max(1, (int)std::ceil(std::fabs(r.tau) / r.dt));
      const double dt = r.tau / nsteps;
      const size_t eb = r.dtype == TS_C128 ? 16 : 8;
      if (r.in != r.out &&
          hipMemcpyAsync(r.out, r.in, eb * q->plan->N, hipMemcpyDeviceToDevice, q->st) != hipSuccess)
        rc = TS_ERR_DEVICE;
      q->task = make_split_task(q->plan, r.V2, r.out, dt, nsteps, TS_STRANG_BAB, r.dtype, r.prec, *q->ctx);
    } else {
      q->task = make_exp_task(q->plan, r.tau, r.in, r.out, r.dtype, r.prec, *q->ctx);
    }
  }
  if (rc == TS_OK) rc = q->task->start(q->st);
  if (rc == TS_OK && hipEventCreateWithFlags(&q->ev, hipEventDisableTiming) != hipSuccess) rc = TS_ERR_DEVICE;
  if (rc == TS_OK && hipEventRecord(q->ev, q->st) != hipSuccess) rc = TS_ERR_DEVICE;
  active.push_back(q);
  if (rc != TS_OK) {
    // let queued work (if any) drain before the scratch is reused
    hipStreamSynchronize(q->st);
    finish(q, rc);
  }
  return true;
}

// Called with mu held.
void ts_server::finish(Request* q, int status) {
  q->status = status;
  q->t_done = clock();
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
  for (;;) {
    if (stop && pending.empty() && active.empty()) break;
    bool progressed = false;
    // admission: first fit in arrival order
    for (auto it = pending.begin(); it != pending.end();) {
      Request* q = *it;
      if (try_admit(q)) {
        it = pending.erase(it);
        progressed = true;
      } else {
        ++it;
      }
    }
    // progress: advance every request whose last unit has completed
    std::vector<Request*> snapshot(active);
    for (Request* q : snapshot) {
      if (q->done || !q->ev) continue;
      hipError_t e = hipEventQuery(q->ev);
      if (e == hipErrorNotReady) continue;
      progressed = true;
      if (e != hipSuccess) {
        finish(q, TS_ERR_DEVICE);
        continue;
      }
      bool done = false;
      int rc = q->task->advance(q->st, &done);
      if (rc != TS_OK) {
        hipStreamSynchronize(q->st);
        finish(q, rc);
        continue;
      }
      if (done) {
        q->iters = q->task->iters;
        q->relres = q->task->relres;
        finish(q, q->task->status);
        continue;
      }
      if (hipEventRecord(q->ev, q->st) != hipSuccess) finish(q, TS_ERR_DEVICE);
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

int ts_serve_create(size_t hbm_budget_bytes, int n_streams, int max_active, ts_server** out) {
  if (!out || n_streams < 1 || n_streams > 64 || max_active < 0 || hbm_budget_bytes < kAlign) {
    set_error("bad argument");
    return TS_ERR_INVALID;
  }
  *out = nullptr;
  std::unique_ptr<ts_server> s(new ts_server());
  s->t0 = std::chrono::steady_clock::now();
  hipGetDevice(&s->device);
  if (!s->arena.init(hbm_budget_bytes)) {
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
  // resident factors: build the plan outside the server lock (host work)
  const std::string key = plan_key(q->r);
  ts_plan* plan = nullptr;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) plan = it->second;
  }
  if (!plan) {
    const double* fp[TS_MAX_D];
    for (int k = 0; k < req->d; ++k) fp[k] = q->r.f[k];
    int rc = ts_setup(req->d, req->n, req->L, fp, req->sigma, &plan);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {
      ts_destroy(plan);
      plan = it->second;
    } else {
      s->plans[key] = plan;
    }
  }
  if (req->kind == TS_REQ_INVERSE && !(plan->lam_min + req->sigma > 0.0)) {
    set_error("H1 + sigma is not positive definite");
    return TS_ERR_NOT_SPD;
  }
  q->plan = plan;
  request_needs(q->r, plan, q->slot_bytes);
  q->need = 0;
  for (int i = 0; i < kSlots; ++i) q->need += round_up((int64_t)q->slot_bytes[i], kAlign);
  if (q->need > s->arena.size()) {
    set_error("request scratch (" + std::to_string(q->need) + " bytes) exceeds the server budget");
    return TS_ERR_NOMEM;
  }
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
  for (auto& kv : s->plans) ts_destroy(kv.second);
  if (s->pinned) hipHostFree(s->pinned);
  delete s;
  return TS_OK;
}

}  // extern "C"
