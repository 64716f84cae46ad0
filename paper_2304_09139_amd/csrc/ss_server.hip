// ss_server.hip -- continuous batching of quench requests (ss_submit / ss_poll).
//
// A worker thread owns one stream and keeps one batched minimiser step in
// flight for every configuration it is running (the batched launches of
// ss_batch.hip).  Requests wait in submission order; at every step boundary the
// worker walks the queue and admits every request for which there are a free
// slot and arena space (first fit over the caller's device arena), so a large
// request that does not fit yet does not hold back smaller ones behind it --
// until it has been overtaken kMaxOvertake times, after which nothing else is
// admitted before it (no starvation).  Admitted requests get their starting
// evaluation and join the work lists; configurations that stop are copied out (positions
// and final state, through pinned memory) and their slot and arena space are
// reused.  Each configuration's launch shape comes from the tile table by
// (d, N, M) alone, so a request's result is bitwise the same whatever else is
// being served, and the same as ss_minimize_batch gives for it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "ss.h"
#include "ss_engine.h"
#include "ss_internal.h"
#include "ss_min.h"

namespace ss {
hipError_t launch_weights(const int32_t* n, int64_t M, int d, int64_t R2, int vkind, double* v, hipStream_t st);

namespace {
using namespace eng;
using Clock = std::chrono::steady_clock;

constexpr int kDepth = 3;  // minimiser steps in flight
// admissions that may overtake the oldest queued request before the worker
// admits nothing else ahead of it
constexpr int kMaxOvertake = 16;

// first-fit allocator of byte ranges of the arena, coalescing on release
class RangeAlloc {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t o = it->first, rem = it->second - n;
      free_.erase(it);
      if (rem) free_[o + n] = rem;
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
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
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  ss_problem prob{};
  ss_min_opts opts{};
  eng::HostSlot h;          // plan, launch shape and sizes (built by ss_submit)
  std::vector<double> pos;  // [2][d][N]: the start, then the result
  int state = 0;            // 0 queued, 1 running, 2 copying out, 3 done, 4 failed
  int rc = SS_OK;
  ss_min_result res{};
  Clock::time_point t_submit;
  // while running
  int slot = -1;
  size_t off = 0, bytes = 0;
  void* pin = nullptr;  // pinned copy-out buffer: positions then MinState
  hipEvent_t done_ev = nullptr;
  int64_t iters64 = 0, evals64 = 0;  // a staged quench's FP64 stage
  size_t need = 0;      // arena bytes: workspace, positions and weights
  int overtaken = 0;    // admissions that went ahead of it while it waited
};

// arena bytes of one served configuration: its workspace, its positions and
// (weighted) its weight table
size_t request_bytes(const eng::HostSlot& h, const ss_problem& p) {
  const size_t vec = eng::al256(sizeof(double) * 2 * (size_t)h.nv);
  const size_t wbytes = p.vkind ? eng::al256(sizeof(double) * 2 * (size_t)p.M) : 0;
  return h.bytes + vec + wbytes;
}

struct InFlight {
  hipEvent_t ev;
  int q;
  std::vector<std::pair<int, uint64_t>> listed;  // (slot, occupant generation)
};

}  // namespace
}  // namespace ss

struct ss_server {
  ss_ctx* ctx = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  std::thread worker;
  std::mutex mu;  // guards everything below up to `worker-owned`
  std::condition_variable cv;
  bool stop = false;
  int error = SS_OK;
  std::string error_msg;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<ss::Request>> queue;
  ss_server_counters stats{};  // counters (under mu)
  std::map<uint64_t, std::shared_ptr<ss::Request>> tickets;
  // worker-owned
  hipStream_t st = nullptr;
  ss::RangeAlloc ranges;
  std::vector<ss::eng::HostSlot> hs;
  std::vector<std::shared_ptr<ss::Request>> slot_req;
  std::vector<uint64_t> slot_gen;
  std::vector<int> free_slots;
  std::vector<int> active;
  std::vector<std::shared_ptr<ss::Request>> copying;
  ss::EvalSlot* d_es = nullptr;
  ss::MinSlot* d_ms = nullptr;
  ss::SlotFlags* d_flags = nullptr;
  int32_t* d_list = nullptr;
  ss::BUnit* d_units = nullptr;
  size_t units_cap = 0;
  ss::SlotFlags* h_flags = nullptr;  // pinned [kDepth][max_slots]
  char* h_desc = nullptr;      // pinned [max_slots] x (EvalSlot, MinSlot) upload staging
};

namespace ss {
namespace {

void fail_all(ss_server* S, int rc, const std::string& msg) {
  std::lock_guard<std::mutex> g(S->mu);
  if (S->error == SS_OK) {
    S->error = rc;
    S->error_msg = msg;
  }
  for (auto& kv : S->tickets)
    if (kv.second->state < 3) {
      kv.second->state = 4;
      kv.second->rc = rc;
    }
  S->queue.clear();
  S->cv.notify_all();
}

class Worker {
 public:
  explicit Worker(ss_server* s) : S(s), st(s->st) {}

  void run() {
    int rc = loop();
    if (rc != SS_OK) fail_all(S, rc, err_msg);
    hipStreamSynchronize(st);
    for (auto& r : S->copying) release_copy(r);
    S->copying.clear();
    free_stages();
  }

 private:
  ss_server* S;
  hipStream_t st;
  std::string err_msg;
  std::deque<InFlight> inflight;
  std::vector<hipEvent_t> ring;
  int64_t tick = 0;
  Lists L;
  std::vector<BUnit> U;
  std::vector<int32_t> list;

  int hip_fail(hipError_t e, const char* what) {
    err_msg = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EHIP;
  }
#define W_HIP(call)                                    \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

  // work lists go through a ring of pinned staging buffers, each reused only
  // after its previous copy has completed
  struct Stage {
    char* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  };
  Stage stage[4];
  int stage_next = 0;

  int upload_lists(const std::vector<int>& slots) {
    build_lists(S->hs, slots, U, list, L);
    if (U.size() > S->units_cap) {
      W_HIP(hipStreamSynchronize(st));
      if (S->d_units) W_HIP(hipFree(S->d_units));
      S->d_units = nullptr;
      size_t cap = std::max<size_t>(U.size() * 2, 1 << 16);
      W_HIP(hipMalloc(&S->d_units, sizeof(BUnit) * cap));
      S->units_cap = cap;
    }
    Stage& sg = stage[stage_next];
    stage_next = (stage_next + 1) % 4;
    if (sg.used) W_HIP(hipEventSynchronize(sg.ev));
    const size_t ub = sizeof(BUnit) * U.size(), lb = sizeof(int32_t) * list.size();
    if (ub + lb > sg.cap) {
      if (sg.p) W_HIP(hipHostFree(sg.p));
      sg.p = nullptr;
      sg.cap = std::max<size_t>(2 * (ub + lb), 1 << 20);
      W_HIP(hipHostMalloc((void**)&sg.p, sg.cap, hipHostMallocDefault));
    }
    if (!sg.ev) W_HIP(hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming));
    memcpy(sg.p, U.data(), ub);
    memcpy(sg.p + ub, list.data(), lb);
    if (ub) W_HIP(hipMemcpyAsync(S->d_units, sg.p, ub, hipMemcpyHostToDevice, st));
    if (lb) W_HIP(hipMemcpyAsync(S->d_list, sg.p + ub, lb, hipMemcpyHostToDevice, st));
    W_HIP(hipEventRecord(sg.ev, st));
    sg.used = true;
    return SS_OK;
  }

  void free_stages() {
    for (Stage& sg : stage) {
      if (sg.p) hipHostFree(sg.p);
      if (sg.ev) hipEventDestroy(sg.ev);
      sg = Stage();
    }
  }

  DevArrays dev() const { return DevArrays{S->d_es, S->d_ms, S->d_units, S->d_list, S->d_flags}; }

  // admit queued requests in submission order while slots last: each one whose
  // arena range fits now is taken; one that does not fit is passed over, unless
  // it is the oldest and has already been overtaken kMaxOvertake times
  int admit() {
    std::vector<std::shared_ptr<Request>> waiting;
    {
      std::lock_guard<std::mutex> g(S->mu);
      waiting.assign(S->queue.begin(), S->queue.end());
    }
    std::vector<int> admitted;
    std::vector<std::shared_ptr<Request>> taken;
    std::vector<Request*> passed;  // waiting requests this scan went past
    int64_t overtook = 0;          // admissions that went ahead of a waiting request
    for (auto& r : waiting) {
      if (S->free_slots.empty()) break;
      const HostSlot& h = r->h;
      size_t off = 0;
      if (!S->ranges.alloc(r->need, &off)) {
        passed.push_back(r.get());
        if (r->overtaken >= kMaxOvertake) break;  // reserve the arena for it
        continue;
      }
      for (Request* p : passed) p->overtaken += 1;
      if (!passed.empty()) ++overtook;
      taken.push_back(r);
      const int slot = S->free_slots.back();
      S->free_slots.pop_back();
      char* mem = S->arena + off;
      const size_t vec = al256(sizeof(double) * 2 * (size_t)h.nv);
      double* x = (double*)(mem + h.bytes);
      double* v = r->prob.vkind ? (double*)(mem + h.bytes + vec) : nullptr;
      // descriptors staged in this slot's pinned cell: its previous upload was
      // consumed before the previous occupant's first step, long complete
      EvalSlot* es = (EvalSlot*)(S->h_desc + (size_t)slot * (sizeof(EvalSlot) + sizeof(MinSlot)));
      MinSlot* ms = (MinSlot*)((char*)es + sizeof(EvalSlot));
      fill_slot(h, mem, x, v, es, ms);
      W_HIP(hipMemcpyAsync(x, r->pos.data(), sizeof(double) * r->pos.size(), hipMemcpyHostToDevice, st));
      if (v) W_HIP(launch_weights(h.pl->canon_n, r->prob.M, r->prob.d, r->prob.R2, r->prob.vkind, v, st));
      W_HIP(hipMemcpyAsync(S->d_es + slot, es, sizeof(EvalSlot), hipMemcpyHostToDevice, st));
      W_HIP(hipMemcpyAsync(S->d_ms + slot, ms, sizeof(MinSlot), hipMemcpyHostToDevice, st));
      S->hs[slot] = h;
      S->slot_req[slot] = r;
      S->slot_gen[slot] += 1;
      r->slot = slot;
      r->off = off;
      r->bytes = r->need;
      admitted.push_back(slot);
    }
    if (admitted.empty()) return SS_OK;
    {
      std::lock_guard<std::mutex> g(S->mu);
      for (auto& r : taken) {
        r->state = 1;
        S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
      }
      S->stats.admitted += (int64_t)taken.size();
      S->stats.overtaking += overtook;
      S->stats.queued = (int64_t)S->queue.size();
    }
    int rc = upload_lists(admitted);
    if (rc) return rc;
    W_HIP(launch_start(S->ctx, dev(), L, st));
    for (int s : admitted) S->active.push_back(s);
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->stats.running = (int64_t)S->active.size();
      if (S->stats.running > S->stats.max_running) S->stats.max_running = S->stats.running;
    }
    return upload_lists(S->active);
  }

  int enqueue_tick() {
    W_HIP(launch_tick(S->ctx, dev(), L, st));
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->stats.steps += 1;
    }
    const int q = (int)(tick % kDepth);
    SlotFlags* hf = S->h_flags + (size_t)q * S->max_slots;
    W_HIP(hipMemcpyAsync(hf, S->d_flags, sizeof(SlotFlags) * S->max_slots, hipMemcpyDeviceToHost, st));
    W_HIP(hipEventRecord(ring[q], st));
    InFlight f{ring[q], q, {}};
    for (int s : S->active) f.listed.push_back({s, S->slot_gen[s]});
    inflight.push_back(std::move(f));
    ++tick;
    return SS_OK;
  }

  // the oldest step in flight: configurations it saw stop are copied out
  int retire_oldest() {
    InFlight f = std::move(inflight.front());
    inflight.pop_front();
    W_HIP(hipEventSynchronize(f.ev));
    const SlotFlags* hf = S->h_flags + (size_t)f.q * S->max_slots;
    bool changed = false;
    std::vector<int> sw;
    for (auto& [s, gen] : f.listed) {
      if (hf[s].running != 0 || S->slot_gen[s] != gen || !S->slot_req[s]) continue;
      auto it = std::find(S->active.begin(), S->active.end(), s);
      if (it == S->active.end()) continue;
      HostSlot& h = S->hs[s];
      if (h.phase == 0 && h.opts.precision == 2 && hf[s].status != 3) {
        // a staged quench's FP64 stage has stopped: double-double from here
        if (std::find(sw.begin(), sw.end(), s) == sw.end()) {
          S->slot_req[s]->iters64 = hf[s].iter;
          S->slot_req[s]->evals64 = hf[s].evals;
          sw.push_back(s);
        }
        continue;
      }
      S->active.erase(it);
      changed = true;
      int rc = copy_out(s);
      if (rc) return rc;
    }
    if (!sw.empty()) {
      for (int s : sw) {
        HostSlot& h = S->hs[s];
        h.phase = 1;
        // flags of steps already in flight still show the stopped FP64 stage:
        // a new generation makes them stale
        S->slot_gen[s] += 1;
        // the slot's pinned descriptor cell: its previous copy ran before this
        // configuration's first step
        MinSlot* ms = (MinSlot*)(S->h_desc + (size_t)s * (sizeof(EvalSlot) + sizeof(MinSlot)) + sizeof(EvalSlot));
        ms->P = stage_params(h, S->slot_req[s]->iters64);
        ms->keep = 1;
        W_HIP(hipMemcpyAsync(S->d_ms + s, ms, sizeof(MinSlot), hipMemcpyHostToDevice, st));
      }
      int rc = upload_lists(sw);
      if (rc) return rc;
      W_HIP(launch_start(S->ctx, dev(), L, st));
      changed = true;
    }
    if (changed && !S->active.empty()) return upload_lists(S->active);
    return SS_OK;
  }

  int copy_out(int s) {
    std::shared_ptr<Request> r = S->slot_req[s];
    const HostSlot& h = S->hs[s];
    const size_t pbytes = sizeof(double) * r->pos.size();
    W_HIP(hipHostMalloc(&r->pin, pbytes + sizeof(MinState), hipHostMallocDefault));
    W_HIP(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    const double* x = (const double*)(S->arena + r->off + h.bytes);
    // the state lives in the configuration's own workspace (see fill_slot)
    MinSlot ms;
    EvalSlot es;
    fill_slot(h, S->arena + r->off, (double*)x, nullptr, &es, &ms);
    W_HIP(hipMemcpyAsync(r->pin, x, pbytes, hipMemcpyDeviceToHost, st));
    W_HIP(hipMemcpyAsync((char*)r->pin + pbytes, ms.S, sizeof(MinState), hipMemcpyDeviceToHost, st));
    W_HIP(hipEventRecord(r->done_ev, st));
    {
      std::lock_guard<std::mutex> g(S->mu);
      r->state = 2;
      S->stats.running = (int64_t)S->active.size();
    }
    // later work on this stream runs after the copies: the slot and the range
    // can be handed out at once
    S->ranges.release(r->off, r->bytes);
    S->slot_req[s].reset();
    S->free_slots.push_back(s);
    S->copying.push_back(r);
    return SS_OK;
  }

  void release_copy(std::shared_ptr<Request>& r) {
    if (r->pin) hipHostFree(r->pin);
    if (r->done_ev) hipEventDestroy(r->done_ev);
    r->pin = nullptr;
    r->done_ev = nullptr;
  }

  // finished copies become results
  int collect(bool wait) {
    for (size_t i = 0; i < S->copying.size();) {
      std::shared_ptr<Request> r = S->copying[i];
      hipError_t e = wait ? hipEventSynchronize(r->done_ev) : hipEventQuery(r->done_ev);
      if (e == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (e != hipSuccess) return hip_fail(e, "copy-out event");
      const size_t pbytes = sizeof(double) * r->pos.size();
      memcpy(r->pos.data(), r->pin, pbytes);
      MinState ms;
      memcpy(&ms, (char*)r->pin + pbytes, sizeof(MinState));
      release_copy(r);
      {
        std::lock_guard<std::mutex> g(S->mu);
        r->res.status = ms.status;
        r->res.iters = ms.iter + r->iters64;
        r->res.evals = ms.evals + r->evals64;
        r->res.grad_evals = r->res.evals;
        r->res.phi[0] = ms.f[0];
        r->res.phi[1] = ms.f[1];
        r->res.smax[0] = ms.smax[0];
        r->res.smax[1] = ms.smax[1];
        const bool all64 = r->opts.precision == 1;
        r->res.iters_fp64 = all64 ? ms.iter : r->iters64;
        r->res.evals_fp64 = all64 ? ms.evals : r->evals64;
        r->res.seconds = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
        r->state = 3;
        S->stats.completed += 1;
        S->cv.notify_all();
      }
      S->copying.erase(S->copying.begin() + i);
    }
    return SS_OK;
  }

  int loop() {
    W_HIP(hipSetDevice(S->ctx->device));
    ring.assign(kDepth, nullptr);
    for (auto& e : ring) W_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int rc = SS_OK;
    for (;;) {
      if ((rc = admit())) break;
      if (S->active.empty()) {
        while (!inflight.empty())
          if ((rc = retire_oldest())) break;
        if (rc) break;
        if ((rc = collect(true))) break;
        std::unique_lock<std::mutex> g(S->mu);
        if (S->queue.empty() && S->stop) break;
        if (S->queue.empty()) S->cv.wait(g, [&] { return !S->queue.empty() || S->stop; });
        continue;
      }
      if ((rc = enqueue_tick())) break;
      if (inflight.size() >= (size_t)kDepth && (rc = retire_oldest())) break;
      if ((rc = collect(false))) break;
    }
    for (auto& e : ring)
      if (e) hipEventDestroy(e);
    return rc;
  }
#undef W_HIP
};

int check_request(ss_ctx* ctx, const ss_request* q, ss_problem* p) {
  if (!q) {
    ctx->last_error = "NULL request";
    return SS_EINVAL;
  }
  int64_t M = 0;
  if (q->d < 1 || q->d > 4 || q->N < 1 || q->R2 < 1 || ss_count(q->d, q->R2, &M) != SS_OK) {
    ctx->last_error = "invalid request shape";
    return SS_EINVAL;
  }
  if (q->vkind != 0 && q->vkind != 1) {
    ctx->last_error = "served requests take vkind 0 or 1";
    return SS_EINVAL;
  }
  if (!min_opts_valid(&q->opts)) {
    ctx->last_error = "invalid minimiser options";
    return SS_EINVAL;
  }
  if (!(q->L > 0.0) || !isfinite(q->L)) {
    ctx->last_error = "L must be positive and finite";
    return SS_EINVAL;
  }
  *p = ss_problem{q->d, q->N, q->R2, M, q->L, q->vkind};
  return SS_OK;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" int ss_server_start(ss_ctx* ctx, void* arena_dev, size_t arena_bytes, int max_slots) {
  if (!ctx || !arena_dev || arena_bytes == 0 || max_slots < 1 || max_slots > 65536) return SS_EINVAL;
  if (ctx->server) {
    ctx->last_error = "a server is already running on this context";
    return SS_ESTATE;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return SS_EHIP;
  ss_server* S = new (std::nothrow) ss_server();
  if (!S) return SS_ENOMEM;
  S->ctx = ctx;
  S->arena = (char*)arena_dev;
  S->arena_bytes = arena_bytes;
  S->max_slots = max_slots;
  S->ranges.reset(arena_bytes);
  S->hs.assign(max_slots, eng::HostSlot());
  S->slot_req.assign(max_slots, nullptr);
  S->slot_gen.assign(max_slots, 0);
  for (int s = max_slots - 1; s >= 0; --s) S->free_slots.push_back(s);
  bool ok = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(&S->d_es, sizeof(EvalSlot) * max_slots) == hipSuccess &&
            hipMalloc(&S->d_ms, sizeof(MinSlot) * max_slots) == hipSuccess &&
            hipMalloc(&S->d_flags, sizeof(SlotFlags) * max_slots) == hipSuccess &&
            hipMalloc(&S->d_list, sizeof(int32_t) * max_slots) == hipSuccess &&
            hipMemset(S->d_flags, 0, sizeof(SlotFlags) * max_slots) == hipSuccess &&
            hipHostMalloc((void**)&S->h_flags, sizeof(SlotFlags) * max_slots * kDepth, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void**)&S->h_desc, (sizeof(EvalSlot) + sizeof(MinSlot)) * max_slots,
                          hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    if (S->st) hipStreamDestroy(S->st);
    hipFree(S->d_es);
    hipFree(S->d_ms);
    hipFree(S->d_flags);
    hipFree(S->d_list);
    if (S->h_flags) hipHostFree(S->h_flags);
    if (S->h_desc) hipHostFree(S->h_desc);
    delete S;
    ctx->last_error = "server allocation failed";
    return SS_ENOMEM;
  }
  ctx->server = S;
  S->worker = std::thread([S] {
    Worker w(S);
    w.run();
  });
  return SS_OK;
}

extern "C" int ss_submit(ss_ctx* ctx, const ss_request* req, uint64_t* ticket) {
  if (!ctx || !ticket) return SS_EINVAL;
  ss_server* S = ctx->server;
  if (!S) {
    ctx->last_error = "no server is running (ss_server_start)";
    return SS_ESTATE;
  }
  ss_problem p;
  int rc = check_request(ctx, req, &p);
  if (rc) return rc;
  auto r = std::make_shared<Request>();
  r->prob = p;
  r->opts = req->opts;
  rc = eng::setup_slot(ctx, &p, &req->opts, &r->h);
  if (rc) return rc;
  r->need = request_bytes(r->h, p);
  if (r->need > S->arena_bytes) {
    ctx->last_error = "request needs " + std::to_string(r->need) + " arena bytes, the server arena holds " +
                      std::to_string(S->arena_bytes);
    return SS_ENOMEM;
  }
  if (req->pos_host) {
    r->pos.assign(req->pos_host, req->pos_host + (size_t)2 * p.d * p.N);
  } else {
    r->pos.resize((size_t)2 * p.d * p.N);
    rc = ss_uniform_positions(p.d, p.N, req->seed, r->pos.data());
    if (rc) return rc;
  }
  for (double x : r->pos)
    if (!isfinite(x)) {
      ctx->last_error = "positions are not finite";
      return SS_EINVAL;
    }
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> g(S->mu);
  if (S->error != SS_OK) {
    ctx->last_error = S->error_msg;
    return S->error;
  }
  if (S->stop) {
    ctx->last_error = "server is stopping";
    return SS_ESTATE;
  }
  r->ticket = S->next_ticket++;
  S->tickets[r->ticket] = r;
  S->queue.push_back(r);
  S->stats.submitted += 1;
  S->stats.queued = (int64_t)S->queue.size();
  *ticket = r->ticket;
  S->cv.notify_all();
  return SS_OK;
}

extern "C" int ss_poll(ss_ctx* ctx, uint64_t ticket, ss_min_result* out, double* pos_host_out) {
  if (!ctx) return SS_EINVAL;
  ss_server* S = ctx->server;
  if (!S) {
    ctx->last_error = "no server is running";
    return SS_ESTATE;
  }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return SS_ENOTFOUND;
  std::shared_ptr<Request> r = it->second;
  if (r->state < 3) return SS_PENDING;
  S->tickets.erase(it);
  if (r->state == 4) {
    ctx->last_error = r->rc == SS_ENOMEM && S->error == SS_OK ? "request does not fit in the server arena"
                                                               : (S->error_msg.empty() ? "request failed" : S->error_msg);
    return r->rc;
  }
  if (out) *out = r->res;
  if (pos_host_out) memcpy(pos_host_out, r->pos.data(), sizeof(double) * r->pos.size());
  return SS_OK;
}

extern "C" int ss_server_stats(ss_ctx* ctx, ss_server_counters* out) {
  if (!ctx || !out) return SS_EINVAL;
  ss_server* S = ctx->server;
  if (!S) {
    ctx->last_error = "no server is running";
    return SS_ESTATE;
  }
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->stats;
  return SS_OK;
}

extern "C" int ss_server_stop(ss_ctx* ctx) {
  if (!ctx) return SS_EINVAL;
  ss_server* S = ctx->server;
  if (!S) return SS_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  const int err = S->error;
  hipStreamSynchronize(S->st);
  hipStreamDestroy(S->st);
  hipFree(S->d_es);
  hipFree(S->d_ms);
  hipFree(S->d_flags);
  hipFree(S->d_list);
  if (S->d_units) hipFree(S->d_units);
  hipHostFree(S->h_flags);
  hipHostFree(S->h_desc);
  ctx->server = nullptr;
  delete S;
  return err;
}
