// Serving loop: many independent ppRPA solves on one device (continuous batching).
//
// * Admission (admission thread): requests are taken in arrival order; each needs one contiguous
//   reservation of its exact device footprint (staged integrals, sigma buffers, Davidson
//   workspace) inside the server's HBM arena, and a free slot (stream + pinned status buffer).
//   A request that does not fit waits until finished requests release memory; one larger than
//   the whole arena fails with ENOMEM. The build and the initial subspace run on the slot's
//   stream; after that the caller's input buffers are no longer read.
// * Progress (worker thread): every in-flight solve is a Davidson phase machine. Each pass the
//   worker advances every solve whose stream has drained. A solve that needs a sigma product has
//   its block unpacked at once on its own stream; the solves waiting for sigma are then launched
//   together as one grouped grid on the group stream, ordered after each member's unpack by an
//   event, with the epilogue back on each request's stream, ordered after the grid by an event.
//   Solves come in two size classes by the cost of one sigma product (small and large), each
//   with its own group stream and at most one grid in flight, so a small solve's sigma does not
//   queue behind a large one's. Within a class the solves that become ready while its grid runs
//   form the next group (continuous batching), so the groups grow with the load; a small-class
//   launch is held for up to HOLD_US while other small solves of the same variant are still in
//   their Davidson phases, so that solves running side by side fall into one grid. Solves of
//   different kernel variants (sigma precision, FP64 kernel by size) cannot share a grid; the
//   variant whose waiting block has waited longest goes next, so no request is overtaken by more
//   than one launch per other variant of its class. A member's work units are
//   those of a launch of its own (same decomposition, same partial-sum buffer), so its results do
//   not depend on the mix it was served in.
// * Finished solves copy out their roots, release their reservation and slot, and wake the
//   admission thread.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "solver.h"

namespace pprpa {
namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of byte ranges in one device allocation (offsets 256-byte aligned).
class Arena {
 public:
  bool init(size_t bytes) {
    size_ = bytes / 256 * 256;
    free_.clear();
    if (size_) free_[0] = size_;
    return size_ > 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    const size_t b = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      *off = it->first;
      const size_t rest = it->second - b;
      const size_t roff = it->first + b;
      free_.erase(it);
      if (rest) free_[roff] = rest;
      used_ += b;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    const size_t b = (bytes + 255) / 256 * 256;
    used_ -= b;
    auto it = free_.emplace(off, b).first;
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
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  pprpa_build_args b{};
  pprpa_davidson_args d{};
  size_t footprint = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  size_t off = 0;
  Slab slab;
  pprpa_ctx* ctx = nullptr;
  std::unique_ptr<Solver> sv;
  bool unpacked = false;  // the pending sigma block is unpacked (ctx->e0 marks its end)
  int cls = 0;            // size class: 0 small, 1 large (one sigma product >= LARGE_FLOPS)
  double t_wait = 0;      // when the pending sigma block started waiting for a grouped launch
  int overtaken = 0;      // launch rounds of other variants while the pending block waited
  int max_overtaken = 0;
  pprpa_status status = PPRPA_OK;
  std::string message;
  double omega[64] = {0}, resid[64] = {0};
  pprpa_report rep{};
};

struct TimedGroup {
  hipEvent_t a, b;
  double flops;
  int members;
  int cls;
};

constexpr int NCLS = 2;
constexpr double LARGE_FLOPS = 1e10;  // flops of one single-vector sigma from which a solve is large
constexpr double HOLD_US = 300.0;     // longest hold of a small-class launch for more members

}  // namespace
}  // namespace pprpa

using namespace pprpa;

struct pprpa_server {
  int device = 0;
  Clock::time_point t0;
  size_t budget = 0;
  int max_inflight = 0;
  char* base = nullptr;  // the arena's device memory
  Arena arena;
  std::vector<hipStream_t> streams;  // one per slot
  hipStream_t gstream[2] = {nullptr, nullptr};  // grouped sigma launches, per size class
  double* pinned = nullptr;          // max_inflight * PINNED_ELEMS
  std::vector<int> free_slots;

  std::mutex mu;
  std::condition_variable cv_admit, cv_work, cv_done;
  bool stop = false, admitter_done = false;
  uint64_t next_ticket = 1;
  std::deque<Request*> queue;
  std::vector<Request*> admitted;  // built, not yet picked up by the worker
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  pprpa_serving_stats st{};

  std::thread admitter, worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void finish_request(pprpa_server* S, Request* r, pprpa_status status, const std::string& msg) {
  // called with S->mu held
  r->status = status;
  r->message = msg;
  r->state = 2;
  r->t_done = S->now();
  S->st.completed += 1;
  if (status != PPRPA_OK) S->st.failed += 1;
  S->cv_done.notify_all();
}

void release_resources(pprpa_server* S, Request* r) {
  // called with S->mu held; the request's stream has drained
  if (r->slot >= 0) {
    S->free_slots.push_back(r->slot);
    r->slot = -1;
  }
  if (r->slab.base) {
    S->arena.release(r->off, r->footprint);
    r->slab = Slab{};
    S->st.reserved = S->arena.used();
  }
  S->cv_admit.notify_all();
}

void admission_loop(pprpa_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_admit.wait(lk, [&] { return S->stop || (!S->queue.empty() && !S->free_slots.empty()); });
    if (S->stop) break;
    Request* r = S->queue.front();
    if (r->footprint > S->arena.size()) {
      S->queue.pop_front();
      S->st.queued = (int64_t)S->queue.size();
      char buf[160];
      snprintf(buf, sizeof buf, "request needs %zu bytes of device memory, the server holds %zu",
               r->footprint, S->arena.size());
      finish_request(S, r, PPRPA_ENOMEM, buf);
      continue;
    }
    size_t off = 0;
    if (!S->arena.alloc(r->footprint, &off)) {
      S->cv_admit.wait(lk);  // woken when a finished request releases memory (or on stop)
      continue;
    }
    S->queue.pop_front();
    S->st.queued = (int64_t)S->queue.size();
    r->off = off;
    r->slab.base = S->base + off;
    r->slab.size = r->footprint;
    r->slab.top = 0;
    r->slot = S->free_slots.back();
    S->free_slots.pop_back();
    S->st.reserved = S->arena.used();
    S->st.peak_reserved = std::max<uint64_t>(S->st.peak_reserved, S->arena.used());
    r->t_admit = S->now();
    lk.unlock();

    pprpa_build_args b = r->b;
    b.stream = S->streams[r->slot];
    pprpa_status rc = build_context(&b, &r->slab, S->pinned + (size_t)r->slot * PINNED_ELEMS, &r->ctx);
    std::string msg = rc == PPRPA_OK ? std::string() : std::string(pprpa_last_error());
    if (rc == PPRPA_OK) {
      r->sv.reset(new Solver(r->ctx, r->d));
      r->sv->start();  // errors end in phase DONE; the worker finishes the request
      rc = hipStreamSynchronize(S->streams[r->slot]) == hipSuccess ? PPRPA_OK : PPRPA_EDEVICE;
      if (rc != PPRPA_OK) msg = "device error after the initial subspace";
    }

    lk.lock();
    if (rc != PPRPA_OK) {
      if (r->ctx) {
        free_context(r->ctx);
        r->ctx = nullptr;
      }
      r->sv.reset();
      release_resources(S, r);
      finish_request(S, r, rc, msg);
      continue;
    }
    r->state = 1;
    {
      const Geometry& g = r->ctx->g;
      const double f1 = 4.0 * g.naux * (double)(g.nv + g.no) * ((double)g.nv * g.nv + (double)g.no * g.no);
      r->cls = f1 >= LARGE_FLOPS ? 1 : 0;
    }
    S->admitted.push_back(r);
    S->st.inflight += 1;
    S->st.peak_inflight = std::max(S->st.peak_inflight, S->st.inflight);
    S->cv_work.notify_all();
  }
  S->admitter_done = true;
  S->cv_work.notify_all();
}

// Grouped sigma for the solves in `grp` (all in NEED_SIGMA with their block unpacked, one kernel
// variant).
// Returns false if the group launch failed (its members are then failed by the caller).
bool launch_group(pprpa_server* S, std::vector<Request*>& grp, int cls,
                  std::vector<TimedGroup>& timed, std::vector<hipEvent_t>& pool) {
  hipStream_t gs = S->gstream[cls];
  GroupMember m[GROUP_MAX];
  int ns[GROUP_MAX];
  double flops = 0.0;
  const int cnt = (int)grp.size();
  for (int i = 0; i < cnt; ++i) {
    Request* r = grp[i];
    pprpa_ctx* c = r->ctx;
    Solver& sv = *r->sv;
    const int k = sv.sig_k;
    ns[i] = nsplit_for(c, k);
    if (hipStreamWaitEvent(gs, c->e0, 0) != hipSuccess) return false;
    SigmaLaunch la{};
    la.L = c->L;
    la.ZT = c->ZT;
    la.Sp = c->Sp;
    la.k = k;
    la.nsplit = ns[i];
    la.npan_v = c->plan.npan_v;
    la.plane = c->plane;
    la.zplane = c->zplane;
    la.nprod = c->nprod;
    m[i] = GroupMember{&c->g, &c->plan, la};
    const Geometry& g = c->g;
    flops += 4.0 * g.naux * (double)(g.nv + g.no) * ((double)g.nv * g.nv + (double)g.no * g.no) * k;
  }
  TimedGroup tg{};
  auto take = [&](hipEvent_t* e) {
    if (!pool.empty()) {
      *e = pool.back();
      pool.pop_back();
      return hipSuccess;
    }
    return hipEventCreate(e);
  };
  if (take(&tg.a) != hipSuccess || take(&tg.b) != hipSuccess) return false;
  tg.flops = flops;
  tg.members = cnt;
  tg.cls = cls;
  if (hipEventRecord(tg.a, gs) != hipSuccess) return false;
  if (launch_sigma_group(m, cnt, gs) != hipSuccess) return false;
  if (hipEventRecord(tg.b, gs) != hipSuccess) return false;
  timed.push_back(tg);
  for (int i = 0; i < cnt; ++i) {
    Request* r = grp[i];
    pprpa_ctx* c = r->ctx;
    Solver& sv = *r->sv;
    const int64_t n = c->g.n;
    if (hipStreamWaitEvent(c->stream, tg.b, 0) != hipSuccess) return false;
    if (launch_epilogue(c->g, c->st, sv.w.V + (size_t)sv.sig_m0 * n, sv.sig_k, c->Sp, ns[i], c->ptab,
                        c->epair, sv.w.SV + (size_t)sv.sig_m0 * n, c->stream) != hipSuccess)
      return false;
    r->unpacked = false;
    sv.sigma_done(false);
  }
  return true;
}

void worker_loop(pprpa_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<Request*> active;
  std::vector<TimedGroup> timed;
  std::vector<hipEvent_t> pool;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (active.empty() && S->admitted.empty()) {
        if (S->admitter_done) break;
        S->cv_work.wait(lk, [&] { return !S->admitted.empty() || S->admitter_done; });
      }
      active.insert(active.end(), S->admitted.begin(), S->admitted.end());
      S->admitted.clear();
    }
    bool progressed = false;
    std::map<int, std::vector<Request*>> need[NCLS];  // per class, by kernel variant
    std::map<int, int> busy_phases[NCLS];             // per class and variant: solves in phases
    std::vector<Request*> finished;
    for (Request* r : active) {
      Solver& sv = *r->sv;
      if (sv.phase == Solver::RR_LAUNCH) {
        sv.advance();
        progressed = true;
      } else if (sv.phase != Solver::NEED_SIGMA && sv.phase != Solver::DONE) {
        const hipError_t q = hipStreamQuery(r->ctx->stream);
        if (q == hipSuccess) {
          sv.advance();
          progressed = true;
        } else if (q != hipErrorNotReady) {
          (void)hipGetLastError();
          sv.phase = Solver::DONE;
          sv.status = PPRPA_EDEVICE;
          sv.message = std::string("stream error: ") + hipGetErrorString(q);
        }
      }
      if (sv.phase == Solver::NEED_SIGMA) {
        pprpa_ctx* c = r->ctx;
        if (sv.sig_k > c->kcap) {
          // a block wider than the request's sigma buffers (initial guesses): its own launches
          const int64_t n = c->g.n;
          if (sigma_device(c, sv.sig_k, sv.w.V + (size_t)sv.sig_m0 * n,
                           sv.w.SV + (size_t)sv.sig_m0 * n) != PPRPA_OK) {
            sv.phase = Solver::DONE;
            sv.status = PPRPA_EDEVICE;
            sv.message = pprpa_last_error();
          } else {
            sv.sigma_done(false);
          }
          progressed = true;
        } else {
          if (!r->unpacked) {
            const int64_t n = c->g.n;
            if (launch_unpack(c->g, c->st, sv.w.V + (size_t)sv.sig_m0 * n, sv.sig_k, c->ptab, c->ZT,
                              c->zplane, c->stream) != hipSuccess ||
                hipEventRecord(c->e0, c->stream) != hipSuccess) {
              (void)hipGetLastError();
              sv.phase = Solver::DONE;
              sv.status = PPRPA_EDEVICE;
              sv.message = "unpack launch failed";
            } else {
              r->unpacked = true;
              r->t_wait = S->now();
              r->overtaken = 0;
              progressed = true;
            }
          }
          if (r->unpacked) need[r->cls][c->plan.variant * 8 + c->nprod].push_back(r);
        }
      } else if (sv.phase != Solver::DONE) {
        busy_phases[r->cls][r->ctx->plan.variant * 8 + r->ctx->nprod] += 1;
      }
      if (sv.phase == Solver::DONE) finished.push_back(r);
    }
    // fold finished group timings into the statistics (grids of the two classes finish in any
    // order)
    bool cls_busy[NCLS] = {false, false};
    for (size_t i = 0; i < timed.size();) {
      if (hipEventQuery(timed[i].b) != hipSuccess) {
        cls_busy[timed[i].cls] = true;
        ++i;
        continue;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, timed[i].a, timed[i].b);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.group_launches += 1;
        S->st.grouped_products += timed[i].members;
        S->st.sigma_seconds += ms * 1e-3;
        S->st.sigma_flops += timed[i].flops;
      }
      pool.push_back(timed[i].a);
      pool.push_back(timed[i].b);
      timed.erase(timed.begin() + i);
    }

    // per class, one grouped grid in flight at a time: once the last one is done, launch the
    // waiting solves of the variant whose block has waited longest (all of them, in grids of
    // GROUP_MAX); a small-class launch waits up to HOLD_US for solves of that variant still in
    // their phases
    const double now_s = S->now();
    for (int cls = 0; cls < NCLS; ++cls) {
      if (cls_busy[cls] || need[cls].empty()) continue;
      auto oldest = [](const std::vector<Request*>& v) {
        double t = v.front()->t_wait;
        for (const Request* r : v) t = std::min(t, r->t_wait);
        return t;
      };
      auto pick = need[cls].begin();
      for (auto it = need[cls].begin(); it != need[cls].end(); ++it)
        if (oldest(it->second) < oldest(pick->second)) pick = it;
      if (cls == 0 && busy_phases[cls][pick->first] > 0 &&
          (now_s - oldest(pick->second)) * 1e6 < HOLD_US)
        continue;  // hold: more members are on their way
      const std::vector<Request*>& list = pick->second;
      for (auto& kv : need[cls]) {
        if (kv.first == pick->first) continue;
        for (Request* r : kv.second) r->overtaken += 1;
      }
      for (Request* r : list) {
        r->max_overtaken = std::max(r->max_overtaken, r->overtaken);
        r->overtaken = 0;
      }
      for (size_t i0 = 0; i0 < list.size(); i0 += GROUP_MAX) {
        std::vector<Request*> grp(list.begin() + i0,
                                  list.begin() + std::min(list.size(), i0 + GROUP_MAX));
        if (!launch_group(S, grp, cls, timed, pool)) {
          (void)hipGetLastError();
          for (Request* r : grp) {
            r->sv->phase = Solver::DONE;
            r->sv->status = PPRPA_EDEVICE;
            r->sv->message = "grouped sigma launch failed";
            if (std::find(finished.begin(), finished.end(), r) == finished.end()) finished.push_back(r);
          }
        }
        progressed = true;
      }
    }
    for (Request* r : finished) {
      Solver& sv = *r->sv;
      pprpa_status status = sv.status;
      std::string msg = sv.message;
      (void)hipStreamSynchronize(r->ctx->stream);
      if (sv.results(r->omega, nullptr, r->resid, &r->rep) != PPRPA_OK && status == PPRPA_OK) {
        status = PPRPA_EDEVICE;
        msg = pprpa_last_error();
      }
      free_context(r->ctx);
      r->ctx = nullptr;
      r->sv.reset();
      active.erase(std::find(active.begin(), active.end(), r));
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.inflight -= 1;
      release_resources(S, r);
      finish_request(S, r, status, msg);
      progressed = true;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  for (auto& t : timed) {
    (void)hipEventSynchronize(t.b);
    pool.push_back(t.a);
    pool.push_back(t.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

void destroy_server(pprpa_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Request* r : S->queue)
      finish_request(S, r, PPRPA_EBUSY, "server destroyed before the request was admitted");
    S->queue.clear();
  }
  S->cv_admit.notify_all();
  if (S->admitter.joinable()) S->admitter.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->admitter_done = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (hipStream_t s : S->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipStream_t g : S->gstream)
    if (g) (void)hipStreamDestroy(g);
  if (S->pinned) (void)hipHostFree(S->pinned);
  if (S->base) (void)hipFree(S->base);
  delete S;
}

}  // namespace

extern "C" {

pprpa_status pprpa_server_create(size_t hbm_budget_bytes, int32_t max_inflight, pprpa_server** out) {
  if (!out) {
    set_error("out is NULL");
    return PPRPA_EINVAL;
  }
  *out = nullptr;
  if (max_inflight < 1 || max_inflight > 64) {
    set_error("max_inflight=%d outside [1, 64]", max_inflight);
    return PPRPA_EINVAL;
  }
  if (hbm_budget_bytes < (size_t(1) << 20)) {
    set_error("hbm_budget_bytes=%zu below 1 MiB", hbm_budget_bytes);
    return PPRPA_EINVAL;
  }
  pprpa_server* S = new (std::nothrow) pprpa_server();
  if (!S) {
    set_error("host allocation failed");
    return PPRPA_EINVAL;
  }
  S->t0 = Clock::now();
  S->max_inflight = max_inflight;
  auto fail = [&](pprpa_status s, const char* what, hipError_t e) {
    (void)hipGetLastError();
    set_error("%s: %s", what, hipGetErrorString(e));
    destroy_server(S);
    return s;
  };
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) return fail(PPRPA_EDEVICE, "hipGetDevice", e);
  S->arena.init(hbm_budget_bytes);
  S->budget = S->arena.size();
  e = hipMalloc((void**)&S->base, S->budget);
  if (e != hipSuccess) return fail(PPRPA_ENOMEM, "reserving the serving arena", e);
  e = hipHostMalloc((void**)&S->pinned, (size_t)max_inflight * PINNED_ELEMS * sizeof(double),
                    hipHostMallocDefault);
  if (e != hipSuccess) return fail(PPRPA_ENOMEM, "pinned status buffers", e);
  S->streams.assign(max_inflight, nullptr);
  for (int i = 0; i < max_inflight; ++i) {
    e = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) return fail(PPRPA_EDEVICE, "stream creation", e);
    S->free_slots.push_back(max_inflight - 1 - i);
  }
  for (hipStream_t& g : S->gstream) {
    e = hipStreamCreateWithFlags(&g, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(PPRPA_EDEVICE, "stream creation", e);
  }
  if (prepare_kernels() != hipSuccess) return fail(PPRPA_EDEVICE, "kernel set-up", hipGetLastError());
  S->st.budget = S->budget;
  S->admitter = std::thread(admission_loop, S);
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return PPRPA_OK;
}

pprpa_status pprpa_server_submit(pprpa_server* S, const pprpa_build_args* b,
                                 const pprpa_davidson_args* d, uint64_t* ticket) {
  if (!S || !b || !d || !ticket) {
    set_error("server, build args, Davidson args and ticket must not be NULL");
    return PPRPA_EINVAL;
  }
  PPRPA_TRY(check_build_args(b));
  if (d->direct) {
    set_error("the serving loop runs the Davidson solver only (direct=0)");
    return PPRPA_EUNSUPPORTED;
  }
  std::unique_ptr<Request> r(new Request());
  r->b = *b;
  r->b.dense = 0;
  r->b.stream = nullptr;
  // sigma buffers wide enough for every block of the solve
  const int blk = d->block > 0 ? d->block : d->nroot;
  r->b.max_block = std::min(64, std::max(1, std::max(blk, d->nroot)));
  r->d = *d;
  r->footprint = context_footprint(&r->b, &r->d);
  if (r->footprint == 0) {
    if (std::string(pprpa_last_error()).empty()) set_error("invalid request");
    return PPRPA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) {
    set_error("server is shutting down");
    return PPRPA_EBUSY;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = S->now();
  *ticket = r->ticket;
  S->queue.push_back(r.get());
  S->st.submitted += 1;
  S->st.queued = (int64_t)S->queue.size();
  S->all.emplace(r->ticket, std::move(r));
  S->cv_admit.notify_all();
  return PPRPA_OK;
}

pprpa_status pprpa_server_poll(pprpa_server* S, uint64_t ticket, pprpa_request_info* info,
                               double* omega, double* resid, pprpa_report* rep) {
  if (!S || !info) {
    set_error("server and info must not be NULL");
    return PPRPA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) {
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return PPRPA_EINVAL;
  }
  Request* r = it->second.get();
  std::memset(info, 0, sizeof *info);
  info->state = r->state;
  info->status = r->status;
  info->nroot = r->d.nroot;
  info->max_overtaken = r->max_overtaken;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
  info->footprint = r->footprint;
  snprintf(info->message, sizeof info->message, "%s", r->message.c_str());
  if (r->state == 2) {
    if (omega) std::copy(r->omega, r->omega + r->d.nroot, omega);
    if (resid) std::copy(r->resid, r->resid + r->d.nroot, resid);
    if (rep) *rep = r->rep;
    S->all.erase(it);
  }
  return PPRPA_OK;
}

pprpa_status pprpa_server_wait(pprpa_server* S, uint64_t ticket, double timeout_s) {
  if (!S) {
    set_error("server is NULL");
    return PPRPA_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto done = [&] {
    auto it = S->all.find(ticket);
    return it == S->all.end() || it->second->state == 2;
  };
  if (S->all.find(ticket) == S->all.end()) {
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return PPRPA_EINVAL;
  }
  if (timeout_s < 0) {
    S->cv_done.wait(lk, done);
    return PPRPA_OK;
  }
  if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    set_error("request %llu not finished after %.3f s", (unsigned long long)ticket, timeout_s);
    return PPRPA_EBUSY;
  }
  return PPRPA_OK;
}

pprpa_status pprpa_server_stats(pprpa_server* S, pprpa_serving_stats* out) {
  if (!S || !out) {
    set_error("server and out must not be NULL");
    return PPRPA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->reserved = S->arena.used();
  return PPRPA_OK;
}

void pprpa_server_destroy(pprpa_server* S) { destroy_server(S); }

}  // extern "C"
