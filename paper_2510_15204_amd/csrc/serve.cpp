// Serving: ps_submit / ps_wait with continuous batching.
//
// A dispatcher thread owns a small set of slots (stream + device arena + pinned staging).  Queued
// jobs are admitted in arrival order whenever a slot is free and the arenas of all busy slots plus
// the new job fit the context's device-memory budget; each admitted job is enqueued on its own
// slot's stream, so jobs that arrive while others run overlap on the device.  Completion is polled
// with hipEventQuery; host outputs pass through the slot's pinned buffer.  A job's plan (grids,
// tiles, split counts, reduction order) depends only on the job itself, so its results are the same
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "jobs.h"

namespace psint {

namespace {
using clk = std::chrono::steady_clock;
constexpr int kMaxSlots = 4;
constexpr size_t kMaxQueue = 1 << 16;
}  // namespace

struct OwnedJob {
  ps_job job;
  std::vector<ps_atom> atoms;
  std::vector<ps_sto> basis, aux;
  std::vector<ps_pair_grid> pairs;
};

struct Ticket {
  uint64_t id = 0;
  OwnedJob oj;
  clk::time_point submitted, admitted, done_at;
  bool done = false;
  int32_t status = PS_OK;
  ps_job_stats stats{};
  size_t need_bytes = 0;
  int slot = -1;
  Plan plan;
  Layout layout;
};

struct ServeState {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Ticket>> queue;
  std::map<uint64_t, std::shared_ptr<Ticket>> tickets;
  std::vector<Slot> slots;
  std::vector<std::shared_ptr<Ticket>> running;  // per slot
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
};

static void copy_job(const ps_job* j, OwnedJob& o) {
  o.job = *j;
  o.atoms.assign(j->atoms, j->atoms + j->n_atoms);
  if (j->n_bf) o.basis.assign(j->basis, j->basis + j->n_bf);
  if (j->n_aux) o.aux.assign(j->aux, j->aux + j->n_aux);
  if (j->n_pair_grids) o.pairs.assign(j->pair_grids, j->pair_grids + j->n_pair_grids);
  o.job.atoms = o.atoms.data();
  o.job.basis = o.basis.empty() ? nullptr : o.basis.data();
  o.job.aux = o.aux.empty() ? nullptr : o.aux.data();
  o.job.pair_grids = o.pairs.empty() ? nullptr : o.pairs.data();
}

static void finish_ticket(ps_ctx* ctx, ServeState& S, int si) {
  auto t = S.running[si];
  Slot& s = S.slots[si];
  t->done_at = clk::now();
  if (t->status == PS_OK) {
    // host outputs: unpack the pinned bounce region
    const ps_job& j = t->oj.job;
    if (j.out_location == PS_OUT_HOST) {
      const Plan& p = t->plan;
      const size_t nb2 = (size_t)p.n_bf * p.n_bf * 8, na2 = (size_t)p.n_aux * p.n_aux * 8;
      double* dsts[6] = {j.S, j.T, j.V, j.PQ, j.PQ_chol, j.abP};
      size_t sizes[6] = {nb2, nb2, nb2, na2, na2, (size_t)p.n_aux * nb2};
      const char* src = (const char*)s.pinned + t->layout.meta_end;
      for (int k = 0; k < 6; ++k) {
        if (!dsts[k] || !sizes[k]) continue;
        std::memcpy(dsts[k], src, sizes[k]);
        src += sizes[k];
      }
    }
    double total = std::chrono::duration<double, std::milli>(t->done_at - t->submitted).count();
    double queue = std::chrono::duration<double, std::milli>(t->admitted - t->submitted).count();
    t->status = finish_stats(ctx, s, t->plan, t->layout, &t->stats, total, queue);
  }
  t->plan = Plan();
  t->done = true;
  S.running[si].reset();
}

static void worker_loop(ps_ctx* ctx) {
  ServeState& S = *ctx->serve.load();
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(S.mu);
  while (true) {
    // completions
    bool any_done = false;
    for (int si = 0; si < (int)S.slots.size(); ++si) {
      if (!S.running[si]) continue;
      hipError_t q = hipEventQuery(S.slots[si].ev_end);
      if (q == hipSuccess) {
        finish_ticket(ctx, S, si);
        any_done = true;
      } else if (q != hipErrorNotReady) {
        S.running[si]->status = PS_E_DEVICE;
        set_err(ctx, std::string("serving: ") + hipGetErrorString(q));
        finish_ticket(ctx, S, si);
        any_done = true;
      }
    }
    if (any_done) S.cv_done.notify_all();
    // admissions, in arrival order
    while (!S.queue.empty()) {
      auto t = S.queue.front();
      // the synchronous slot's arena (ps_compute on this context) shares the budget
      size_t busy = ctx->sync_arena_bytes.load();
      int free_slot = -1;
      for (int si = 0; si < (int)S.slots.size(); ++si) {
        if (S.running[si]) busy += S.slots[si].arena_size;
        else if (free_slot < 0 || S.slots[si].arena_size > S.slots[free_slot].arena_size) free_slot = si;
      }
      if (free_slot < 0) break;
      // no ps_compute running: its slot's arena (kept for a repeat of its last job) goes back to
      // the pool, with the plan and graph that refer to it; false if a ps_compute holds the slot
      auto reclaim_sync = [&]() {
        if (!ctx->sync_mu.try_lock()) return false;
        release_sync_arena(ctx);
        ctx->sync_mu.unlock();
        return true;
      };
      bool sync_busy = false;
      if (busy + t->need_bytes > ctx->budget && ctx->sync_arena_bytes.load() > 0) {
        sync_busy = !reclaim_sync();
        busy = ctx->sync_arena_bytes.load();
        for (int si = 0; si < (int)S.slots.size(); ++si)
          if (S.running[si]) busy += S.slots[si].arena_size;
      }
      if (busy + t->need_bytes > ctx->budget) break;  // wait for memory to free up
      // the job's arena: the free slot's own range if large enough, else a range from the context's
      // pool, after giving back the ranges of idle slots (then of an idle ps_compute slot) if the
      // pool has no room
      Slot& s = S.slots[free_slot];
      if (s.arena_size < t->need_bytes) {
        pool_release(ctx, s.arena, s.arena_size);
        s.arena = nullptr;
        s.arena_size = 0;
        size_t got = 0;
        void* p = pool_alloc(ctx, t->need_bytes, &got);
        if (!p) {
          for (int si = 0; si < (int)S.slots.size(); ++si)
            if (!S.running[si] && S.slots[si].arena) {
              pool_release(ctx, S.slots[si].arena, S.slots[si].arena_size);
              S.slots[si].arena = nullptr;
              S.slots[si].arena_size = 0;
            }
          p = pool_alloc(ctx, t->need_bytes, &got);
        }
        if (!p) {
          sync_busy = !reclaim_sync();
          p = pool_alloc(ctx, t->need_bytes, &got);
        }
        bool any_running = sync_busy;
        for (auto& r : S.running) any_running = any_running || (bool)r;
        if (!p && any_running) break;  // wait for a running job to give its range back
        s.arena = p;
        s.arena_size = p ? got : 0;
      }
      S.queue.pop_front();
      t->admitted = clk::now();
      t->slot = free_slot;
      const bool host_out = t->oj.job.out_location == PS_OUT_HOST;
      int32_t rc = bind_slot(ctx, s, t->plan, t->layout, host_out ? output_bytes(t->plan, t->oj.job) : 0,
                             t->oj.job.PQ_chol != nullptr);
      if (rc == PS_OK) rc = enqueue_job(ctx, s, t->plan, t->layout);
      if (rc == PS_OK)
        rc = enqueue_outputs(ctx, s, t->plan, t->layout, t->oj.job,
                             t->oj.job.out_location == PS_OUT_HOST ? (char*)s.pinned + t->layout.meta_end : nullptr);
      S.running[free_slot] = t;
      if (rc != PS_OK) {
        t->status = rc;
        (void)hipStreamSynchronize(s.stream);
        finish_ticket(ctx, S, free_slot);
        S.cv_done.notify_all();
      }
    }
    bool busy = false;
    for (auto& r : S.running)
      if (r) busy = true;
    if (S.stop && !S.queue.empty()) {
      // ps_destroy: jobs not yet admitted are not started (running ones finish first)
      for (auto& q : S.queue) {
        q->status = PS_E_DEVICE;
        q->done = true;
      }
      S.queue.clear();
      S.cv_done.notify_all();
    }
    if (S.stop && S.queue.empty() && !busy) break;
    if (busy)
      S.cv_work.wait_for(lk, std::chrono::microseconds(50));
    else if (!S.queue.empty())  // waiting for a ps_compute on this context to finish
      S.cv_work.wait_for(lk, std::chrono::microseconds(500));
    else
      S.cv_work.wait(lk, [&] { return S.stop || !S.queue.empty(); });
  }
}

static int32_t serve_start(ps_ctx* ctx) {
  if (ctx->serve.load()) return PS_OK;
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  if (ctx->serve.load()) return PS_OK;
  ServeState* st = new ServeState();
  st->slots.resize(kMaxSlots);
  st->running.resize(kMaxSlots);
  for (auto& s : st->slots) {
    int32_t rc = slot_init(ctx, s, nullptr);
    if (rc) {
      for (auto& s2 : st->slots) slot_free(ctx, s2);
      delete st;
      return rc;
    }
  }
  ctx->serve.store(st);
  st->worker = std::thread(worker_loop, ctx);
  return PS_OK;
}

void serve_shutdown(ps_ctx* ctx) {
  ServeState* st = ctx->serve.load();
  if (!st) return;
  {
    std::lock_guard<std::mutex> g(st->mu);
    st->stop = true;
  }
  st->cv_work.notify_all();
  if (st->worker.joinable()) st->worker.join();
  for (auto& s : st->slots) slot_free(ctx, s);
  ctx->serve.store(nullptr);
  delete st;
}

void release_idle_serve_arenas(ps_ctx* ctx) {
  ServeState* st = ctx->serve.load();
  if (!st) return;
  std::lock_guard<std::mutex> g(st->mu);
  for (int si = 0; si < (int)st->slots.size(); ++si)
    if (!st->running[si] && st->slots[si].arena) {
      pool_release(ctx, st->slots[si].arena, st->slots[si].arena_size);
      st->slots[si].arena = nullptr;
      st->slots[si].arena_size = 0;
    }
}

}  // namespace psint

using namespace psint;

extern "C" {

int32_t ps_submit(ps_ctx* ctx, const ps_job* job, uint64_t* ticket) {
  if (!ctx || !job || !ticket) return PS_E_INVALID;
  auto t = std::make_shared<Ticket>();
  t->submitted = clk::now();
  // plan once on the caller's thread; bad or oversized jobs are rejected here
  copy_job(job, t->oj);
  int32_t rc = plan_job(ctx, &t->oj.job, t->plan, t->layout);
  if (rc) return rc;
  t->need_bytes = t->layout.total;
  rc = serve_start(ctx);
  if (rc) return rc;
  ServeState& S = *ctx->serve.load();
  {
    std::lock_guard<std::mutex> g(S.mu);
    if (S.queue.size() >= kMaxQueue) return PS_E_QUEUE_FULL;
    t->id = S.next_id++;
    S.tickets[t->id] = t;
    S.queue.push_back(t);
    *ticket = t->id;
  }
  S.cv_work.notify_all();
  return PS_OK;
}

int32_t ps_wait(ps_ctx* ctx, uint64_t ticket, int64_t timeout_us, ps_job_stats* st) {
  if (!ctx) return PS_E_INVALID;
  ServeState* sp = ctx->serve.load();
  if (!sp) return PS_E_NOT_FOUND;
  ServeState& S = *sp;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.tickets.find(ticket);
  if (it == S.tickets.end()) return PS_E_NOT_FOUND;
  auto t = it->second;
  auto pred = [&] { return t->done; };
  if (timeout_us < 0)
    S.cv_done.wait(lk, pred);
  else if (!S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
    return PS_E_TIMEOUT;
  if (st) *st = t->stats;
  int32_t rc = t->status;
  S.tickets.erase(it);
  return rc;
}

}  // extern "C"
