// Context and per-job device slots (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/psint.h"
#include "plan.h"
#include "ranges.h"

namespace psint {

// Device layout of one planned job: tables, then arrays, workspace and the FP64 output buffer.
struct Layout {
  size_t grids, lines, shells, ments, wcols, segs, ssegs, smembers, tasks, tiles, reds, ints, items, status;
  size_t meta_end;
  size_t arrays, ws, out;
  size_t total;
  std::vector<int32_t> items_host;  // reduce item ids, concatenated per (pass, phase)
};

// Device resources of one in-flight job: stream, arena (tables + arrays + workspace + outputs),
// pinned staging for its tables, and timing events.
struct Slot {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* arena = nullptr;
  size_t arena_size = 0;
  void* pinned = nullptr;
  size_t pinned_size = 0;
  hipEvent_t ev_start = nullptr, ev_kernels_done = nullptr, ev_end = nullptr;
  // overlapped passes: the next pass's evaluation runs on `side`, forked from and joined back to
  // `stream` around each contraction segment (created with the first such job)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> ev_contract;
  int n_contract = 0;
  bool want_chol = false;
  // the plan last staged on this slot, reused when the same job comes again (ps_compute)
  std::vector<char> plan_inputs;  // serialised job inputs + tiling + budget; empty = no valid plan
  Plan plan;
  Layout layout;
  // device work of that plan captured once it repeats, replayed segment by segment as graph launches
  std::vector<hipGraphExec_t> graphs;  // one per segment of the job's device work
  bool graph_failed = false;       // capture not possible on this stream: stay with stream launches
};

struct ServeState;

// A context's device memory: chunks from hipMalloc kept until ps_destroy, handed out as ranges
// (slot arenas).  Device memory that has been freed is cleared by the driver before it can be
// mapped again, so a large hipFree followed by hipMalloc costs seconds (about 6 s for 160-200 GB
// on MI355X); a range taken from a kept chunk costs nothing.  The sum of the chunks stays within
// the context's budget.
struct DevicePool {
  struct Chunk {
    char* base = nullptr;
    RangeMap ranges;
  };
  std::mutex mu;
  std::vector<Chunk> chunks;
  size_t total = 0;
};

}  // namespace psint

struct ps_ctx {
  int device = 0;
  size_t budget = 0;
  hipStream_t user_stream = nullptr;
  std::string err;     // last error text: written through set_err, read by ps_last_error (err_mu)
  std::mutex err_mu;
  psint::TileShape shape;
  bool shape_explicit = false;  // false: the default shape of the job's precision
  int ksplit = 0;
  int share_third = -1;  // PS_OPT_SHARE_THIRD_CENTRE: -1 automatic (FP64 jobs), 0 off, 1 on
  int overlap_passes = 0;  // PS_OPT_OVERLAP_PASSES: 0 off (the default, also set by -1), 1 on
  psint::Slot sync_slot;
  std::mutex sync_mu;  // held while ps_compute / ps_autotune use sync_slot; the serving dispatcher
                       // takes an idle sync_slot's arena back when a queued job needs the memory
  std::atomic<size_t> sync_arena_bytes{0};  // sync_slot.arena_size as last published under sync_mu
  std::atomic<psint::ServeState*> serve{nullptr};  // created by the first ps_submit (under
  std::mutex serve_init_mu;                       // serve_init_mu), freed by ps_destroy
  psint::DevicePool pool;              // slot arenas
};

namespace psint {

struct Layout;
int32_t slot_init(ps_ctx* ctx, Slot& s, hipStream_t stream);
void slot_free(ps_ctx* ctx, Slot& s);
void serve_shutdown(ps_ctx* ctx);
// A range of at least `bytes` from the context's pool (nullptr: no room within the budget, even after
// giving back chunks that hold no range).  Ranges are 2 MiB multiples; `*got` receives the size.
void* pool_alloc(ps_ctx* ctx, size_t bytes, size_t* got);
void pool_release(ps_ctx* ctx, void* p, size_t bytes);
void pool_destroy(ps_ctx* ctx);
// Looks up the allocation-free RI entry point's static scratch address on `device` (current).
int32_t ri_noalloc_init(int device);
// Records the context's last error text (serving and synchronous calls may overlap).
void set_err(ps_ctx* ctx, const std::string& msg);
// Synchronous calls that find no room in the pool: the ranges kept by idle serving slots go back to
// it.  Called with sync_mu held (the serving dispatcher only try-locks sync_mu).
void release_idle_serve_arenas(ps_ctx* ctx);

}  // namespace psint
