// C ABI of the library (include/psint.h): contexts, synchronous jobs, inspection hooks.  The
// serving entry points (ps_submit / ps_wait) live in serve.cpp.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "jobs.h"

namespace psint {

hipError_t launch_eval_shared(bool fp32, const ShareSegDev* segs, int nseg, int64_t nblocks, const GridDev* grids,
                              const double* lines, const ShellDev* shells, const MEntry* ments, hipStream_t st);
hipError_t launch_eval(bool fp32, const SegDev* segs, int nseg, int64_t nblocks, const GridDev* grids,
                       const double* lines, const ShellDev* shells, const MEntry* ments, const WColDev* wcols,
                       hipStream_t st);
hipError_t launch_contract_f64(int wm, int wn, int sc, int wr, const TaskDev* tasks, const TileDev* tiles,
                               int ntiles, double* ws, hipStream_t st);
hipError_t launch_contract_mixed(int wm, int wn, int sc, int wr, const TaskDev* tasks, const TileDev* tiles,
                                 int ntiles, double* ws, hipStream_t st);
hipError_t launch_reduce(const TaskDev* tasks, const RedDev* reds, const int32_t* items, int nitems,
                         const double* ws, hipStream_t st);
int contract_resident_workgroups(bool mixed, int wm, int wn, int sc, int wr);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_mfma_rate(bool fp64, int blocks, int iters, double* out, hipStream_t st);
hipError_t launch_symmetrize(double* X, int n, hipStream_t st);
hipError_t launch_cholesky(const double* A, double* L, int n, int* status, hipStream_t st);

// Offset, within the 64-byte status slot of the staged tables, at which the host receives the
// device's status word after a job (the slot's first half is staged to the device, zeroed).
constexpr size_t kStatusReadback = 32;
hipError_t launch_grid_points(const GridDev& G, const double* lines, const double* RA, double* xyzw, hipStream_t st);
hipError_t launch_eval_points(int what, const ShellDev& sh, const MEntry& me, const double* c, const double* X,
                              const double* Y, const double* Z, int64_t n, double* out, hipStream_t st);

namespace {
double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}
constexpr double kPi = 3.141592653589793238462643383279502884;
}  // namespace

#define HIP_TRY(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_err(ctx, std::string(#call) + ": " + hipGetErrorString(e_));                       \
      return PS_E_DEVICE;                                                                    \
    }                                                                                        \
  } while (0)

int32_t ensure_pinned(ps_ctx* ctx, Slot& s, size_t bytes) {
  if (s.pinned_size >= bytes) return PS_OK;
  if (s.pinned) (void)hipHostFree(s.pinned);
  s.pinned = nullptr;
  s.pinned_size = 0;
  size_t want = bytes + bytes / 4 + 4096;
  HIP_TRY(hipHostMalloc(&s.pinned, want, hipHostMallocDefault));
  s.pinned_size = want;
  return PS_OK;
}

void* pool_alloc(ps_ctx* ctx, size_t bytes, size_t* got) {
  constexpr size_t kGran = (size_t)2 << 20;
  bytes = (bytes + kGran - 1) / kGran * kGran;
  DevicePool& P = ctx->pool;
  std::lock_guard<std::mutex> g(P.mu);
  auto take = [&](DevicePool::Chunk& c) -> void* {
    size_t off = 0;
    if (!c.ranges.take(bytes, &off)) return nullptr;
    *got = bytes;
    return c.base + off;
  };
  for (auto& c : P.chunks)
    if (void* p = take(c)) return p;
  // a new chunk: a large request (a quarter of the budget or more) takes everything the budget has
  // left, so that later arenas of any size fit without another allocation
  auto add_chunk = [&](size_t size) -> void* {
    DevicePool::Chunk c;
    if (hipMalloc((void**)&c.base, size) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    c.ranges = RangeMap(size);
    P.total += size;
    P.chunks.push_back(c);
    return take(P.chunks.back());
  };
  auto room = [&]() { return ctx->budget > P.total ? (ctx->budget - P.total) / kGran * kGran : (size_t)0; };
  auto size_for = [&]() { return bytes >= ctx->budget / 4 ? std::max(bytes, room()) : bytes; };
  // (the larger chunk may not be there to take, e.g. held by another context: then the exact size)
  auto add = [&]() -> void* {
    void* p = add_chunk(size_for());
    return p || size_for() == bytes ? p : add_chunk(bytes);
  };
  if (bytes <= room())
    if (void* p = add()) return p;
  // give back chunks without ranges in use (their memory is cleared by the driver before reuse)
  for (size_t i = 0; i < P.chunks.size();) {
    auto& c = P.chunks[i];
    if (c.ranges.unused()) {
      (void)hipFree(c.base);
      P.total -= c.ranges.size();
      P.chunks.erase(P.chunks.begin() + i);
    } else {
      ++i;
    }
  }
  if (bytes <= room()) return add();
  return nullptr;
}

void pool_release(ps_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  DevicePool& P = ctx->pool;
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& c : P.chunks) {
    if ((char*)p < c.base || (char*)p >= c.base + c.ranges.size()) continue;
    c.ranges.give((size_t)((char*)p - c.base), bytes);
    return;
  }
}

void pool_destroy(ps_ctx* ctx) {
  DevicePool& P = ctx->pool;
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& c : P.chunks) (void)hipFree(c.base);
  P.chunks.clear();
  P.total = 0;
}

void set_err(ps_ctx* ctx, const std::string& msg) {
  std::lock_guard<std::mutex> g(ctx->err_mu);
  ctx->err = msg;
}

int32_t ensure_arena(ps_ctx* ctx, Slot& s, size_t bytes) {
  if (s.arena_size >= bytes) return PS_OK;
  if (s.arena) {
    HIP_TRY(hipStreamSynchronize(s.stream));
    pool_release(ctx, s.arena, s.arena_size);
  }
  s.arena = nullptr;
  s.arena_size = 0;
  size_t got = 0;
  void* p = pool_alloc(ctx, bytes, &got);
  if (!p && &s == &ctx->sync_slot) {
    // the synchronous slot (caller holds sync_mu): idle serving slots give their ranges back
    release_idle_serve_arenas(ctx);
    p = pool_alloc(ctx, bytes, &got);
  }
  if (!p) {
    char buf[160];
    snprintf(buf, sizeof buf, "no device memory for a %.2f GB arena within the %.2f GB budget", bytes / 1e9,
             ctx->budget / 1e9);
    set_err(ctx, buf);
    return PS_E_NOMEM;
  }
  s.arena = p;
  s.arena_size = got;
  return PS_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void compute_layout(const Plan& p, Layout& L) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  L.items_host.clear();
  for (auto& ps : p.passes)
    for (auto& v : ps.red_by_phase) L.items_host.insert(L.items_host.end(), v.begin(), v.end());
  L.grids = take(p.grids.size() * sizeof(GridDev));
  L.lines = take(p.lines.size() * sizeof(double));
  L.shells = take(p.shells.size() * sizeof(ShellDev));
  L.ments = take(p.ments.size() * sizeof(MEntry));
  L.wcols = take(p.wcols.size() * sizeof(WColDev));
  L.segs = take(p.segs.size() * sizeof(SegDev));
  L.ssegs = take(p.ssegs.size() * sizeof(ShareSegDev));
  size_t nmem = 0;
  for (int h : p.ssegs) nmem += p.shares[h].grids.size();
  L.smembers = take(nmem * sizeof(ShareMember));
  L.tasks = take(p.tasks.size() * sizeof(TaskDev));
  L.tiles = take(p.tiles.size() * sizeof(TileDev));
  L.reds = take(p.reds.size() * sizeof(RedDev));
  L.ints = take(p.ints.size() * sizeof(int32_t));
  L.items = take(L.items_host.size() * sizeof(int32_t));
  L.status = take(64);
  L.meta_end = o;
  L.arrays = take(p.max_array_bytes);  // each pass's region: its arrays, then its partial tiles
  L.ws = L.arrays;
  L.out = take((size_t)p.out_elems * sizeof(double));
  L.total = o;
}

// Fill the pinned staging buffer with the job's tables, pointers bound to the arena at `base`.
static void stage_meta(const Plan& p, const Layout& L, char* base, char* host) {
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(host + off, src, bytes);
  };
  std::vector<GridDev> grids(p.grids.size());
  for (size_t i = 0; i < p.grids.size(); ++i) grids[i] = p.grids[i].dev;
  put(L.grids, grids.data(), grids.size() * sizeof(GridDev));
  put(L.lines, p.lines.data(), p.lines.size() * sizeof(double));
  put(L.shells, p.shells.data(), p.shells.size() * sizeof(ShellDev));
  put(L.ments, p.ments.data(), p.ments.size() * sizeof(MEntry));
  put(L.wcols, p.wcols.data(), p.wcols.size() * sizeof(WColDev));
  std::vector<SegDev> segs(p.segs.size());
  for (size_t i = 0; i < p.segs.size(); ++i) {
    segs[i] = p.segs[i].dev;
    auto at = [&](int a) -> void* { return a >= 0 ? base + L.arrays + p.arrays[a].offset : nullptr; };
    segs[i].arr0 = at(p.segs[i].arr0);
    segs[i].arr1 = at(p.segs[i].arr1);
    segs[i].arr0d = at(p.segs[i].arr0d);
    segs[i].arr1d = at(p.segs[i].arr1d);
  }
  put(L.segs, segs.data(), segs.size() * sizeof(SegDev));
  {
    std::vector<ShareSegDev> ss;
    std::vector<ShareMember> mem;
    auto at = [&](int a) -> void* { return a >= 0 ? base + L.arrays + p.arrays[a].offset : nullptr; };
    for (int h : p.ssegs) {
      const ShareHost& sh = p.shares[h];
      ShareSegDev d = sh.dev;
      d.members = (const ShareMember*)(base + L.smembers) + mem.size();
      d.cells = (const int32_t*)(base + L.ints) + sh.cells_off;
      for (size_t c = 0; c < sh.grids.size(); ++c) {
        ShareMember m;
        m.arr0 = at(sh.arr0[c]);
        m.arr0d = at(sh.arr0d[c]);
        m.grid = sh.grids[c];
        m.pad0 = 0;
        mem.push_back(m);
      }
      ss.push_back(d);
    }
    put(L.ssegs, ss.data(), ss.size() * sizeof(ShareSegDev));
    put(L.smembers, mem.data(), mem.size() * sizeof(ShareMember));
  }
  const int32_t* ints_dev = (const int32_t*)(base + L.ints);
  double* out_dev = (double*)(base + L.out);
  std::vector<TaskDev> tasks(p.tasks.size());
  for (size_t i = 0; i < p.tasks.size(); ++i) {
    const TaskHost& th = p.tasks[i];
    TaskDev d = th.dev;
    d.U = base + L.arrays + p.arrays[th.U].offset;
    d.V = base + L.arrays + p.arrays[th.V].offset;
    d.Y = base + L.arrays + p.arrays[th.Y].offset;
    d.nfU = p.arrays[th.U].nf;
    d.nfV = p.arrays[th.V].nf;
    d.nfY = p.arrays[th.Y].nf;
    d.nchunks = p.grids[th.grid].dev.npad / KC;
    d.pairs = ints_dev + th.pairs_off;
    d.mapU = ints_dev + reinterpret_cast<intptr_t>(th.dev.mapU);
    d.mapV = ints_dev + reinterpret_cast<intptr_t>(th.dev.mapV);
    d.mapY = ints_dev + reinterpret_cast<intptr_t>(th.dev.mapY);
    d.out = out_dev + th.out_off;
    d.outm = th.outm_off >= 0 ? out_dev + th.outm_off : nullptr;
    tasks[i] = d;
  }
  put(L.tasks, tasks.data(), tasks.size() * sizeof(TaskDev));
  put(L.tiles, p.tiles.data(), p.tiles.size() * sizeof(TileDev));
  put(L.reds, p.reds.data(), p.reds.size() * sizeof(RedDev));
  put(L.ints, p.ints.data(), p.ints.size() * sizeof(int32_t));
  put(L.items, L.items_host.data(), L.items_host.size() * sizeof(int32_t));
  std::memset(host + L.status, 0, 64);
}

// The device work of a planned job in segments: 0 = table copy, output clear and the evaluation of
// pass 0; 2i + 1 = the contraction launches of pass i; 2i + 2 = the reductions of pass i, then the
// evaluation of pass i + 1, or after the last pass the symmetrisation and the Cholesky factorisation.
// With overlapped passes the evaluation of pass i + 1 moves into segment 2i + 1: forked onto the
// slot's side stream before the contraction launches (its region is not the one they read) and joined
// back after them, so every segment still ends with all of its work ordered on the slot's stream.
int num_segments(const Plan& p) { return 2 * (int)p.passes.size() + 1; }

int32_t ensure_side(ps_ctx* ctx, Slot& s) {
  if (!s.side) HIP_TRY(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking));
  if (!s.ev_fork) HIP_TRY(hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming));
  if (!s.ev_join) HIP_TRY(hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming));
  return PS_OK;
}

int32_t enqueue_segment(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, int k) {
  (void)ctx;
  char* base = (char*)s.arena;
  const hipStream_t st = s.stream;
  double* out = (double*)(base + L.out);
  const GridDev* grids = (const GridDev*)(base + L.grids);
  const double* lines = (const double*)(base + L.lines);
  const SegDev* segs = (const SegDev*)(base + L.segs);
  const TaskDev* tasks = (const TaskDev*)(base + L.tasks);
  const TileDev* tiles = (const TileDev*)(base + L.tiles);
  const RedDev* reds = (const RedDev*)(base + L.reds);
  const int32_t* items = (const int32_t*)(base + L.items);
  const bool mixed = p.precision == PS_PREC_MIXED;
  auto eval = [&](const Pass& ps, hipStream_t es) {
    hipError_t e = launch_eval(mixed, segs + ps.seg0, ps.seg1 - ps.seg0, ps.eval_blocks, grids, lines,
                               (const ShellDev*)(base + L.shells), (const MEntry*)(base + L.ments),
                               (const WColDev*)(base + L.wcols), es);
    if (e != hipSuccess) return e;
    return launch_eval_shared(mixed, (const ShareSegDev*)(base + L.ssegs) + ps.sseg0, ps.sseg1 - ps.sseg0,
                              ps.shared_blocks, grids, lines, (const ShellDev*)(base + L.shells),
                              (const MEntry*)(base + L.ments), es);
  };
  if (k == 0) {
    HIP_TRY(hipMemcpyAsync(base, s.pinned, L.meta_end, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_fill(out, p.out_elems, 0.0, st));
    if (!p.passes.empty()) HIP_TRY(eval(p.passes[0], st));
    return PS_OK;
  }
  const int pi = (k - 1) / 2;
  const Pass& ps = p.passes[pi];
  double* ws = (double*)(base + L.arrays + ps.ws_offset);
  const bool fork = p.overlap && k % 2 == 1 && pi + 1 < (int)p.passes.size();
  if (fork) {
    if (!s.side) return PS_E_DEVICE;  // ensure_side comes first
    HIP_TRY(hipEventRecord(s.ev_fork, st));
    HIP_TRY(hipStreamWaitEvent(s.side, s.ev_fork, 0));
    HIP_TRY(eval(p.passes[pi + 1], s.side));
    HIP_TRY(hipEventRecord(s.ev_join, s.side));
  }
  if (k % 2 == 1) {
    // one launch per tile shape: (ab|P) tiles, 64 x 64 tiles, narrow last-column tiles
    for (const auto& lc : ps.launches) {
      const int n = lc.tile1 - lc.tile0;
      if (n <= 0) continue;
      const TileShape& sh = lc.shape;
      if (mixed && !lc.f64)
        HIP_TRY(launch_contract_mixed(sh.wm, sh.wn, sh.sc, sh.wr, tasks, tiles + lc.tile0, n, ws, st));
      else
        HIP_TRY(launch_contract_f64(sh.wm, sh.wn, sh.sc, sh.wr, tasks, tiles + lc.tile0, n, ws, st));
    }
    if (fork) HIP_TRY(hipStreamWaitEvent(st, s.ev_join, 0));
    return PS_OK;
  }
  size_t item_pos = 0;
  for (int q = 0; q < pi; ++q)
    for (auto& ph : p.passes[q].red_by_phase) item_pos += ph.size();
  for (auto& ph : ps.red_by_phase) {
    HIP_TRY(launch_reduce(tasks, reds, items + item_pos, (int)ph.size(), ws, st));
    item_pos += ph.size();
  }
  if (pi + 1 < (int)p.passes.size()) {
    if (p.overlap) return PS_OK;  // evaluated during this pass's contraction
    return eval(p.passes[pi + 1], st) == hipSuccess ? PS_OK : PS_E_DEVICE;
  }
  const int nb = p.n_bf, na = p.n_aux;
  HIP_TRY(launch_symmetrize(out + p.off_S, nb, st));
  HIP_TRY(launch_symmetrize(out + p.off_T, nb, st));
  HIP_TRY(launch_symmetrize(out + p.off_V, nb, st));
  HIP_TRY(launch_symmetrize(out + p.off_PQ, na, st));
  if (s.want_chol && na > 0)
    HIP_TRY(launch_cholesky(out + p.off_PQ, out + p.off_L, na, (int*)(base + L.status), st));
  return PS_OK;
}

// Enqueue every step of a planned job on slot s (no synchronisation), each segment either launched
// directly or, when `graphs` holds one executable per segment, as that segment's graph.  The events
// that time the job and its contraction launches are recorded on the stream between segments (outside
// any graph), so they are measured afresh on every run.
int32_t enqueue_job(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, const std::vector<hipGraphExec_t>* graphs) {
  hipStream_t st = s.stream;
  if (p.overlap && !graphs) {
    int32_t rc = ensure_side(ctx, s);
    if (rc) return rc;
  }
  while (s.ev_contract.size() < 2 * p.passes.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    s.ev_contract.push_back(e);
  }
  HIP_TRY(hipEventRecord(s.ev_start, st));
  s.n_contract = 0;
  const int nseg = num_segments(p);
  for (int k = 0; k < nseg; ++k) {
    if (k % 2 == 1) HIP_TRY(hipEventRecord(s.ev_contract[k - 1], st));
    if (graphs) {
      HIP_TRY(hipGraphLaunch((*graphs)[k], st));
    } else {
      int32_t rc = enqueue_segment(ctx, s, p, L, k);
      if (rc) return rc;
    }
    if (k % 2 == 1) {
      HIP_TRY(hipEventRecord(s.ev_contract[k], st));
      s.n_contract++;
    }
  }
  HIP_TRY(hipEventRecord(s.ev_kernels_done, st));
  return PS_OK;
}

size_t output_bytes(const Plan& p, const ps_job& job) {
  const size_t nb2 = (size_t)p.n_bf * p.n_bf * 8, na2 = (size_t)p.n_aux * p.n_aux * 8;
  size_t b = 0;
  if (job.S) b += nb2;
  if (job.T) b += nb2;
  if (job.V) b += nb2;
  if (job.PQ) b += na2;
  if (job.PQ_chol) b += na2;
  if (job.abP) b += (size_t)p.n_aux * nb2;
  return b;
}

// Copy the requested outputs to the caller's buffers (enqueued on the slot's stream).  With a host
// bounce buffer (pinned), host outputs land there first, packed in S, T, V, PQ, PQ_chol, abP order.
int32_t enqueue_outputs(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, const ps_job& job, char* host_bounce) {
  char* base = (char*)s.arena;
  const double* out = (const double*)(base + L.out);
  const bool dev = job.out_location == PS_OUT_DEVICE;
  hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const size_t nb2 = (size_t)p.n_bf * p.n_bf * 8, na2 = (size_t)p.n_aux * p.n_aux * 8;
  struct {
    double* dst;
    int64_t off;
    size_t bytes;
  } outs[6] = {{job.S, p.off_S, nb2},   {job.T, p.off_T, nb2},     {job.V, p.off_V, nb2},
               {job.PQ, p.off_PQ, na2}, {job.PQ_chol, p.off_L, na2}, {job.abP, p.off_abP, (size_t)p.n_aux * nb2}};
  size_t bo = 0;
  for (auto& o : outs) {
    if (!o.dst || !o.bytes) continue;
    void* dst = (!dev && host_bounce) ? (void*)(host_bounce + bo) : (void*)o.dst;
    HIP_TRY(hipMemcpyAsync(dst, out + o.off, o.bytes, kind, s.stream));
    bo += o.bytes;
  }
  // The status word is read back into the second half of its 64-byte staging slot: the first half is
  // part of the tables the next run of the same job copies to the device, and must stay zero.
  HIP_TRY(hipMemcpyAsync((char*)s.pinned + L.status + kStatusReadback, base + L.status, sizeof(int),
                         hipMemcpyDeviceToHost, s.stream));
  HIP_TRY(hipEventRecord(s.ev_end, s.stream));
  return PS_OK;
}

int32_t bind_slot(ps_ctx* ctx, Slot& s, const Plan& plan, const Layout& L, size_t extra_pinned, bool want_chol) {
  int32_t rc = ensure_arena(ctx, s, L.total);
  if (rc) return rc;
  rc = ensure_pinned(ctx, s, L.meta_end + extra_pinned);
  if (rc) return rc;
  s.want_chol = want_chol;
  stage_meta(plan, L, (char*)s.arena, (char*)s.pinned);
  return PS_OK;
}

TileShape effective_shape(const ps_ctx* ctx, int32_t precision) {
  TileShape t;  // FP64: 128 x 128 tiles, 16-point stages (two work-groups per CU)
  if (ctx && ctx->shape_explicit) {
    t = ctx->shape;
  } else if (precision == PS_PREC_MIXED) {
    // FP32 operands: 128 x 128 tiles with 32-point stages (the FP32 stage sums of one row block at a
    // time beside the FP64 accumulators fit two waves per SIMD)
    t.sc = 2;
  }
  // resident work-groups of this shape on the context's device: the planner rounds the K splits
  // to whole waves of them (host-only planning without a context leaves 0: no rounding)
  t.slots = t.slots2 = 0;
  if (ctx) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int>, int> cache;
    const bool mixed = precision == PS_PREC_MIXED;
    auto resident_of = [&](bool mx, int wm, int wn, int sc, int wr) {
      const auto key = std::make_tuple(ctx->device, (int)mx, wm, wn, sc, wr);
      auto it = cache.find(key);
      if (it == cache.end()) it = cache.emplace(key, contract_resident_workgroups(mx, wm, wn, sc, wr)).first;
      return it->second;
    };
    auto resident = [&](int wm, int wn, int sc, int wr = 2) { return resident_of(mixed, wm, wn, sc, wr); };
    std::lock_guard<std::mutex> g(mu);
    t.slots = resident(t.wm, t.wn, t.sc, t.wr);
    t.slots2 = resident(2, 2, t.sc);
    for (int w = 1; w < t.wn && w <= 3; ++w) t.slots_n[w] = resident(t.wm, w, t.sc);
    t.slots2n = resident(2, 1, t.sc);
    for (int w = 1; w <= 4; ++w) t.slots_short[w] = resident(1, w, t.sc);
    for (int k = 0; k < 4; ++k) t.slots_tall[k] = resident(2, 2 * k + 1, t.sc, 4);
    if (mixed) {  // the FP64 two-index launches of a mixed job
      t.slots2_f64 = resident_of(false, 2, 2, t.sc, 2);
      t.slots2n_f64 = resident_of(false, 2, 1, t.sc, 2);
      for (int w = 1; w <= 2; ++w) t.slots_short_f64[w] = resident_of(false, 1, w, t.sc, 2);
    }
  }
  return t;
}

// Cross-third-centre reuse for a job: the context's choice, or automatically for FP64 jobs (measured
// on the hydrocarbon job: FP64 0.3% faster with it, mixed 0.2% slower).
bool share_third_for(const ps_ctx* ctx, int32_t precision) {
  return ctx->share_third < 0 ? precision == PS_PREC_FP64 : ctx->share_third != 0;
}

bool overlap_passes_for(const ps_ctx* ctx) { return ctx->overlap_passes == 1; }

int32_t plan_job(ps_ctx* ctx, const ps_job* job, Plan& plan, Layout& L) {
  std::string err;
  const TileShape shape = effective_shape(ctx, job->precision);
  const bool share = share_third_for(ctx, job->precision);
  int32_t rc = build_plan(job, shape, ctx->ksplit, ctx->budget, &plan, &err, share, overlap_passes_for(ctx));
  if (rc) {
    set_err(ctx, err);
    return rc;
  }
  compute_layout(plan, L);
  if (plan.overlap && L.total > ctx->budget) {
    // two regions did not fit after all: one region, passes in series
    rc = build_plan(job, shape, ctx->ksplit, ctx->budget, &plan, &err, share, false);
    if (rc) {
      set_err(ctx, err);
      return rc;
    }
    compute_layout(plan, L);
  }
  if (L.total > ctx->budget) {
    char buf[200];
    snprintf(buf, sizeof buf, "job needs %.2f GB of device memory, budget is %.2f GB", L.total / 1e9,
             ctx->budget / 1e9);
    set_err(ctx, buf);
    return PS_E_NOMEM;
  }
  return PS_OK;
}

void drop_graph(Slot& s) {
  for (auto g : s.graphs) (void)hipGraphExecDestroy(g);
  s.graphs.clear();
}

void release_sync_arena(ps_ctx* ctx) {
  Slot& s = ctx->sync_slot;
  if (!s.arena) return;
  (void)hipStreamSynchronize(s.stream);
  pool_release(ctx, s.arena, s.arena_size);
  s.arena = nullptr;
  s.arena_size = 0;
  s.plan_inputs.clear();
  drop_graph(s);
  ctx->sync_arena_bytes.store(0);
}

int32_t prepare_slot(ps_ctx* ctx, Slot& s, const ps_job* job, Plan& plan, Layout& L) {
  s.plan_inputs.clear();  // the slot's staged tables change
  drop_graph(s);
  int32_t rc = plan_job(ctx, job, plan, L);
  if (rc) return rc;
  return bind_slot(ctx, s, plan, L, 0, job->PQ_chol != nullptr);
}

int32_t finish_stats(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, ps_job_stats* st, double total_ms,
                     double queue_ms) {
  int status = *(int*)((char*)s.pinned + L.status + kStatusReadback);
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->n_grids = (int64_t)p.grids.size();
    st->n_points = p.n_points;
    st->pair_points = p.pair_points;
    st->contract_flops = p.contract_flops;
    st->issued_flops = p.issued_flops;
    st->n_passes = (int64_t)p.passes.size();
    st->passes_overlapped = p.overlap ? 1 : 0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, s.ev_start, s.ev_kernels_done) == hipSuccess) st->device_ms = ms;
    double cms = 0.0;
    for (int i = 0; i < s.n_contract; ++i) {
      float m2 = 0.0f;
      if (hipEventElapsedTime(&m2, s.ev_contract[2 * i], s.ev_contract[2 * i + 1]) == hipSuccess) cms += m2;
    }
    st->contract_ms = cms;
    st->total_ms = total_ms;
    st->queue_ms = queue_ms;
  }
  if (s.want_chol && status) {
    set_err(ctx, "(P|Q) is not positive definite");
    return PS_E_NOT_PD;
  }
  return PS_OK;
}

int32_t slot_init(ps_ctx* ctx, Slot& s, hipStream_t stream) {
  s.own_stream = stream == nullptr;
  if (s.own_stream) {
    HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  } else {
    s.stream = stream;
  }
  HIP_TRY(hipEventCreate(&s.ev_start));
  HIP_TRY(hipEventCreate(&s.ev_kernels_done));
  HIP_TRY(hipEventCreate(&s.ev_end));
  return PS_OK;
}

void slot_free(ps_ctx* ctx, Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  if (s.arena) pool_release(ctx, s.arena, s.arena_size);
  if (s.pinned) (void)hipHostFree(s.pinned);
  drop_graph(s);
  for (auto e : s.ev_contract) (void)hipEventDestroy(e);
  if (s.ev_start) (void)hipEventDestroy(s.ev_start);
  if (s.ev_kernels_done) (void)hipEventDestroy(s.ev_kernels_done);
  if (s.ev_end) (void)hipEventDestroy(s.ev_end);
  if (s.side) {
    (void)hipStreamSynchronize(s.side);
    (void)hipStreamDestroy(s.side);
  }
  if (s.ev_fork) (void)hipEventDestroy(s.ev_fork);
  if (s.ev_join) (void)hipEventDestroy(s.ev_join);
  if (s.own_stream && s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

}  // namespace psint

using namespace psint;

extern "C" {

const char* ps_status_string(int32_t status) {
  switch (status) {
    case PS_OK: return "ok";
    case PS_E_INVALID: return "invalid input";
    case PS_E_UNSUPPORTED: return "unsupported input";
    case PS_E_NOMEM: return "job exceeds the device-memory budget";
    case PS_E_DEVICE: return "device error";
    case PS_E_NOT_PD: return "(P|Q) not positive definite";
    case PS_E_TIMEOUT: return "timeout";
    case PS_E_QUEUE_FULL: return "queue full";
    case PS_E_NOT_FOUND: return "unknown ticket";
    default: return "unknown status";
  }
}

const char* ps_last_error(ps_ctx* ctx) {
  // a copy per calling thread, taken under the context's lock: the text stays valid until this
  // thread's next ps_last_error call, whatever other threads do on the context meanwhile
  static thread_local std::string copy;
  if (!ctx) {
    copy.clear();
    return copy.c_str();
  }
  std::lock_guard<std::mutex> g(ctx->err_mu);
  copy = ctx->err;
  return copy.c_str();
}

int32_t ps_create(int32_t hip_device, size_t hbm_budget_bytes, void* stream, ps_ctx** out) {
  if (!out) return PS_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return PS_E_DEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return PS_E_DEVICE;
  ps_ctx* ctx = new ps_ctx();
  ctx->device = hip_device;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete ctx;
    return PS_E_DEVICE;
  }
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)fr);
  ctx->user_stream = (hipStream_t)stream;
  int32_t rc = slot_init(ctx, ctx->sync_slot, (hipStream_t)stream);
  if (rc) {
    delete ctx;
    return rc;
  }
  // set-up of the allocation-free RI entry point on this device (it retries on its first call)
  (void)ri_noalloc_init(hip_device);
  *out = ctx;
  return PS_OK;
}

int32_t ps_destroy(ps_ctx* ctx) {
  if (!ctx) return PS_E_INVALID;
  serve_shutdown(ctx);
  (void)hipSetDevice(ctx->device);
  slot_free(ctx, ctx->sync_slot);
  pool_destroy(ctx);
  delete ctx;
  return PS_OK;
}

int32_t ps_mfma_rate(ps_ctx* ctx, int32_t precision, double* tflops) {
  if (!ctx) return PS_E_INVALID;
  if (!tflops || (precision != PS_PREC_FP64 && precision != PS_PREC_MIXED)) {
    set_err(ctx, "mfma_rate: tflops must be given, precision PS_PREC_FP64 or PS_PREC_MIXED");
    return PS_E_INVALID;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  std::lock_guard<std::mutex> sync_guard(ctx->sync_mu);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
  const int blocks = 4 * prop.multiProcessorCount;  // 16 waves per CU
  const int iters = 4000;
  const bool fp64 = precision == PS_PREC_FP64;
  size_t got = 0;
  double* out = (double*)pool_alloc(ctx, (size_t)blocks * 4 * sizeof(double), &got);
  if (!out) {
    set_err(ctx, "mfma_rate: no device memory for the probe's output");
    return PS_E_NOMEM;
  }
  hipStream_t st = ctx->sync_slot.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t rc = PS_OK;
  double best_ms = 0.0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = PS_E_DEVICE;
  for (int rep = 0; rep < 4 && rc == PS_OK; ++rep) {  // the first run is untimed
    if (hipEventRecord(e0, st) != hipSuccess || launch_mfma_rate(fp64, blocks, iters, out, st) != hipSuccess ||
        hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = PS_E_DEVICE;
      break;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PS_E_DEVICE;
    if (rep > 0 && (best_ms == 0.0 || ms < best_ms)) best_ms = ms;
  }
  if (rc != PS_OK) set_err(ctx, std::string("mfma_rate: ") + hipGetErrorString(hipGetLastError()));
  (void)hipStreamSynchronize(st);
  pool_release(ctx, out, got);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == PS_OK) *tflops = (double)blocks * 4 * iters * 8 * 2048.0 / (best_ms * 1e-3) / 1e12;
  return rc;
}

int32_t ps_set_option(ps_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return PS_E_INVALID;
  if (value == -1 || value == 0 || value == 1) {
    if (option == PS_OPT_SHARE_THIRD_CENTRE) {
      ctx->share_third = (int)value;
      return PS_OK;
    }
    if (option == PS_OPT_OVERLAP_PASSES) {
      ctx->overlap_passes = value == 1 ? 1 : 0;
      return PS_OK;
    }
  }
  set_err(ctx, "option: PS_OPT_SHARE_THIRD_CENTRE or PS_OPT_OVERLAP_PASSES with value -1, 0 or 1");
  return PS_E_INVALID;
}

int32_t ps_set_tiling(ps_ctx* ctx, int32_t wm, int32_t wn, int32_t stage_chunks, int32_t ksplit) {
  if (!ctx) return PS_E_INVALID;
  if (wm == 0 && wn == 0 && stage_chunks == 0) {
    if (ksplit < 0) {
      set_err(ctx, "tiling: ksplit >= 0");
      return PS_E_INVALID;
    }
    ctx->shape_explicit = false;  // the default shape of each job's precision
    ctx->shape = TileShape();
    ctx->ksplit = ksplit;
    return PS_OK;
  }
  TileShape def;
  if (wm == 0) wm = def.wm;
  if (wn == 0) wn = def.wn;
  if (stage_chunks == 0) stage_chunks = def.sc;
  if (!((wm == 2 || wm == 4) && (wn == 2 || wn == 4) && (stage_chunks == 1 || stage_chunks == 2)) || ksplit < 0) {
    set_err(ctx, "tiling: wm, wn in {2, 4}, stage_chunks in {1, 2}, ksplit >= 0");
    return PS_E_INVALID;
  }
  ctx->shape.wm = wm;
  ctx->shape.wn = wn;
  ctx->shape.sc = stage_chunks;
  ctx->shape_explicit = true;
  ctx->ksplit = ksplit;
  return PS_OK;
}

// Everything a plan depends on, serialised: the job's inputs, the tiling, the budget and whether
// the factor is wanted (output buffers and their placement are bound at enqueue time).
static std::vector<char> plan_inputs(const ps_ctx* ctx, const ps_job* job) {
  std::vector<char> v;
  auto put = [&](const void* p, size_t n) {
    if (n) v.insert(v.end(), (const char*)p, (const char*)p + n);
  };
  put(&job->n_atoms, sizeof job->n_atoms);
  put(&job->n_bf, sizeof job->n_bf);
  put(&job->n_aux, sizeof job->n_aux);
  put(&job->n_pair_grids, sizeof job->n_pair_grids);
  if (job->n_atoms > 0 && job->atoms) put(job->atoms, sizeof(ps_atom) * job->n_atoms);
  if (job->n_bf > 0 && job->basis) put(job->basis, sizeof(ps_sto) * job->n_bf);
  if (job->n_aux > 0 && job->aux) put(job->aux, sizeof(ps_sto) * job->n_aux);
  if (job->n_pair_grids > 0 && job->pair_grids) put(job->pair_grids, sizeof(ps_pair_grid) * job->n_pair_grids);
  put(&job->grid, sizeof job->grid);
  put(&job->precision, sizeof job->precision);
  const TileShape t = effective_shape(ctx, job->precision);
  const int tv[4] = {t.wm, t.wn, t.sc, ctx->ksplit};
  put(tv, sizeof tv);
  put(&ctx->budget, sizeof ctx->budget);
  const char chol = job->PQ_chol != nullptr, share = share_third_for(ctx, job->precision),
             overlap = overlap_passes_for(ctx);
  put(&chol, 1);
  put(&share, 1);
  put(&overlap, 1);
  return v;
}

int32_t ps_compute(ps_ctx* ctx, const ps_job* job, ps_job_stats* st) {
  if (!ctx || !job) return PS_E_INVALID;
  std::lock_guard<std::mutex> sync_guard(ctx->sync_mu);
  auto t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  Slot& s = ctx->sync_slot;
  // the same job again on this context: its plan and staged tables are still on the slot
  std::vector<char> key = plan_inputs(ctx, job);
  const bool repeat = !s.plan_inputs.empty() && s.plan_inputs == key;
  if (!repeat) {
    int32_t rc = prepare_slot(ctx, s, job, s.plan, s.layout);
    ctx->sync_arena_bytes.store(s.arena_size);
    if (rc) return rc;
    s.plan_inputs = std::move(key);
  }
  const Plan& plan = s.plan;
  const Layout& L = s.layout;
  int32_t rc = PS_OK;
  if (repeat && s.graphs.empty() && !s.graph_failed) {
    // second run of the same plan: capture each segment of its device work (kernels, the table copy;
    // no memset nodes) into a graph of its own, replayed from now on between the timing events
    if (plan.overlap) {
      rc = ensure_side(ctx, s);
      if (rc) return rc;
    }
    for (int k = 0; k < num_segments(plan) && !s.graph_failed; ++k) {
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        s.graph_failed = true;
        break;
      }
      rc = enqueue_segment(ctx, s, plan, L, k);
      hipError_t e = hipStreamEndCapture(s.stream, &g);
      if (rc == PS_OK && e == hipSuccess && g && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess)
        s.graphs.push_back(x);
      else
        s.graph_failed = true;
      if (g) (void)hipGraphDestroy(g);
      if (rc != PS_OK) {
        drop_graph(s);
        s.plan_inputs.clear();
        return rc;
      }
    }
    if (s.graph_failed) {
      drop_graph(s);
      (void)hipGetLastError();
    }
  }
  const bool replay = repeat && !s.graphs.empty();
  rc = enqueue_job(ctx, s, plan, L, replay ? &s.graphs : nullptr);
  if (rc) {
    s.plan_inputs.clear();
    return rc;
  }
  rc = enqueue_outputs(ctx, s, plan, L, *job);
  if (rc) {
    s.plan_inputs.clear();
    return rc;
  }
  HIP_TRY(hipStreamSynchronize(s.stream));
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  rc = finish_stats(ctx, s, plan, L, st, ms, 0.0);
  if (st) st->graph_replay = replay ? 1 : 0;
  return rc;
}

int32_t ps_plan_work(ps_ctx* ctx, const ps_job* job, double* pair_points, int64_t* n_grids, int64_t* n_points,
                     size_t* device_bytes) {
  // ctx may be NULL: host-only planning with the default tiling and an unbounded budget
  Plan plan;
  std::string err;
  if (!job) return PS_E_INVALID;
  TileShape shape = effective_shape(ctx, job->precision);
  int32_t rc = build_plan(job, shape, ctx ? ctx->ksplit : 0, ctx ? ctx->budget : ((size_t)1 << 62), &plan, &err);
  if (rc) {
    if (ctx) set_err(ctx, err);
    return rc;
  }
  Layout L;
  compute_layout(plan, L);
  if (pair_points) *pair_points = plan.pair_points;
  if (n_grids) *n_grids = (int64_t)plan.grids.size();
  if (n_points) *n_points = plan.n_points;
  if (device_bytes) *device_bytes = L.total;
  return PS_OK;
}

int32_t ps_grid_points(ps_ctx* ctx, const ps_atom* atoms, int32_t n_atoms, int32_t A, int32_t B, int32_t C,
                       const ps_grid_spec* spec, double* xyzw, int64_t* n_points) {
  if (!ctx || !atoms || !spec || !n_points) return PS_E_INVALID;
  GridHost g;
  std::string err;
  int32_t rc = build_grid(atoms, n_atoms, A, B, C, *spec, &g, &err);
  if (rc) {
    set_err(ctx, err);
    return rc;
  }
  *n_points = g.dev.npts;
  if (!xyzw) return PS_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  std::vector<double> lines;
  g.dev.lines = 0;
  lines.insert(lines.end(), g.mu.begin(), g.mu.end());
  lines.insert(lines.end(), g.nu.begin(), g.nu.end());
  lines.insert(lines.end(), g.phi.begin(), g.phi.end());
  g.dev.gl = (int)lines.size();
  double x[16], w[16];
  gauss_legendre(g.dev.q, x, w);
  lines.insert(lines.end(), x, x + g.dev.q);
  lines.insert(lines.end(), w, w + g.dev.q);
  double *dl = nullptr, *dp = nullptr;
  hipStream_t st = ctx->sync_slot.stream;
  HIP_TRY(hipMalloc(&dl, lines.size() * 8));
  hipError_t e = hipMalloc(&dp, (size_t)g.dev.npts * 4 * 8);
  if (e != hipSuccess) {
    (void)hipFree(dl);
    set_err(ctx, hipGetErrorString(e));
    return PS_E_DEVICE;
  }
  e = hipMemcpyAsync(dl, lines.data(), lines.size() * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_grid_points(g.dev, dl, atoms[A].xyz, dp, st);
  if (e == hipSuccess) e = hipMemcpyAsync(xyzw, dp, (size_t)g.dev.npts * 32, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dl);
  (void)hipFree(dp);
  if (e != hipSuccess) {
    set_err(ctx, hipGetErrorString(e));
    return PS_E_DEVICE;
  }
  return PS_OK;
}

int32_t ps_eval_function(ps_ctx* ctx, int32_t what, const ps_sto* fn, const double* center, int64_t npts,
                         const double* x, const double* y, const double* z, double* out) {
  if (!ctx || !fn || !center || (npts > 0 && (!x || !y || !z || !out)) || what < 0 || what > 2)
    return PS_E_INVALID;
  if (fn->n < 1 || fn->l < 0 || fn->l >= fn->n || fn->m < -fn->l || fn->m > fn->l || !(fn->zeta > 0.0))
    return PS_E_INVALID;
  if (fn->l > LMAX || fn->n > NMAX) return PS_E_UNSUPPORTED;
  if (npts == 0) return PS_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  ShellDev sh;
  sh.zeta = fn->zeta;
  sh.n = fn->n;
  sh.l = fn->l;
  sh.norm = std::pow(2.0 * fn->zeta, fn->n + 0.5) / std::sqrt(factorial(2 * fn->n));
  sh.pre = 4.0 * kPi / (2.0 * fn->l + 1.0) * sh.norm * std::pow(fn->zeta, -(fn->n + 1.0));
  sh.m_off = 0;
  sh.nm = 1;
  MEntry me;
  int am = std::abs(fn->m);
  me.f = std::sqrt((2.0 * fn->l + 1.0) / (4.0 * kPi) * factorial(fn->l - am) / factorial(fn->l + am)) *
         (am ? std::sqrt(2.0) : 1.0);
  me.m = fn->m;
  me.col = 0;
  double* d = nullptr;
  hipStream_t st = ctx->sync_slot.stream;
  HIP_TRY(hipMalloc(&d, (size_t)npts * 4 * 8));
  hipError_t e = hipMemcpyAsync(d, x, npts * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d + npts, y, npts * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d + 2 * npts, z, npts * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_eval_points(what, sh, me, center, d, d + npts, d + 2 * npts, npts, d + 3 * npts, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d + 3 * npts, npts * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  if (e != hipSuccess) {
    set_err(ctx, hipGetErrorString(e));
    return PS_E_DEVICE;
  }
  return PS_OK;
}

}  // extern "C"
