// Job preparation and enqueueing shared by the synchronous and serving paths (internal).
#pragma once
#include <cstdint>
#include <vector>

#include "ctx.h"

namespace psint {

void compute_layout(const Plan& p, Layout& L);
// The contraction tile shape for a job: the context's explicit choice, else the precision's default.
TileShape effective_shape(const ps_ctx* ctx, int32_t precision);
// Whether a job of this precision on this context uses cross-third-centre reuse.
bool share_third_for(const ps_ctx* ctx, int32_t precision);
// Whether jobs on this context that need several memory passes overlap them.
bool overlap_passes_for(const ps_ctx* ctx);
// The slot's side stream and fork/join events for overlapped passes (created once).
int32_t ensure_side(ps_ctx* ctx, Slot& s);
// Plan the job and size its device layout (PS_E_NOMEM beyond the budget).
int32_t plan_job(ps_ctx* ctx, const ps_job* job, Plan& plan, Layout& L);
// Size the slot's arena and pinned staging (plus `extra_pinned` bytes) and stage the tables.
int32_t bind_slot(ps_ctx* ctx, Slot& s, const Plan& plan, const Layout& L, size_t extra_pinned, bool want_chol);
// plan_job + bind_slot.
int32_t prepare_slot(ps_ctx* ctx, Slot& s, const ps_job* job, Plan& plan, Layout& L);
// Segments of a job's device work: table copy + evaluation, then per pass its contraction launches
// (odd segments) and its reductions + the next pass's evaluation or the final assembly (even).
int num_segments(const Plan& p);
int32_t enqueue_segment(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, int k);
// Enqueue all device work of a prepared job on the slot's stream, with the timing events between the
// segments; `graphs` (one executable per segment) replays captured segments instead of launching.
int32_t enqueue_job(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L,
                    const std::vector<hipGraphExec_t>* graphs = nullptr);
// Enqueue the output copies (to the caller's buffers, or to `host_bounce` for host outputs when
// non-null) and the end event.
int32_t enqueue_outputs(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, const ps_job& job,
                        char* host_bounce = nullptr);
// Fill the stats of a completed job and turn the Cholesky status into a return code.
int32_t finish_stats(ps_ctx* ctx, Slot& s, const Plan& p, const Layout& L, ps_job_stats* st, double total_ms,
                     double queue_ms);
int32_t ensure_pinned(ps_ctx* ctx, Slot& s, size_t bytes);
int32_t ensure_arena(ps_ctx* ctx, Slot& s, size_t bytes);
// Destroy the slot's captured graph (its kernels refer to the slot's current arena and tables).
void drop_graph(Slot& s);
// Give the arena ps_compute keeps for a repeat of its last job back to the device pool, with the
// plan and graphs that refer to it.  The caller holds ctx->sync_mu.
void release_sync_arena(ps_ctx* ctx);
size_t output_bytes(const Plan& p, const ps_job& job);

}  // namespace psint
