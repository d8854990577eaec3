// Host-side planner: validation, grid construction (lines, frame, third-centre moves), routing of
// integral blocks to grids, device array layout, evaluation segments, contraction tasks and tiles.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/psint.h"
#include "psint_internal.h"

namespace psint {

// Contraction tile shape: 4 waves in a 2 x 2 arrangement, each wave WM x WN MFMA blocks of 16 x 16.
struct TileShape {
  int wm = 4, wn = 4;
  int wr = 2;                             // waves along the rows: 2 (2 x 2) or 4 (4 x 1)
  int sc = 1;                             // storage chunks (16 points each) per contraction stage
  int slots = 0;                          // work-groups of this shape resident on the device at once
                                          // (0 = unknown: no rounding of the K splits)
  int slots2 = 0;                         // the same for the 64 x 64 two-index shape
  int slots_n[4] = {0, 0, 0, 0};          // the same for this shape narrowed to wn = 1..3 (index wn)
  int slots2n = 0;                        // the same for the 64 x 32 shape
  int slots2_f64 = 0, slots2n_f64 = 0;    // 64 x 64 and 64 x 32 in FP64 within a mixed job
  int slots_short[5] = {0, 0, 0, 0, 0};   // the 32-row shapes (wm = 1) of width wn = 1..4 (index wn)
  int slots_short_f64[3] = {0, 0, 0};     // FP64 32 x 32 and 32 x 64 within a mixed job
  int slots_tall[4] = {0, 0, 0, 0};       // the 4 x 1 shapes 128 x (16, 48, 80, 112) (index (wn - 1) / 2)
  int bm() const { return 16 * wm * wr; }
  int bn() const { return 16 * wn * (4 / wr); }
  int maxuv() const { return bm() + 4; }  // staged U + V columns per tile
  static constexpr int SC_MAX = 2;        // tiles start and end on multiples of this many chunks
};

struct GridHost {
  int A, B, C;          // A < B, C = -1 for none
  bool pair_grid;       // G(A,B|C*) or the only grid of a diatomic
  ps_grid_spec spec;
  GridDev dev;
  std::vector<double> mu, nu, phi;
};

// A device array of nf columns over a grid's padded points (chunked SoA).
struct ArrayHost {
  int grid;
  int nf;
  size_t es = 8;        // bytes per element: 8 (FP64) or 4 (FP32 operands of a mixed job)
  int64_t offset;       // bytes from the array area start (its pass's region start, plus its place there)
  std::vector<int32_t> map;  // column -> caller index (or output selector)
  int64_t map_off;      // int offset in the int table
};

struct SegHost {
  SegDev dev;
  int arr0, arr1;       // array ids (-1: none)
  int arr0d = -1, arr1d = -1;  // FP64 copies written beside FP32 arr0 / arr1 (mixed jobs)
};

// A shared evaluation (cross-third-centre reuse): the device segment, its members' array ids and
// the members' own basis segments (which skip the shared cells).
struct ShareHost {
  ShareSegDev dev;
  std::vector<int> grids, arr0, arr0d, segs;
  int64_t cells_off = 0;    // int offset of the shared mu and nu cell lists
  bool dropped = false;     // members in different memory passes: no sharing
};

struct TaskHost {
  TaskDev dev;
  int grid;
  int U, V, Y;          // array ids
  int64_t pairs_off;    // int offset of the pair list
  int out_kind;         // 0 S, 1 T, 2 V, 3 PQ, 4 abP (for offsets)
  int64_t out_off, outm_off;  // element offsets in the internal output buffer (-1 = none)
  int phase;
  double pair_points;   // algorithmic work of the task (unique elements x points)
};

struct Pass {
  int grid0, grid1;     // grids [grid0, grid1)
  int seg0, seg1;       // segments
  int task0, task1;     // tasks
  int tile0, tile1;     // all tiles of the pass
  int sseg0 = 0, sseg1 = 0;     // shared evaluation segments (Plan::ssegs)
  int64_t shared_blocks = 0;    // blocks of their launch
  struct Launch {
    int tile0, tile1;   // consecutive tiles of one contraction launch
    TileShape shape;    // wm == 0: the merged launch of the 128-row shapes (TileDev::shape per tile)
    bool f64 = false;   // FP64 contraction within a mixed job (its two-index tasks)
  };
  std::vector<Launch> launches;  // main shape, 64 x 64 shape, then narrow last-column-tile shapes
  std::vector<std::vector<int>> red_by_phase;  // reduce item ids per phase
  int64_t eval_blocks;
  size_t array_bytes;
  size_t ws_elems;
  size_t ws_offset;     // bytes from the array area's start to the pass's partial tiles (after its arrays)
  size_t region_off = 0;  // bytes from the array area's start to the pass's region (overlapped passes)
};

struct Plan {
  // copied inputs
  std::vector<ps_atom> atoms;
  std::vector<ps_sto> basis, aux;
  int n_bf = 0, n_aux = 0, n_atoms = 0;
  int precision = 0;
  TileShape tile;        // (ab|P) tasks
  TileShape tile2;       // two-index tasks (S, T, V, (P|Q)): a smaller tile wastes less on their short
                         // column ranges (one atom's basis or auxiliary functions)
  int ksplit_override = 0;

  std::vector<GridHost> grids;
  std::vector<double> lines;         // device line buffer contents
  std::vector<ArrayHost> arrays;
  std::vector<ShellDev> shells;
  std::vector<MEntry> ments;
  std::vector<WColDev> wcols;
  std::vector<SegHost> segs;
  std::vector<ShareHost> shares;     // all candidate shared segments (some dropped)
  std::vector<int> ssegs;            // kept shares, in pass order (indices into shares)
  std::vector<TaskHost> tasks;
  std::vector<TileDev> tiles;
  std::vector<RedDev> reds;
  std::vector<int32_t> ints;         // pair lists and column maps
  std::vector<Pass> passes;

  // internal output buffer (FP64 elements)
  int64_t off_S = 0, off_T = 0, off_V = 0, off_PQ = 0, off_abP = 0, off_L = 0, out_elems = 0;

  double pair_points = 0.0;
  double contract_flops = 0.0;
  double issued_flops = 0.0;
  int64_t n_points = 0;
  size_t max_array_bytes = 0;  // array area: one region (arrays, then partial tiles) per pass, or two
                               // alternating regions when passes overlap
  // Overlapped passes: pass i + 1's evaluation runs while pass i's contraction reads its own region,
  // so consecutive passes take alternate halves of the array budget.
  bool overlap = false;
  size_t max_ws_bytes = 0;     // partial tiles alone (max over passes)
  size_t meta_bytes = 0;
};

// Validate the job; returns PS_OK or an error code with a message.
int32_t validate_job(const ps_job* job, std::string* err);

// Build the full plan.  `budget` bounds array + workspace bytes per pass.  With `overlap_passes`, a job
// that needs more than one memory pass is planned with two alternating regions (Plan::overlap).
int32_t build_plan(const ps_job* job, const TileShape& shape, int ksplit_override, size_t budget,
                   Plan* plan, std::string* err, bool share_third = false, bool overlap_passes = false);

// Grid construction alone (used by the inspection hook).
int32_t build_grid(const ps_atom* atoms, int n_atoms, int A, int B, int C, const ps_grid_spec& spec,
                   GridHost* g, std::string* err);

// Gauss-Legendre nodes/weights on [-1, 1].
void gauss_legendre(int q, double* x, double* w);

}  // namespace psint
