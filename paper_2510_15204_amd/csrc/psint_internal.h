// Internal descriptors shared by the host planner (plan.cpp) and the gfx950 kernels (kernels.hip).
//
// Data layout in HBM ("chunked SoA"): every per-point quantity of a grid lives in an array of
// nf columns over the grid's padded point count npad.  Points are grouped in chunks of KC = 16;
// element (column f, point g) sits at  ((g / KC) * nf + f) * KC + g % KC.  One chunk of one column is
// a 128-byte line, so the evaluation kernels (one thread per point) write whole lines and the
// contraction kernels load a contiguous run of columns of a chunk as one contiguous segment.
#pragma once
#include <stdint.h>

namespace psint {

constexpr int KC = 16;          // points per chunk
constexpr int PAD_POINTS = 256; // grids are padded to a multiple of this many points (zero weight)
constexpr int LMAX = 6;         // highest angular momentum the kernels are built for
constexpr int NMAX = 12;        // highest principal quantum number

// One prolate spheroidal grid G(A,B|C) on the device (Sections 2.1-2.3 of the paper).
struct GridDev {
  double a;                 // half the A-B distance
  double ex[3], ey[3], ez[3];
  double cx, cz;            // third centre in the local frame: (cx, 0, cz)
  double lines_mu_off;      // unused padding for alignment
  int32_t has_c;
  int32_t nmu, nnu, nphi, q, nsp, split, istar, jstar;
  int32_t lines;            // offset of mu[0..nmu], nu[0..nnu], phi[0..nphi] in the line buffer
  int32_t gl;               // offset of GL nodes[q] then weights[q] in the line buffer
  int32_t pad0;
  int64_t npts, npad, n_reg;
};

// Evaluation modes.
enum : int32_t {
  EV_CHI = 0,      // chi -> arr0
  EV_CHI_KIN = 1,  // chi -> arr0, -1/2 lap chi -> arr1 (same column)
  EV_POT_W = 2,    // w * V_P -> arr0
  EV_WEIGHTS = 3   // weight columns -> arr0
};

enum : int32_t { CEN_A = 0, CEN_B = 1, CEN_C = 2 };

// A shell: functions of one atom sharing (n, l, zeta); its m components and output columns are
// listed in the m-list at [m_off, m_off + nm).
struct ShellDev {
  double zeta, norm;  // norm = (2 zeta)^(n+1/2) / sqrt((2n)!)
  double pre;         // potential prefactor 4 pi / (2l+1) * norm * zeta^-(n+1)
  int32_t n, l, m_off, nm;
};

// One m component of a shell: real-harmonic factor f (Y_lm = f * C_l^m or f * S_l^|m| of the unit
// vector, see kernels.hip) and the output column (-1: not in the basis).  A shell's entries are dense
// in m = -l..l, entry m_off + l + m.
struct MEntry {
  double f;
  int32_t m, col;
};

// Weight column programs (EV_WEIGHTS): value = w * (kind==0 ? 1 : -(zA/rA + zB/rB + zC/rC)), or 1.
struct WColDev {
  double zA, zB, zC;
  int32_t kind;  // 0: w, 1: ones, 2: w * nuclear potential
  int32_t col;
};

// A run of evaluation work: one grid, one centre, a list of shells (sorted by l) or weight columns.
struct SegDev {
  void* arr0;         // output array base (double or float per precision; NULL: none)
  void* arr1;         // second output (EV_CHI_KIN)
  void* arr0d;        // FP64 copies of arr0 / arr1 written by the FP32 (mixed) evaluation for the
  void* arr1d;        // two-index contractions, which stay in FP64 (NULL: none)
  int64_t block0;     // first block index of this segment in the launch
  int32_t grid;       // index into the grid table
  int32_t mode;
  int32_t centre;     // CEN_A / CEN_B / CEN_C
  int32_t nf;         // columns of arr0 (and arr1)
  int32_t item_off;   // shells or weight columns
  int32_t n_items;
  int32_t l_off[LMAX + 2];  // shells of angular momentum l are items [l_off[l], l_off[l+1])
  // Regular cells (i, j, any k) whose bits are set in both masks are written by a shared segment
  // (ShareSegDev) instead; only basis segments of grids with Q = 4 and at most 128 cells per axis.
  int32_t skip;
  int32_t pad1;
  uint64_t skip_mu[2], skip_nu[2];
};

// One grid of a shared evaluation: its output array for the shared atom's basis values (FP32 or FP64
// per precision; NULL: none) and FP64 twin (mixed jobs; NULL: none).
struct ShareMember {
  void* arr0;
  void* arr0d;
  int32_t grid;
  int32_t pad0;
};

// Basis values of one atom (centre A or B) at corresponding points of several grids G(A,B|C) of one
// pair.  Those grids differ only by a rotation about the A-B axis and by their moved lines, so in
// the regular cells that no member's moved lines touch, their points share (mu, nu, phi), the
// distances to A and B and hence every radial factor; each wave takes one such cell (Q = 4: 64
// points), computes the radial factors once and the angular factors in each member's frame.
struct ShareSegDev {
  const ShareMember* members;
  const int32_t* cells;     // shared mu cell indices [n_si], then shared nu cell indices [n_sj]
  int64_t block0;           // first block of this segment in the shared-evaluation launch
  int32_t centre;           // CEN_A / CEN_B
  int32_t nf;               // columns of each member's array
  int32_t n_members, n_si, n_sj;
  int32_t item_off, n_items;
  int32_t l_off[LMAX + 2];
};

// One contraction C[(u,v)][y] = sum_g U[u][g] V[v][g] Y[y][g] over one grid.  The result for pair
// (u, v) and column y goes to out[mapU[u]*s1 + mapV[v]*s2 + mapY[y]*s3] (+= alpha * C) and, with a
// mirror, also to outm[mapU[u]*t1 + mapV[v]*t2 + mapY[y]*t3]; the maps give caller-order indices.
struct TaskDev {
  const void* U;
  const void* V;
  const void* Y;
  const int32_t* pairs;  // 2 * npairs ints: (u column, v column)
  const int32_t* mapU;
  const int32_t* mapV;
  const int32_t* mapY;
  double* out;
  double* outm;          // NULL = no mirror
  int64_t s1, s2, s3, t1, t2, t3;
  double alpha;
  int64_t nchunks;       // K chunks of the grid
  int32_t nfU, nfV, nfY;
  int32_t npairs;
  int32_t y0, ny;        // Y columns [y0, y0 + ny)
  int32_t skip_diag;     // mirror skipped when mapU[u] == mapV[v] (one-centre diagonal)
  int32_t pad0;
};

// The 128-row tile shapes that share one merged contraction launch per memory pass, as (WM, WN, WR):
// the 2 x 2-wave shapes 128 x 128, 96, 64, 32 and the 4 x 1-wave (tall) shapes 128 x 16, 48, 80, 112.
// A tile of a merged launch names its shape by its index here (TileDev::shape).
constexpr int kMergedShapes[8][3] = {{4, 4, 2}, {4, 3, 2}, {4, 2, 2}, {4, 1, 2},
                                     {2, 1, 4}, {2, 3, 4}, {2, 5, 4}, {2, 7, 4}};

// One work-group's share: a (pair-rows x y-columns) tile of a task over a range of point chunks.
struct TileDev {
  int32_t task;
  int32_t row0, nrows;   // pair rows
  int32_t ulo, nu;       // U columns staged
  int32_t vlo, nv;       // V columns staged
  int32_t p0, np;        // y columns [y0 + p0, y0 + p0 + np)
  int32_t shape;         // index into kMergedShapes in a merged launch; 0 in a single-shape launch
  int64_t kc0, nkc;      // chunk range
  int64_t ws;            // workspace offset (elements) of the BM x BN partial tile
};

// A reduction item: the splits of one (task, row tile, column tile), consecutive in the tile list.
struct RedDev {
  int32_t task;
  int32_t row0, nrows, p0, np;
  int32_t nsplit;
  int32_t bm, bn;        // tile shape of the item's partial tiles (row-major, bn columns)
  int64_t ws;            // workspace offset of split 0; split s at ws + s * bm * bn
};

}  // namespace psint
