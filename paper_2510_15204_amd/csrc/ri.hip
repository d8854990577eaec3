// RI assembly (eq. 14): B = L^-1 A with A[P][ab] = (ab|P) over canonical pairs a >= b, then the
// electron-repulsion matrix eri[ab][cd] = sum_R B[R][ab] B[R][cd].  Kernels, all FP64:
//   ri_gather_kernel  (ab|P) [P][a][b] -> A [P][ab]                 (HBM-bound copy)
//   ri_inv_kernel     inverses of the 32 x 32 diagonal blocks of L (substitution, one per work-group)
//   ri_offdiag_kernel L times those inverses below the diagonal blocks
//   ri_subst_kernel   the whole forward substitution on LDS strips of X (n_aux <= 1024)
//   ri_solve_kernel   otherwise one block step of it per launch, as a product on FP64 MFMA
//   ri_syrk_kernel    128 x 128 output tiles on or above the diagonal, v_mfma_f64_16x16x4f64 with
//                     the 16-row slices of B staged in LDS; the mirror tile is written through an LDS
//                     transpose so both halves are stored with coalesced rows
//   ri_tiles_kernel   the product's tile list, written on the device (allocation-free entry point)
// Host entry points: ps_ri_assemble (scratch from the context's device memory) and
// ps_ri_assemble_noalloc (scratch in a fixed static device array; device arrays only).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "ctx.h"
#include "jobs.h"
#include "ri_tiles.h"

namespace psint {

typedef double d4_t __attribute__((ext_vector_type(4)));

// (ab|P) [P][a][b] -> A[P][a(a+1)/2 + b] for b <= a: one wave per row a of one P (blockIdx.y), lanes
// over b, so reads and writes are contiguous runs and no index is divided.
__global__ __launch_bounds__(256) void ri_gather_kernel(const double* __restrict__ abP, int nb,
                                                        double* __restrict__ A) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= nb) return;
  const int64_t P = blockIdx.y;
  const int64_t npair = (int64_t)nb * (nb + 1) / 2;
  const double* __restrict__ src = abP + (P * nb + a) * nb;
  double* __restrict__ dst = A + P * npair + (int64_t)a * (a + 1) / 2;
  for (int b = threadIdx.x & 63; b <= a; b += 64) dst[b] = src[b];
}

constexpr int TR_ROWS = 32;  // rows of B per block step of the forward substitution

// Blocked forward substitution with inverted diagonal blocks.  With D_k the inverse of the k-th
// 32 x 32 diagonal block of L, the transformed factor G holds G_kk = D_k and, below the diagonal
// blocks, G_ik = L_ik D_k.  Then block step k is one product with the not-yet-solved rows X_k:
//   B_k = G_kk X_k        and        X_i -= G_ik X_k for every block row i below k.

// G_kk = D_k by right-looking substitution on X = I in LDS: at step q row q is final once divided by
// L[q][q], and every row below subtracts L[r][q] times it, all (r, j) in parallel.  Each entry sees
// the same operations in the same order as the row-by-row forward substitution.  One 32 x 32 block
// per work-group.
__global__ __launch_bounds__(64) void ri_inv_kernel(const double* __restrict__ L, int na, double* __restrict__ G) {
  __shared__ double Ld[TR_ROWS][TR_ROWS + 1];
  __shared__ double Xd[TR_ROWS][TR_ROWS + 1];
  const int r0 = blockIdx.x * TR_ROWS, nr = min(TR_ROWS, na - r0);
  const int tid = threadIdx.x;
  for (int e = tid; e < TR_ROWS * TR_ROWS; e += 64) {
    const int r = e / TR_ROWS, q = e - r * TR_ROWS;
    Ld[r][q] = (r < nr && q < nr) ? L[(int64_t)(r0 + r) * na + r0 + q] : (r == q ? 1.0 : 0.0);
    Xd[r][q] = r == q ? 1.0 : 0.0;
  }
  __syncthreads();
  const int j = tid & (TR_ROWS - 1), h = tid / TR_ROWS;  // column; half of the rows below
  for (int q = 0; q < TR_ROWS; ++q) {
    if (tid < TR_ROWS) Xd[q][j] /= Ld[q][q];
    __syncthreads();
    const double xq = Xd[q][j];
    for (int r = q + 1 + h; r < TR_ROWS; r += 2) Xd[r][j] -= Ld[r][q] * xq;
    __syncthreads();
  }
  for (int e = tid; e < TR_ROWS * TR_ROWS; e += 64) {
    const int r = e / TR_ROWS, q = e - r * TR_ROWS;
    if (r < nr && q < nr) G[(int64_t)(r0 + r) * na + r0 + q] = q <= r ? Xd[r][q] : 0.0;
  }
}

// G_ik = L_ik D_k for every element (i, c) whose column block lies left of row i's block.
__global__ __launch_bounds__(256) void ri_offdiag_kernel(const double* __restrict__ L, int na, double* __restrict__ G) {
  const int64_t total = (int64_t)na * na;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / na), c = (int)(e - (int64_t)i * na);
    const int k = c / TR_ROWS, r0 = k * TR_ROWS;
    if (i < r0 + TR_ROWS) continue;  // on or above the diagonal blocks
    const int nr = min(TR_ROWS, na - r0), sc = c - r0;
    double v = 0.0;
    for (int t = sc; t < nr; ++t) v += L[(int64_t)i * na + r0 + t] * G[(int64_t)(r0 + t) * na + c];
    G[e] = v;
  }
}

constexpr int UP_T = 64;  // solve tile: 64 rows x 64 columns, K = the 32 rows of block k

// Block step k on FP64 MFMA.  blockIdx.y == 0: B[r0 .. r0 + nr) = G_kk X_k; blockIdx.y >= 1: a
// 64-row tile below the block, X_i -= G_ik X_k.  X rows of block k are only read in this launch.
__global__ __launch_bounds__(256) void ri_solve_kernel(const double* __restrict__ G, int na, int64_t n,
                                                      double* __restrict__ X, double* __restrict__ Bo, int r0) {
  __shared__ double As[TR_ROWS][UP_T + 1], Bs[TR_ROWS][UP_T];
  const int nr = min(TR_ROWS, na - r0);
  const bool diag = blockIdx.y == 0;
  const int64_t i0 = diag ? r0 : r0 + nr + (int64_t)(blockIdx.y - 1) * UP_T;
  const int64_t iend = diag ? r0 + nr : na;
  const int64_t c0 = (int64_t)blockIdx.x * UP_T;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave >> 1, wj = wave & 1, kl = lane >> 4, lc = lane & 15;
  for (int e = tid; e < UP_T * TR_ROWS; e += 256) {
    const int ii = e / TR_ROWS, k = e - ii * TR_ROWS;  // reads along G's rows
    As[k][ii] = (i0 + ii < iend && k < nr) ? G[(i0 + ii) * na + r0 + k] : 0.0;
  }
  for (int e = tid; e < TR_ROWS * UP_T; e += 256) {
    const int k = e / UP_T, c = e - k * UP_T;
    Bs[k][c] = (k < nr && c0 + c < n) ? X[(int64_t)(r0 + k) * n + c0 + c] : 0.0;
  }
  __syncthreads();
  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < TR_ROWS / 4; ++s) {
    double av[2], bv[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) av[m] = As[4 * s + kl][wi * 32 + m * 16 + lc];
#pragma unroll
    for (int m = 0; m < 2; ++m) bv[m] = Bs[4 * s + kl][wj * 32 + m * 16 + lc];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wi * 32 + a * 16 + 4 * r + kl, col = c0 + wj * 32 + b * 16 + lc;
        if (row < iend && col < n) {
          if (diag)
            Bo[row * n + col] = acc[a][b][r];
          else
            X[row * n + col] -= acc[a][b][r];
        }
      }
}

// The whole forward substitution in one launch while a strip of X fits in LDS: the columns of X
// (pairs ab) are independent, so a work-group takes SB_W of them over all n_aux rows and runs every
// block step on its LDS copy, B_k = G_kk X_k and X_i -= G_ik X_k for the 16-row blocks below, with
// G (L2-resident) as the MFMA A operand.  Larger n_aux: one launch per block step
// (ri_solve_kernel).
constexpr int SB_W = 16;                   // columns of X per work-group
constexpr int SB_LD = SB_W + 2;            // padded LDS row, doubles
constexpr int SB_MAX_NA = 1024;            // 1024 x 18 doubles = 144 KB of LDS
constexpr int SB_MAX_LDS = SB_MAX_NA * SB_LD * 8;

__global__ __launch_bounds__(256) void ri_subst_kernel(const double* __restrict__ G, int na, int64_t n,
                                                      const double* __restrict__ X, double* __restrict__ Bo) {
  extern __shared__ __attribute__((aligned(16))) double Xs[];  // na_pad rows x SB_LD
  const int na_pad = (na + TR_ROWS - 1) / TR_ROWS * TR_ROWS;
  const int64_t c0 = (int64_t)blockIdx.x * SB_W;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kl = lane >> 4, lc = lane & 15;
  for (int e = tid; e < na_pad * SB_W; e += 256) {
    const int r = e / SB_W, c = e - r * SB_W;
    Xs[r * SB_LD + c] = (r < na && c0 + c < n) ? X[(int64_t)r * n + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int k0 = 0; k0 < na_pad; k0 += TR_ROWS) {
    // The 16-row blocks j of rows k0 + 16 j: j = 0, 1 form B_k = G_kk X_k (held in registers), the
    // others X_i -= G_ik X_k (G_ik = L_ik D_k already holds the diagonal block's inverse); all read
    // X_k as it stands, and B_k replaces it once every read is done.  Wave w takes j = w, w + 4, ...,
    // four blocks at a time: their G operands are loaded together and their MFMA chains interleave.
    const int nrb = (na_pad - k0) / 16;
    d4_t bk = (d4_t){0.0, 0.0, 0.0, 0.0};
    for (int j0 = wave; j0 < nrb; j0 += 16) {
      double a[4][TR_ROWS / 4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int gr = k0 + 16 * (j0 + 4 * jj) + lc;
#pragma unroll
        for (int st = 0; st < TR_ROWS / 4; ++st) {
          const int q = k0 + 4 * st + kl;
          a[jj][st] = (gr < na && q < na) ? G[(int64_t)gr * na + q] : 0.0;
        }
      }
      d4_t u[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) u[jj] = (d4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < TR_ROWS / 4; ++st) {
        const double xv = Xs[(k0 + 4 * st + kl) * SB_LD + lc];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) u[jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[jj][st], xv, u[jj], 0, 0, 0);
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = j0 + 4 * jj;
        if (j < 2) {
          bk = u[jj];
        } else if (j < nrb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Xs[(k0 + 16 * j + 4 * r + kl) * SB_LD + lc] -= u[jj][r];
        }
      }
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Xs[(k0 + 16 * wave + 4 * r + kl) * SB_LD + lc] = bk[r];
    }
    __syncthreads();
  }
  for (int e = tid; e < na * SB_W; e += 256) {
    const int r = e / SB_W, c = e - r * SB_W;
    if (c0 + c < n) Bo[(int64_t)r * n + c0 + c] = Xs[r * SB_LD + c];
  }
}

constexpr int SY_T = 128;  // output tile (4 waves in 2 x 2, 64 x 64 each: 4 x 4 MFMA blocks)
constexpr int SY_K = 16;   // rows of B per stage
constexpr int SY_LD = SY_T + 16;  // padded LDS row, doubles: rows k and k + 1 fall in opposite bank halves

// C = X^T X for X (nk x n, row-major); tile list holds (ti, tj) with ti <= tj.  Each stage's 16 rows
// of the tile's two column ranges are loaded into registers while the MFMAs of the previous stage
// run and then stored into the other of two LDS buffers, so one barrier per stage suffices.  The
// tile is stored from the accumulators with 16 consecutive columns per row; off the diagonal its
// transpose goes through a 16 x 16 LDS block per wave, so that it is stored with coalesced rows too.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ri_syrk_kernel(
    const double* __restrict__ X, int nk, int64_t n, const int2* __restrict__ tiles, double* __restrict__ C) {
  constexpr int BUF = SY_K * SY_LD;
  __shared__ __attribute__((aligned(16))) double As[2 * BUF];
  __shared__ __attribute__((aligned(16))) double Bs[2 * BUF];
  const int2 tl = tiles[blockIdx.x];
  const int64_t i0 = (int64_t)tl.x * SY_T, j0 = (int64_t)tl.y * SY_T;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1, kl = lane >> 4, lc = lane & 15;
  d4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (d4_t){0.0, 0.0, 0.0, 0.0};
  constexpr int PER = SY_K * SY_T / 256;  // values per thread and operand per stage
  double ra[PER], rb[PER];
  const int lcol = tid & (SY_T - 1), lrow = tid / SY_T;  // thread's column, first row (rows step by 2)
  // loads without branches: out-of-range rows and columns read a clamped (valid) address, and are
  // replaced by zero only when stored to LDS, after the MFMAs that hide the loads' latency
  const bool ain = i0 + lcol < n, bin = j0 + lcol < n;
  const double* xa = X + (ain ? i0 + lcol : n - 1);
  const double* xb = X + (bin ? j0 + lcol : n - 1);
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int64_t off = (int64_t)min(k0 + lrow + 2 * q, nk - 1) * n;
      ra[q] = xa[off];
      rb[q] = xb[off];
    }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const bool kin = k0 + lrow + 2 * q < nk;
      As[buf * BUF + (lrow + 2 * q) * SY_LD + lcol] = (kin && ain) ? ra[q] : 0.0;
      Bs[buf * BUF + (lrow + 2 * q) * SY_LD + lcol] = (kin && bin) ? rb[q] : 0.0;
    }
  };
  load(0);
  store(0, 0);
  __syncthreads();
  const int nst = (nk + SY_K - 1) / SY_K;
  // Operand registers, two slots: step s + 1's operands are read from LDS while step s's MFMAs run.
  // The next stage's rows go into LDS and the barrier follows before the MFMAs of a stage's last step
  // (whose operands are already in registers); the next stage's first operands are read right after
  // the barrier, so those MFMAs cover that read.  SY_K / 4 is even: a stage starts in slot 0.
  double av[2][4], bv[2][4];
  auto operands = [&](const double* Ac, const double* Bc, int s, int slot) {
#pragma unroll
    for (int m = 0; m < 4; ++m) av[slot][m] = Ac[(4 * s + kl) * SY_LD + wm * 64 + m * 16 + lc];
#pragma unroll
    for (int m = 0; m < 4; ++m) bv[slot][m] = Bc[(4 * s + kl) * SY_LD + wn * 64 + m * 16 + lc];
  };
  if (nst > 0) operands(As, Bs, 0, 0);
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) load((st + 1) * SY_K);
    const double* Ac = As + (st & 1) * BUF;
    const double* Bc = Bs + (st & 1) * BUF;
#pragma unroll
    for (int s = 0; s < SY_K / 4; ++s) {
      const int sl = s & 1;
      if (s + 1 < SY_K / 4) {
        operands(Ac, Bc, s + 1, sl ^ 1);
      } else if (more) {
        __builtin_amdgcn_sched_barrier(0);
        store((st + 1) & 1, (st + 1) * SY_K);
        __syncthreads();
        operands(As + ((st + 1) & 1) * BUF, Bs + ((st + 1) & 1) * BUF, 0, sl ^ 1);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[sl][a], bv[sl][b], acc[a][b], 0, 0, 0);
      // issue order: the next step's eight LDS reads two at a time between the first MFMAs
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // two LDS reads
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the tile: accumulator register r of lane (kl, lc) is row 4 r + kl, column lc of its 16 x 16 block
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wm * 64 + a * 16 + 4 * r + kl, col = j0 + wn * 64 + b * 16 + lc;
        if (row < n && col < n) C[row * n + col] = acc[a][b][r];
      }
  if (tl.x == tl.y) return;  // (uniform) a diagonal tile holds both halves already
  // the transpose, block by block through this wave's 16 x 17 LDS patch
  double* Tw = As + wave * 16 * 17;
  __syncthreads();  // every wave is done with As
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Tw[(4 * r + kl) * 17 + lc] = acc[a][b][r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = 4 * r + kl;  // column of the block = row of the transpose
        const int64_t row = j0 + wn * 64 + b * 16 + x, col = i0 + wm * 64 + a * 16 + lc;
        if (row < n && col < n) C[row * n + col] = Tw[lc * 17 + x];
      }
      __syncthreads();
    }
}

// Tile list of ri_syrk_kernel, one entry per thread, in the order of ri_syrk_tile.
__global__ __launch_bounds__(256) void ri_tiles_kernel(int64_t nt, int64_t ntiles, int2* __restrict__ tiles) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int i, j;
  ri_syrk_tile(t, nt, &i, &j);
  tiles[t] = make_int2(i, j);
}

// The kernel chain of one RI assembly on `st`: gather, inverses of the diagonal blocks, the
// transformed factor, the forward substitution into Bo and, when C is given, the product over the
// ntiles tiles listed at `tiles`.  X, G and Bo are the call's scratch (Bo may be the caller's B).
hipError_t ri_launch_chain(hipStream_t st, int n_bf, int n_aux, const double* abP, const double* L, double* X,
                           double* G, double* Bo, const int2* tiles, int64_t ntiles, double* C) {
  const int64_t na = n_aux, npair = (int64_t)n_bf * (n_bf + 1) / 2;
  hipLaunchKernelGGL(ri_gather_kernel, dim3((unsigned)((n_bf + 3) / 4), (unsigned)n_aux), dim3(256), 0, st, abP,
                     n_bf, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nblk = (n_aux + TR_ROWS - 1) / TR_ROWS;
  hipLaunchKernelGGL(ri_inv_kernel, dim3((unsigned)nblk), dim3(64), 0, st, L, n_aux, G);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t blocks = (na * na + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(ri_offdiag_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, n_aux, G);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (n_aux <= SB_MAX_NA) {
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)ri_subst_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, SB_MAX_LDS);
    if (attr != hipSuccess) return attr;
    const size_t lds = (size_t)((n_aux + TR_ROWS - 1) / TR_ROWS * TR_ROWS) * SB_LD * sizeof(double);
    hipLaunchKernelGGL(ri_subst_kernel, dim3((unsigned)((npair + SB_W - 1) / SB_W)), dim3(256), lds, st,
                       (const double*)G, n_aux, npair, (const double*)X, Bo);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    for (int r0 = 0; r0 < n_aux; r0 += TR_ROWS) {
      const int below = n_aux - std::min(n_aux, r0 + TR_ROWS);
      hipLaunchKernelGGL(ri_solve_kernel,
                         dim3((unsigned)((npair + UP_T - 1) / UP_T), (unsigned)(1 + (below + UP_T - 1) / UP_T)),
                         dim3(256), 0, st, (const double*)G, n_aux, npair, X, Bo, r0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (C) {
    hipLaunchKernelGGL(ri_syrk_kernel, dim3((unsigned)ntiles), dim3(256), 0, st, (const double*)Bo, n_aux, npair,
                       tiles, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace psint

using namespace psint;

namespace {

// The call's device scratch, taken from the context's device pool (the same budget and memory as
// job arenas) and given back when the call returns; the stream is drained first, so no kernel of
// the call still uses it, also after an error.
struct RiScratch {
  ps_ctx* ctx;
  hipStream_t st;
  void* p = nullptr;
  size_t size = 0;
  RiScratch(ps_ctx* c, hipStream_t s) : ctx(c), st(s) {}
  ~RiScratch() {
    if (!p) return;
    (void)hipStreamSynchronize(st);
    pool_release(ctx, p, size);
  }
};

// Timing events of one call, destroyed on every return path.
struct RiEvents {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~RiEvents() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

#define RI_TRY(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) {                                       \
      set_err(ctx, std::string(#call) + ": " + hipGetErrorString(e_)); \
      return PS_E_DEVICE;                                         \
    }                                                             \
  } while (0)

extern "C" int32_t ps_ri_assemble(ps_ctx* ctx, int32_t n_bf, int32_t n_aux, int32_t location, const double* abP,
                                  const double* L, double* B, double* eri, double* device_ms) {
  if (!ctx) return PS_E_INVALID;
  if (n_bf < 1 || n_aux < 1 || !abP || !L || (location != PS_OUT_HOST && location != PS_OUT_DEVICE)) {
    set_err(ctx, "ri: n_bf, n_aux >= 1, abP and L required, location PS_OUT_HOST or PS_OUT_DEVICE");
    return PS_E_INVALID;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  // the synchronous stream is shared with ps_compute and ps_autotune: one of them at a time
  std::lock_guard<std::mutex> sync_guard(ctx->sync_mu);
  const bool dev = location == PS_OUT_DEVICE;
  const int64_t nb = n_bf, na = n_aux, npair = nb * (nb + 1) / 2;
  const size_t abp_b = (size_t)na * nb * nb * 8, l_b = (size_t)na * na * 8, x_b = (size_t)na * npair * 8,
               eri_b = (size_t)npair * npair * 8;
  // scratch: X always; host inputs and host eri staged on the device
  size_t off_abp = 0, off_l = 0, off_x = 0, off_eri = 0, total = 0;
  if (!dev) {
    off_abp = total;
    total = align256(total + abp_b);
    off_l = total;
    total = align256(total + l_b);
  }
  off_x = total;
  total = align256(total + x_b);
  const size_t off_b = total;
  total = align256(total + x_b);
  const size_t off_g = total;
  total = align256(total + l_b);
  const size_t ntiles = (size_t)((npair + SY_T - 1) / SY_T) * ((npair + SY_T - 1) / SY_T + 1) / 2;
  const size_t off_tiles = total;
  total = align256(total + ntiles * sizeof(int2));
  if (eri && !dev) {
    off_eri = total;
    total = align256(total + eri_b);
  }
  if (total > ctx->budget) {
    char buf[160];
    snprintf(buf, sizeof buf, "ri: needs %.2f GB of device memory, budget is %.2f GB", total / 1e9, ctx->budget / 1e9);
    set_err(ctx, buf);
    return PS_E_NOMEM;
  }
  hipStream_t st = ctx->sync_slot.stream;
  RiScratch scratch(ctx, st);
  scratch.p = pool_alloc(ctx, total, &scratch.size);
  if (!scratch.p) {
    // the arena kept for a repeat of the last ps_compute job is the one other user of the budget
    // that is idle now (this call holds sync_mu)
    release_sync_arena(ctx);
    scratch.p = pool_alloc(ctx, total, &scratch.size);
  }
  if (!scratch.p) {
    // then the ranges idle serving slots keep
    release_idle_serve_arenas(ctx);
    scratch.p = pool_alloc(ctx, total, &scratch.size);
  }
  if (!scratch.p) {
    char buf[160];
    snprintf(buf, sizeof buf, "ri: no device memory for %.2f GB of scratch within the %.2f GB budget", total / 1e9,
             ctx->budget / 1e9);
    set_err(ctx, buf);
    return PS_E_NOMEM;
  }
  char* base = (char*)scratch.p;
  const double* d_abp = dev ? abP : (const double*)(base + off_abp);
  const double* d_l = dev ? L : (const double*)(base + off_l);
  double* d_x = (double*)(base + off_x);
  double* d_b = (double*)(base + off_b);
  double* d_g = (double*)(base + off_g);
  int2* d_tiles = (int2*)(base + off_tiles);
  double* d_eri = eri ? (dev ? eri : (double*)(base + off_eri)) : nullptr;
  if (!dev) {
    RI_TRY(hipMemcpyAsync((void*)d_abp, abP, abp_b, hipMemcpyHostToDevice, st));
    RI_TRY(hipMemcpyAsync((void*)d_l, L, l_b, hipMemcpyHostToDevice, st));
  }
  std::vector<int2> tl;
  if (eri) {
    tl.resize(ntiles);
    const int64_t nt = (npair + SY_T - 1) / SY_T;
    for (size_t t = 0; t < ntiles; ++t) ri_syrk_tile((int64_t)t, nt, &tl[t].x, &tl[t].y);
    RI_TRY(hipMemcpyAsync(d_tiles, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  }
  RiEvents ev;
  RI_TRY(hipEventCreate(&ev.e0));
  RI_TRY(hipEventCreate(&ev.e1));
  RI_TRY(hipEventRecord(ev.e0, st));
  RI_TRY(ri_launch_chain(st, n_bf, n_aux, d_abp, d_l, d_x, d_g, d_b, d_tiles, (int64_t)tl.size(), d_eri));
  RI_TRY(hipEventRecord(ev.e1, st));
  if (B) RI_TRY(hipMemcpyAsync(B, d_b, x_b, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  if (eri && !dev) RI_TRY(hipMemcpyAsync(eri, d_eri, eri_b, hipMemcpyDeviceToHost, st));
  RI_TRY(hipStreamSynchronize(st));
  float ms = 0.0f;
  RI_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
  if (device_ms) *device_ms = ms;
  return PS_OK;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free RI assembly: the call's scratch lives in a fixed static device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name to a kernel or copy (in
// host code it is only a stand-in for the symbol): the device address of each GPU's copy is looked
// up once per device with hipGetSymbolAddress and kept in scratch_ptr.
// ---------------------------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[PS_RI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Device address of `device`'s scratch copy; that device must be current.  Looked up on the first
// call per device and kept.
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

namespace psint {

// Called by ps_create with the context's device current, so that the allocation-free entry point
// finds its scratch address already looked up.
int32_t ri_noalloc_init(int device) {
  void* p = nullptr;
  return scratch_address(device, &p) == hipSuccess ? PS_OK : PS_E_DEVICE;
}

}  // namespace psint

extern "C" int32_t ps_ri_assemble_noalloc(ps_ctx* ctx, int32_t n_bf, int32_t n_aux, const double* abP,
                                          const double* L, double* B, double* eri) {
  if (!ctx) return PS_E_INVALID;
  if (n_bf < 1 || n_aux < 1 || !abP || !L) {
    set_err(ctx, "ri (no-alloc): n_bf, n_aux >= 1, abP and L required");
    return PS_E_INVALID;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return PS_E_DEVICE;
  std::lock_guard<std::mutex> sync_guard(ctx->sync_mu);
  const int64_t nb = n_bf, na = n_aux, npair = nb * (nb + 1) / 2;
  const int64_t nt = (npair + SY_T - 1) / SY_T;
  const int64_t ntiles = eri ? nt * (nt + 1) / 2 : 0;
  const size_t x_b = (size_t)na * npair * 8, g_b = (size_t)na * na * 8;
  // X, then B unless the caller's B receives it, then G, then the tile list
  const size_t off_x = 0;
  size_t total = align256(x_b);
  const size_t off_b = total;
  if (!B) total = align256(total + x_b);
  const size_t off_g = total;
  total = align256(total + g_b);
  const size_t off_t = total;
  total = align256(total + (size_t)ntiles * sizeof(int2));
  if (total > (size_t)PS_RI_NOALLOC_SCRATCH_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "ri (no-alloc): needs %.1f MiB of scratch (n_aux %d, n_pair %lld%s), the static scratch holds %.1f MiB",
             total / 1048576.0, n_aux, (long long)npair, B ? "" : ", B not given", PS_RI_NOALLOC_SCRATCH_BYTES / 1048576.0);
    set_err(ctx, buf);
    return PS_E_NOMEM;
  }
  void* base_v = nullptr;
  RI_TRY(scratch_address(ctx->device, &base_v));
  char* base = (char*)base_v;
  double* d_x = (double*)(base + off_x);
  double* d_b = B ? B : (double*)(base + off_b);
  double* d_g = (double*)(base + off_g);
  int2* d_tiles = (int2*)(base + off_t);
  hipStream_t st = ctx->sync_slot.stream;
  if (eri) {
    hipLaunchKernelGGL(ri_tiles_kernel, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, nt, ntiles,
                       d_tiles);
    RI_TRY(hipGetLastError());
  }
  RI_TRY(ri_launch_chain(st, n_bf, n_aux, abP, L, d_x, d_g, d_b, d_tiles, ntiles, eri));
  return PS_OK;
}
