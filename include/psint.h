/*
 * psint.h -- C ABI of the MI355X (gfx950) library for Slater-type-orbital integrals by quadrature on
 * prolate spheroidal grids.
 *
 * Method: Stark, Meier, Hatch, Kammeraad, Dang, Zimmerman, "Numerical Integration of Slater Basis
 * Functions Over Prolate Spheroidal Grids", arXiv 2510.15204.  The caller passes a geometry, a Slater
 * basis, an auxiliary Slater basis and a grid specification, and receives FP64 integral blocks:
 *   S_ab      = sum_g w_g chi_a chi_b                                  (eq. 9 with O = 1)
 *   T_ab      = 1/2 sum_g w_g (chi_a L chi_b + L chi_a chi_b), L = -1/2 lap   (eq. 9, kinetic)
 *   V_ab      = sum_g w_g chi_a chi_b (-sum_C Z_C / r_C)               (eq. 9, nuclear attraction)
 *   (ab|P)    = sum_g w_g chi_a chi_b V_P                              (eq. 16)
 *   (P|Q)     = 1/2 sum_g w_g (V_P chi_Q + V_Q chi_P)                  (eqs. 14-16, RI metric)
 *   (P|Q) = L L^T, lower Cholesky factor in FP64                       (eq. 14 needs (PQ)^-1)
 * with chi = N r^(n-1) e^(-zeta r) Y_lm (eq. 1; real, orthonormal Y_lm, no Condon-Shortley phase,
 * N = (2 zeta)^(n+1/2) / sqrt((2n)!)), V_P the Coulomb potential of the auxiliary function chi_P, and
 * the sums running over the points and weights of prolate spheroidal grids (eqs. 2-7, 10-12, 17;
 * Algorithms 1-2) with third-centre line moving and N_SP splitting (Sections 2.2-2.3).
 *
 * Which grid each integral is summed on follows the paper's 3-atom-subset rule (Section 4): for two
 * atoms one unrefined grid serves everything; for N >= 3 atoms there is one grid G(A,B|C) per atom
 * pair A<B and third atom C, refined at C.  The "pair grid" of (A,B) is G(A,B|C*) with C* the atom
 * nearest the A-B midpoint; one-centre blocks of atom X use the pair grid of X and its nearest
 * neighbour (and, for a potential or nucleus on another atom C, the pair grid of X and C).
 *
 * Units are bohr and hartree.  All entry points are thread-compatible (one context per thread, or
 * serialise calls on a context) and never throw; they return a ps_status code.
 */
#ifndef PSINT_H
#define PSINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------------------------- */
enum {
  PS_OK = 0,
  PS_E_INVALID = -1,     /* malformed input: indices, quantum numbers, exponents, geometry, spec  */
  PS_E_UNSUPPORTED = -2, /* valid but outside the built kernels: l > 6, n > 12, q > 16            */
  PS_E_NOMEM = -3,       /* the job can never fit the context's device-memory budget            */
  PS_E_DEVICE = -4,      /* a HIP call failed; ps_last_error has the text                        */
  PS_E_NOT_PD = -5,      /* (P|Q) not positive definite; every other output is still valid       */
  PS_E_TIMEOUT = -6,     /* ps_wait timed out; the job keeps running                             */
  PS_E_QUEUE_FULL = -7,  /* ps_submit: too many jobs in flight                                   */
  PS_E_NOT_FOUND = -8    /* unknown ticket                                                       */
};

/* ---- inputs --------------------------------------------------------------------------------- */
typedef struct {
  double xyz[3]; /* position, bohr */
  double Z;      /* nuclear charge (>= 0) */
} ps_atom;

typedef struct {
  int32_t atom;  /* index into the atom array */
  int32_t n;     /* principal quantum number, 1 <= n <= 12 */
  int32_t l;     /* 0 <= l < n, l <= 6 */
  int32_t m;     /* -l <= m <= l (real harmonics: m > 0 cos branch, m < 0 sin branch) */
  double zeta;   /* exponent > 0 */
} ps_sto;

typedef struct {
  int32_t n_mu, n_nu, n_phi; /* CELLS per axis (the paper's N_mu, N_nu, N_phi), each >= 2          */
  int32_t q;                 /* Gauss-Legendre points per axis per cell (paper: Q = 4), 1..16      */
  int32_t n_sp;              /* third-centre split per axis (paper: N_SP = 3; 1 = move lines only) */
  double c1_scale, c1_exp;   /* C1 = c1_scale * a^c1_exp, a = half the pair distance (2.3, 0.25)   */
} ps_grid_spec;

typedef struct {
  int32_t atom_a, atom_b;    /* unordered atom pair whose grids use `spec` instead of the default */
  ps_grid_spec spec;
} ps_pair_grid;

typedef enum {
  PS_PREC_FP64 = 0,  /* every step in FP64                                                          */
  PS_PREC_MIXED = 1  /* FP32 function values and FP32 MFMA over short point chunks, flushed into FP64
                        accumulators; FP64 grid coordinates/Jacobian, block sums and Cholesky      */
} ps_precision;

/* Output placement. */
enum { PS_OUT_HOST = 0, PS_OUT_DEVICE = 1 };

typedef struct {
  const ps_atom* atoms;  int32_t n_atoms;      /* n_atoms >= 2                                  */
  const ps_sto* basis;   int32_t n_bf;
  const ps_sto* aux;     int32_t n_aux;
  ps_grid_spec grid;                           /* default spec for every pair                    */
  const ps_pair_grid* pair_grids; int32_t n_pair_grids;  /* per-pair overrides (may be NULL/0)  */
  int32_t precision;                           /* ps_precision                                   */
  int32_t out_location;                        /* PS_OUT_HOST or PS_OUT_DEVICE                   */
  /* Outputs (NULL = not wanted).  Row-major FP64, caller-owned, on the host or (PS_OUT_DEVICE) on
   * the context's device.  S, T, V: n_bf x n_bf, full symmetric.  PQ: n_aux x n_aux symmetric.
   * PQ_chol: lower factor L with PQ = L L^T, upper triangle zeroed.
   * abP: [P][a][b], element abP[((size_t)P * n_bf + a) * n_bf + b], symmetric in a, b. */
  double *S, *T, *V, *PQ, *PQ_chol, *abP;
} ps_job;

typedef struct {
  int64_t n_grids;       /* grids summed over                                                    */
  int64_t n_points;      /* total quadrature points over those grids                            */
  double pair_points;    /* sum over output elements of the points of each grid the element is
                            summed on (unique elements: a <= b within one atom, both orders once
                            for two atoms); one pair-point is one multiply-add                   */
  double queue_ms;       /* submit -> start on the device (serving)                              */
  double device_ms;      /* first kernel -> last kernel, HIP events                              */
  double total_ms;       /* call (or submit) -> results ready                                     */
  double contract_ms;    /* time inside the contraction kernels, HIP events                      */
  double contract_flops; /* algorithmic FLOPs of the contraction kernels (2 per pair-point)      */
  double issued_flops;   /* FLOPs the contraction tiles issue, padding included                   */
  int64_t n_passes;      /* grid batches run one after another to fit the device-memory budget   */
  int64_t graph_replay;  /* 1: the device work ran as a replay of a captured HIP graph (ps_compute of
                            a job identical to the previous one on the context), else 0           */
  int64_t passes_overlapped; /* 1: the passes ran overlapped (PS_OPT_OVERLAP_PASSES), else 0      */
} ps_job_stats;

typedef struct ps_ctx ps_ctx;

/* ---- context -------------------------------------------------------------------------------- */
/* Create a context on HIP device `hip_device` that keeps at most `hbm_budget_bytes` of device
 * memory for grids, function tables and workspaces (0 = 80% of the device's free memory).
 * `stream` is a hipStream_t to run on (NULL = the context creates its own).  Returns PS_OK and sets
 * *out, or a negative status.  The context owns all of its device memory: it is allocated as jobs
 * need it (a job needing a quarter of the budget or more reserves the rest of the budget at once),
 * reused by later jobs, and released by ps_destroy. */
int32_t ps_create(int32_t hip_device, size_t hbm_budget_bytes, void* stream, ps_ctx** out);
/* Destroy a context: jobs already running on the device finish, submitted jobs not yet started are
 * dropped, and all device memory of the context is released. */
int32_t ps_destroy(ps_ctx* ctx);

/* ---- synchronous compute -------------------------------------------------------------------- */
/* Validate, plan and run one job; returns when every requested output is written.  Inputs are read
 * before the call returns and may be freed afterwards.  `st` may be NULL. */
int32_t ps_compute(ps_ctx* ctx, const ps_job* job, ps_job_stats* st);

/* ---- serving -------------------------------------------------------------------------------- */
/* Queue a job (inputs are copied before return; output buffers must stay valid until ps_wait
 * returns for the ticket).  Jobs are admitted in arrival order as device memory frees up and run
 * concurrently on the device (continuous batching, up to four at once).  The serving slots and the
 * arena ps_compute keeps on the context share the context's budget.  PS_E_NOMEM if the job can
 * never fit the budget.  One thread may submit while another waits. */
int32_t ps_submit(ps_ctx* ctx, const ps_job* job, uint64_t* ticket);
/* Wait for a ticket (timeout_us < 0: forever).  Returns the job's own status, or PS_E_TIMEOUT. */
int32_t ps_wait(ps_ctx* ctx, uint64_t ticket, int64_t timeout_us, ps_job_stats* st);

/* ---- inspection hooks ----------------------------------------------------------------------- */
/* Points and weights of grid G(A,B|C) (C = -1: unrefined) as computed on the device, in the global
 * frame: xyzw[4*i+0..3] = x, y, z, w.  Pass xyzw = NULL to query *n_points only.  Host memory. */
int32_t ps_grid_points(ps_ctx* ctx, const ps_atom* atoms, int32_t n_atoms, int32_t A, int32_t B,
                       int32_t C, const ps_grid_spec* spec, double* xyzw, int64_t* n_points);

/* Evaluate one function on host-provided points with the device kernels (what: 0 = chi,
 * 1 = -1/2 lap chi, 2 = Coulomb potential of chi).  Host arrays of length npts. */
int32_t ps_eval_function(ps_ctx* ctx, int32_t what, const ps_sto* fn, const double* center,
                         int64_t npts, const double* x, const double* y, const double* z,
                         double* out);

/* Work estimate of a job without running it: pair-points, grids, points and device bytes.  ctx may
 * be NULL (host-only planning with the default tiling and no memory budget; no GPU needed). */
int32_t ps_plan_work(ps_ctx* ctx, const ps_job* job, double* pair_points, int64_t* n_grids,
                     int64_t* n_points, size_t* device_bytes);

/* Contraction tile shape of the (ab|P) tiles for later jobs on this context.  wm, wn in {2, 4}: 16x16
 * MFMA blocks per wave along the pair and column dimensions (a work-group tile is 32*wm pairs x
 * 32*wn columns); stage_chunks in {1, 2}: 16-point chunks per LDS stage; ksplit: point-range splits
 * per tile (0 = sized to fill the device).  wm = wn = stage_chunks = 0 restores the built-in default,
 * which depends on each job's precision (FP64: 4, 4, 1; mixed: 4, 4, 2); a 0 among non-zero values
 * takes the FP64 default for that field.  Two-index tiles (S, T, V, (P|Q)) always use 2, 2 with the
 * same stage_chunks.  PS_E_INVALID otherwise.  ps_compute reuses the plan of the previous job on the
 * context when the job's inputs, the tiling and the budget are unchanged. */
int32_t ps_set_tiling(ps_ctx* ctx, int32_t wm, int32_t wn, int32_t stage_chunks, int32_t ksplit);

/* Context options for later jobs; PS_E_INVALID for other options or values.
 *
 * PS_OPT_SHARE_THIRD_CENTRE (value -1 = automatic, the default: on for FP64 jobs, off for mixed ones;
 * 0 = off; 1 = on): cross-third-centre reuse of basis values.  The grids G(A,B|C) of one atom pair,
 * other than its pair grid, differ only by a rotation about the A-B axis (each places its C at
 * phi = 0, Section 2.3) and by the lines moved onto their C (Section 2.2); in the regular cells that
 * no such grid's moved lines
 * touch their points share (mu, nu, phi) and the distances to A and B.  With the option on, the
 * radial factors of A's and B's functions there are computed once for all of those grids and only
 * the angular factors per grid (grids with Q = 4 and at most 128 cells per axis, all of one pair in
 * one memory pass).  Results are unchanged to rounding.
 *
 * PS_OPT_OVERLAP_PASSES (value 0 = off, the default, also chosen by -1; 1 = on): for a job whose
 * per-point arrays do not fit the budget at once (more than one memory pass), the array budget is split
 * into two regions taken by alternate passes, and each pass's evaluation runs on a second stream of the
 * context while the previous pass's contraction runs.  Passes hold half as many grids.  Results are
 * unchanged to rounding (the reductions of the grids' contributions are grouped differently).  Off by
 * default: on MI355X the evaluation takes compute units from the contraction rather than filling idle
 * ones, and the smaller passes cost more than the overlap hides (hydrocarbon job: FP64 equal, mixed
 * 2.5% slower). */
enum { PS_OPT_SHARE_THIRD_CENTRE = 1, PS_OPT_OVERLAP_PASSES = 2 };
int32_t ps_set_option(ps_ctx* ctx, int32_t option, int64_t value);

/* Measured matrix-pipe throughput of the context's device, for reading roofline fractions against
 * what the chip sustains: a probe kernel in which every wave (16 per compute unit) issues long runs of
 * independent 16x16x4 MFMAs (FP64 for PS_PREC_FP64, FP32 for PS_PREC_MIXED) on register operands;
 * *tflops receives the best of three timed runs, in TFLOP/s (2048 FLOPs per MFMA).  Runs on the
 * context's synchronous stream (about 10 ms of device time); PS_E_INVALID for other precisions. */
int32_t ps_mfma_rate(ps_ctx* ctx, int32_t precision, double* tflops);

/* ---- tile-shape autotuner ------------------------------------------------------------------- */
typedef struct {
  int32_t wm, wn, stage_chunks, ksplit; /* as ps_set_tiling                                         */
  double device_ms;                     /* best device time of the job (first -> last kernel), ms    */
  double contract_ms;                   /* contraction kernels within that run, ms                    */
} ps_tuning;

/* Time the job's device work `reps` times (reps >= 1) under each candidate tiling (wm, wn in {2, 4},
 * stage_chunks in {1, 2}, ksplit 0), keep the fastest on the context as ps_set_tiling would, and
 * return it in *best.  The job's output buffers are not written.  `table` (may be NULL when
 * max_table is 0) receives up to max_table timed candidates in trial order, *n_table (may be NULL)
 * their number.  A candidate whose workspace exceeds the budget is skipped; PS_E_NOMEM if all are.
 * Errors in the job itself return as from ps_compute and leave the tiling unchanged. */
int32_t ps_autotune(ps_ctx* ctx, const ps_job* job, int32_t reps, ps_tuning* best, ps_tuning* table,
                    int32_t max_table, int32_t* n_table);

/* ---- RI assembly (eq. 14) ------------------------------------------------------------------ */
/* The paper's RI form of the electron-repulsion integrals, (ab|cd) ~ sum_PQ (ab|P) [(P|Q)^-1] (Q|cd),
 * evaluated through the Cholesky factor (P|Q) = L L^T:
 *   B[R][ab]   = sum_P (L^-1)[R][P] (ab|P)     (forward substitution, FP64)
 *   eri[ab][cd] = sum_R B[R][ab] B[R][cd]      (FP64 MFMA, symmetric)
 * over canonical pairs a >= b, ab = a(a+1)/2 + b, n_pair = n_bf(n_bf+1)/2.
 * Inputs as ps_compute writes them: abP [P][a][b] (n_aux x n_bf x n_bf), L n_aux x n_aux lower
 * (the upper triangle is not read).  Outputs (NULL = not wanted): B n_aux x n_pair and eri
 * n_pair x n_pair, row-major FP64.  All four arrays live on the host (location PS_OUT_HOST) or on
 * the context's device (PS_OUT_DEVICE).  Device scratch comes from the context's device memory
 * (the budget jobs use; returned to it when the call ends); PS_E_NOMEM if it does not fit.  Runs on
 * the context's synchronous stream, one call at a time with ps_compute and ps_autotune.  *device_ms
 * (may be NULL) receives the kernels' time. */
int32_t ps_ri_assemble(ps_ctx* ctx, int32_t n_bf, int32_t n_aux, int32_t location, const double* abP,
                       const double* L, double* B, double* eri, double* device_ms);

/* ---- allocation-free RI assembly ----------------------------------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same computation and layouts as ps_ri_assemble with all four
 * arrays on the context's device (abP, L inputs; B, eri outputs, NULL = not wanted), but the call's
 * scratch -- the gathered (ab|P) rows and B (n_aux x n_pair each; no B scratch when B is given), the
 * transformed factor (n_aux x n_aux) and the product's tile list -- lives in a static device array of
 * PS_RI_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU the library runs on until the process ends.
 * Nothing is allocated: no hipMalloc, hipFree or context memory.  Sizes whose scratch exceeds the
 * array return PS_E_NOMEM with the need in ps_last_error.  The kernels are enqueued on the context's
 * synchronous stream and the call returns without waiting: the outputs are ready when that stream
 * reaches this point.  Every call on one GPU shares that GPU's array: calls on one context run in
 * order on its stream, but calls that can overlap on one GPU (other contexts or streams) race. */
#define PS_RI_NOALLOC_SCRATCH_BYTES (64u << 20)
int32_t ps_ri_assemble_noalloc(ps_ctx* ctx, int32_t n_bf, int32_t n_aux, const double* abP, const double* L,
                               double* B, double* eri);

const char* ps_status_string(int32_t status);
/* Last error text of the context (valid until the next call on it); ctx may be NULL. */
const char* ps_last_error(ps_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PSINT_H */
