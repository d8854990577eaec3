/*
 * psoracle.h -- plain FP64 CPU oracle for Slater-orbital integrals on prolate spheroidal grids.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct reference that the GPU
 * library is checked against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never links, calls or falls back to it.  It shares no
 * code, headers or tables with the GPU library.
 *
 * Method: Stark, Meier, Hatch, Kammeraad, Dang, Zimmerman, "Numerical Integration of Slater Basis
 * Functions Over Prolate Spheroidal Grids" (arXiv 2510.15204):
 *   - STO definition: eq. 1
 *   - prolate spheroidal map and focus distances: eqs. 2-6 (Section 2.1)
 *   - radial stretching mu = C1 atanh(t): eq. 7, uniform t spacing: eq. 12, C1 = 2.3 a^(1/4): eq. 17
 *   - quadrature sum and weights: eqs. 9-11, Algorithms 1 and 2
 *   - third-centre line moving and N_SP split: Sections 2.2-2.3, Figure 2
 *   - Coulomb 3-index integrals through the potential of an auxiliary STO: eqs. 15-16
 *   - RI metric used with its inverse: eq. 14
 *
 * Pins: closed forms, library routines and an independent 2-D quadrature fix every one- and
 * two-centre value and the three-centre values of collinear atoms.  Three-centre values with the
 * third centre off the pair axis have no closed form: an independent 3-D integration (a fuzzy-cell
 * partition of space with a spherical grid per atom) fixes them to the grid's own error, and the
 * point-charge limit of (ab|P) fixes their leading behaviour.
 *
 * Units: bohr, hartree.  Functions are passed as rows (atom, n, l, m, zeta) of doubles.
 * All functions return 0 on success and a negative code on invalid input.
 */
#ifndef PSORACLE_H
#define PSORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element kinds for orc_compute_elements. */
enum { ORC_S = 0, ORC_T = 1, ORC_V = 2, ORC_PQ = 3, ORC_ABP = 4 };

typedef struct {
  int32_t n_atoms;
  const double* xyz;       /* n_atoms*3 */
  const double* Z;         /* n_atoms   */
  int32_t n_bf;
  const double* bf;        /* n_bf*5: atom, n, l, m, zeta */
  int32_t n_aux;
  const double* aux;       /* n_aux*5 */
  double spec[7];          /* default grid: n_mu, n_nu, n_phi, q, n_sp, c1_scale, c1_exp */
  int32_t n_pair_specs;
  const int32_t* pair_ab;  /* n_pair_specs*2 atom indices */
  const double* pair_spec; /* n_pair_specs*7, same order as spec */
} orc_job;

/* Gauss-Legendre nodes and weights on [-1,1], q <= 64. */
int orc_gauss_legendre(int32_t q, double* x, double* w);

/* Grid G(A,B|C) (C = -1: no third centre).  info[0..7] = n_points, moved_mu, moved_nu, split,
 * istar, jstar, n_cells, reserved.  lines: mu[n_mu+1], nu[n_nu+1], phi[n_phi+1] (may be NULL).
 * frame[13] = a, M(3), ex(3), ey(3), ez(3) (may be NULL). */
int orc_grid_info(const double* xyz, int32_t n_atoms, int32_t A, int32_t B, int32_t C,
                  const double* spec, int64_t* info, double* mu, double* nu, double* phi,
                  double* frame);
/* Points in the global frame and weights; arrays of length n_points. */
int orc_grid_points(const double* xyz, int32_t n_atoms, int32_t A, int32_t B, int32_t C,
                    const double* spec, double* x, double* y, double* z, double* w);

/* Pointwise evaluation of one function at npts global points.
 * what: 0 = chi, 1 = -1/2 lap chi, 2 = Coulomb potential of chi, 3 = real Y_lm of the direction. */
int orc_eval(int32_t what, const double* fn, const double* center, int64_t npts,
             const double* x, const double* y, const double* z, double* out);

/* Integer-order incomplete gamma functions (exposed for pins). */
double orc_lower_gamma(int32_t k, double x);
double orc_upper_gamma(int32_t k, double x);

/* Compute selected integrals.  kind[e] in ORC_*; (i,j,k) = (a,b,-) for S/T/V, (P,Q,-) for PQ,
 * (a,b,P) for ABP.  out[e] receives the value.  work_pp (nullable) receives the pair-point count
 * (sum over elements of the points of every distinct grid the element is summed on). */
int orc_compute_elements(const orc_job* job, int64_t n_el, const int32_t* kind, const int32_t* i,
                         const int32_t* j, const int32_t* k, double* out, double* work_pp);

/* All outputs (any pointer may be NULL).  S,T,V: n_bf^2 row-major; PQ, PQ_chol: n_aux^2 (lower L,
 * upper zeroed); abP: [P][a][b].  Returns -5 if (P|Q) is not positive definite (other outputs valid). */
int orc_compute_full(const orc_job* job, double* S, double* T, double* V, double* PQ,
                     double* PQ_chol, double* abP, double* work_pp);

/* Plain right-looking Cholesky, lower L (upper zeroed).  Returns -5 when a pivot is not larger than
 * 1e-14 times its original diagonal entry (not positive definite to working precision). */
int orc_cholesky(int32_t n, const double* A, double* L);

/* Grid routing (exposed for pins): list of grids of the job, as (A, B, C) triples.  Returns count. */
int64_t orc_grid_list(const orc_job* job, int32_t* abc, int64_t cap);

/* Routing of one element (exposed for pins): its contributions as rows (A, B, C, n_nuc, nuc0, nuc1)
 * -- the grid G(A,B|C) (C = -1: unrefined) it is summed on and, for V, the nuclei whose attraction is
 * summed there.  Writes at most cap rows; returns the number of contributions. */
int orc_route(const orc_job* job, int32_t kind, int32_t i, int32_t j, int32_t k, int32_t* out,
              int32_t cap);

/* OpenMP thread count (0 = leave the runtime default).  Returns the count in use. */
int32_t orc_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
