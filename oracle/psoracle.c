/*
 * psoracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see psoracle.h).
 *
 * Everything here is a direct transcription of the definitions in the paper (arXiv 2510.15204):
 * straightforward loops over grids, points and functions in double precision, with no blocking,
 * fusion or reordering beyond what the definitions state.  Where the paper is silent the reading
 * used is stated next to the code.
 */
#include "psoracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------------ */
/* Small helpers                                                                              */
/* ------------------------------------------------------------------------------------------ */

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

static double dist3(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return (int32_t)omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1, 1] (Section 2.1: GL quadrature in every cell and axis).         */
/* Newton iteration on P_q from the usual cosine initial guesses.                              */
/* ------------------------------------------------------------------------------------------ */

int orc_gauss_legendre(int32_t q, double* x, double* w) {
  if (q < 1 || q > 64) return -1;
  for (int i = 0; i < q; ++i) {
    double t = cos(PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = t; p0 = 1.0; }
      /* p1 = P_q(t), p0 = P_{q-1}(t) */
      dp = q * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    /* recompute derivative at the converged node for the weight */
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = t; p0 = 1.0; }
    dp = q * (t * p1 - p0) / (t * t - 1.0);
    x[q - 1 - i] = t;  /* ascending order */
    w[q - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Grid G(A,B|C): Sections 2.1-2.3, eqs. 2-7, 10-12, 17, Algorithms 1-2.                       */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
  double a;                 /* half the A-B distance (eqs. 2-4) */
  double M[3];              /* midpoint */
  double ex[3], ey[3], ez[3];
  int nmu, nnu, nphi, q, nsp;
  double *mu, *nu, *phi;    /* line positions, n+1 each */
  int moved_mu, moved_nu, istar, jstar, split;
} orc_grid;

static void grid_free(orc_grid* g) {
  free(g->mu);
  free(g->nu);
  free(g->phi);
  g->mu = g->nu = g->phi = NULL;
}

static int spec_valid(const double* spec) {
  int nmu = (int)spec[0], nnu = (int)spec[1], nphi = (int)spec[2], q = (int)spec[3], nsp = (int)spec[4];
  if (nmu < 2 || nnu < 2 || nphi < 2 || q < 1 || q > 16 || nsp < 1 || nsp > 8) return 0;
  if (!(spec[5] > 0.0)) return 0;
  return 1;
}

/* Build lines, frame and third-centre refinement.  A sits at local z = +a, B at -a. */
static int grid_build(const double* xyz, int n_atoms, int A, int B, int C, const double* spec,
                      orc_grid* g) {
  memset(g, 0, sizeof(*g));
  if (A < 0 || B < 0 || A >= n_atoms || B >= n_atoms || A == B) return -1;
  if (C >= n_atoms || C == A || C == B) return -1;
  if (!spec_valid(spec)) return -1;
  const double* RA = xyz + 3 * A;
  const double* RB = xyz + 3 * B;
  double R = dist3(RA, RB);
  if (!(R > 1e-3)) return -1;
  g->a = 0.5 * R;
  for (int d = 0; d < 3; ++d) {
    g->M[d] = 0.5 * (RA[d] + RB[d]);
    g->ez[d] = (RA[d] - RB[d]) / R;
  }
  g->nmu = (int)spec[0];
  g->nnu = (int)spec[1];
  g->nphi = (int)spec[2];
  g->q = (int)spec[3];
  g->nsp = (int)spec[4];

  /* Frame: the third centre goes to the phi = 0 half-plane (Section 2.3).  Without a usable third
   * centre (none, or on the axis) the reading is: the global unit vector least aligned with ez,
   * orthogonalised against ez.  A later axis wins only if it is less aligned by more than 1e-12, so
   * near-ties go to x, then y, then z whatever the rounding of ez. */
  int have_perp = 0;
  if (C >= 0) {
    double v[3], s = 0.0;
    for (int d = 0; d < 3; ++d) v[d] = xyz[3 * C + d] - g->M[d];
    for (int d = 0; d < 3; ++d) s += v[d] * g->ez[d];
    for (int d = 0; d < 3; ++d) v[d] -= s * g->ez[d];
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (n > 1e-10) {
      for (int d = 0; d < 3; ++d) g->ex[d] = v[d] / n;
      have_perp = 1;
    }
  }
  if (!have_perp) {
    int best = 0;
    for (int d = 1; d < 3; ++d)
      if (fabs(g->ez[d]) < fabs(g->ez[best]) - 1e-12) best = d;
    double u[3] = {0, 0, 0};
    u[best] = 1.0;
    double s = g->ez[best];
    for (int d = 0; d < 3; ++d) u[d] -= s * g->ez[d];
    double n = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) g->ex[d] = u[d] / n;
  }
  /* ey = ez x ex */
  g->ey[0] = g->ez[1] * g->ex[2] - g->ez[2] * g->ex[1];
  g->ey[1] = g->ez[2] * g->ex[0] - g->ez[0] * g->ex[2];
  g->ey[2] = g->ez[0] * g->ex[1] - g->ez[1] * g->ex[0];

  /* Lines: mu = C1 atanh(t), t uniform with step 1/(N_mu+1) (eqs. 7, 12, 17); nu, phi uniform. */
  g->mu = (double*)malloc(sizeof(double) * (g->nmu + 1));
  g->nu = (double*)malloc(sizeof(double) * (g->nnu + 1));
  g->phi = (double*)malloc(sizeof(double) * (g->nphi + 1));
  if (!g->mu || !g->nu || !g->phi) { grid_free(g); return -3; }
  double C1 = spec[5] * pow(g->a, spec[6]);
  for (int i = 0; i <= g->nmu; ++i) g->mu[i] = C1 * atanh((double)i / (g->nmu + 1));
  for (int j = 0; j <= g->nnu; ++j) g->nu[j] = PI * j / g->nnu;
  for (int k = 0; k <= g->nphi; ++k) g->phi[k] = 2.0 * PI * k / g->nphi;

  /* Third centre: move the nearest interior mu and nu lines onto it (Sections 2.2-2.3). */
  if (C >= 0) {
    const double* RC = xyz + 3 * C;
    double dp = dist3(RC, RA), dm = dist3(RC, RB);
    double ch = (dp + dm) / (2.0 * g->a);
    if (ch < 1.0) ch = 1.0;
    double muC = acosh(ch);
    double cn = (dm - dp) / (2.0 * g->a);
    if (cn > 1.0) cn = 1.0;
    if (cn < -1.0) cn = -1.0;
    double nuC = acos(cn);
    if (muC > 0.0 && muC < g->mu[g->nmu]) {
      int best = 1;
      for (int i = 2; i <= g->nmu - 1; ++i)
        if (fabs(g->mu[i] - muC) < fabs(g->mu[best] - muC)) best = i;
      g->mu[best] = muC;
      g->istar = best;
      g->moved_mu = 1;
    }
    if (nuC > 0.0 && nuC < PI) {
      int best = 1;
      for (int j = 2; j <= g->nnu - 1; ++j)
        if (fabs(g->nu[j] - nuC) < fabs(g->nu[best] - nuC)) best = j;
      g->nu[best] = nuC;
      g->jstar = best;
      g->moved_nu = 1;
    }
    g->split = (g->moved_mu && g->moved_nu && g->nsp >= 2);
  }
  return 0;
}

/* Is cell (i,j,k) one of the 8 cells touching the third centre (corner at mu*, nu*, phi = 0)? */
static int cell_is_split(const orc_grid* g, int i, int j, int k) {
  if (!g->split) return 0;
  int ok_i = (i == g->istar - 1 || i == g->istar);
  int ok_j = (j == g->jstar - 1 || j == g->jstar);
  int ok_k = (k == g->nphi - 1 || k == 0);
  return ok_i && ok_j && ok_k;
}

static int64_t grid_count(const orc_grid* g) {
  int64_t cells = (int64_t)g->nmu * g->nnu * g->nphi;
  if (g->split) cells += 8 * ((int64_t)g->nsp * g->nsp * g->nsp - 1);
  return cells * g->q * g->q * g->q;
}

/* Enumerate points: cells in (i,j,k) order, subcells in (s_mu, s_nu, s_phi) order, then GL nodes
 * (p,q,r).  Weight (eqs. 10-11 with the standard affine GL map on each axis):
 *   w = (dmu/2 g_p)(dnu/2 g_q)(dphi/2 g_r) a^3 sinh(mu) sin(nu) (sinh^2 mu + sin^2 nu). */
static void grid_points(const orc_grid* g, double* X, double* Y, double* Zc, double* W) {
  double gx[16], gw[16];
  orc_gauss_legendre(g->q, gx, gw);
  int Q = g->q;
  int64_t idx = 0;
  double a = g->a;
  for (int i = 0; i < g->nmu; ++i)
    for (int j = 0; j < g->nnu; ++j)
      for (int k = 0; k < g->nphi; ++k) {
        int ns = cell_is_split(g, i, j, k) ? g->nsp : 1;
        for (int si = 0; si < ns; ++si)
          for (int sj = 0; sj < ns; ++sj)
            for (int sk = 0; sk < ns; ++sk) {
              double mlo = g->mu[i] + (g->mu[i + 1] - g->mu[i]) * si / ns;
              double mhi = g->mu[i] + (g->mu[i + 1] - g->mu[i]) * (si + 1) / ns;
              double nlo = g->nu[j] + (g->nu[j + 1] - g->nu[j]) * sj / ns;
              double nhi = g->nu[j] + (g->nu[j + 1] - g->nu[j]) * (sj + 1) / ns;
              double plo = g->phi[k] + (g->phi[k + 1] - g->phi[k]) * sk / ns;
              double phi_hi = g->phi[k] + (g->phi[k + 1] - g->phi[k]) * (sk + 1) / ns;
              for (int p = 0; p < Q; ++p)
                for (int qq = 0; qq < Q; ++qq)
                  for (int r = 0; r < Q; ++r) {
                    double mu = 0.5 * (mlo + mhi) + 0.5 * (mhi - mlo) * gx[p];
                    double nu = 0.5 * (nlo + nhi) + 0.5 * (nhi - nlo) * gx[qq];
                    double ph = 0.5 * (plo + phi_hi) + 0.5 * (phi_hi - plo) * gx[r];
                    double sh = sinh(mu), chh = cosh(mu), sn = sin(nu), cs = cos(nu);
                    double w = (0.5 * (mhi - mlo) * gw[p]) * (0.5 * (nhi - nlo) * gw[qq]) *
                               (0.5 * (phi_hi - plo) * gw[r]) * a * a * a * sh * sn *
                               (sh * sh + sn * sn);
                    double lx = a * sh * sn * cos(ph);
                    double ly = a * sh * sn * sin(ph);
                    double lz = a * chh * cs;
                    X[idx] = g->M[0] + lx * g->ex[0] + ly * g->ey[0] + lz * g->ez[0];
                    Y[idx] = g->M[1] + lx * g->ex[1] + ly * g->ey[1] + lz * g->ez[1];
                    Zc[idx] = g->M[2] + lx * g->ex[2] + ly * g->ey[2] + lz * g->ez[2];
                    W[idx] = w;
                    ++idx;
                  }
            }
      }
}

int orc_grid_info(const double* xyz, int32_t n_atoms, int32_t A, int32_t B, int32_t C,
                  const double* spec, int64_t* info, double* mu, double* nu, double* phi,
                  double* frame) {
  orc_grid g;
  int rc = grid_build(xyz, n_atoms, A, B, C, spec, &g);
  if (rc) return rc;
  if (info) {
    info[0] = grid_count(&g);
    info[1] = g.moved_mu;
    info[2] = g.moved_nu;
    info[3] = g.split;
    info[4] = g.istar;
    info[5] = g.jstar;
    info[6] = (int64_t)g.nmu * g.nnu * g.nphi + (g.split ? 8 * ((int64_t)g.nsp * g.nsp * g.nsp - 1) : 0);
    info[7] = 0;
  }
  if (mu) memcpy(mu, g.mu, sizeof(double) * (g.nmu + 1));
  if (nu) memcpy(nu, g.nu, sizeof(double) * (g.nnu + 1));
  if (phi) memcpy(phi, g.phi, sizeof(double) * (g.nphi + 1));
  if (frame) {
    frame[0] = g.a;
    for (int d = 0; d < 3; ++d) {
      frame[1 + d] = g.M[d];
      frame[4 + d] = g.ex[d];
      frame[7 + d] = g.ey[d];
      frame[10 + d] = g.ez[d];
    }
  }
  grid_free(&g);
  return 0;
}

int orc_grid_points(const double* xyz, int32_t n_atoms, int32_t A, int32_t B, int32_t C,
                    const double* spec, double* x, double* y, double* z, double* w) {
  orc_grid g;
  int rc = grid_build(xyz, n_atoms, A, B, C, spec, &g);
  if (rc) return rc;
  grid_points(&g, x, y, z, w);
  grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Slater functions (eq. 1) with real orthonormal spherical harmonics (no Condon-Shortley      */
/* phase), built from the associated Legendre recurrence.                                     */
/* ------------------------------------------------------------------------------------------ */

/* P_l^m(x) for m >= 0 without the (-1)^m phase. */
static double assoc_legendre(int l, int m, double x) {
  double s = sqrt(fmax(0.0, (1.0 - x) * (1.0 + x)));
  double pmm = 1.0;
  for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * s;
  if (l == m) return pmm;
  double pm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pm1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
    pmm = pm1;
    pm1 = pll;
  }
  return pll;
}

/* Real Y_lm: m > 0 -> cos(m phi) branch, m < 0 -> sin(|m| phi) branch. */
static double real_ylm(int l, int m, double ct, double ph) {
  int am = m < 0 ? -m : m;
  double norm = sqrt((2.0 * l + 1.0) / (4.0 * PI) * factorial(l - am) / factorial(l + am));
  double p = assoc_legendre(l, am, ct);
  if (m == 0) return norm * p;
  if (m > 0) return sqrt(2.0) * norm * p * cos(am * ph);
  return sqrt(2.0) * norm * p * sin(am * ph);
}

/* STO normalisation N = (2 zeta)^(n + 1/2) / sqrt((2n)!) */
static double sto_norm(int n, double zeta) {
  return pow(2.0 * zeta, n + 0.5) / sqrt(factorial(2 * n));
}

double orc_upper_gamma(int32_t k, double x) {
  /* Gamma(k, x) = (k-1)! e^{-x} sum_{j<k} x^j / j!  (integer k >= 1) */
  double term = 1.0, sum = 1.0;
  for (int j = 1; j < k; ++j) {
    term *= x / j;
    sum += term;
  }
  return factorial(k - 1) * exp(-x) * sum;
}

double orc_lower_gamma(int32_t k, double x) {
  /* gamma(k, x): the series x^k e^{-x} sum_j x^j / (k (k+1) ... (k+j)) for x < k + 1 (no
   * cancellation), else (k-1)! - Gamma(k, x). */
  if (x <= 0.0) return 0.0;
  if (x < k + 1.0) {
    double term = 1.0 / k, sum = term;
    for (int j = 1; j < 2000; ++j) {
      term *= x / (k + j);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    return pow(x, k) * exp(-x) * sum;
  }
  return factorial(k - 1) - orc_upper_gamma(k, x);
}

/* what: 0 chi, 1 -1/2 lap chi, 2 Coulomb potential of chi, 3 Y_lm only */
static double eval_one(int what, int n, int l, int m, double zeta, double dx, double dy, double dz) {
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double ct = r > 0.0 ? dz / r : 1.0;
  double ph = (dx == 0.0 && dy == 0.0) ? 0.0 : atan2(dy, dx);
  double Y = real_ylm(l, m, ct, ph);
  if (what == 3) return Y;
  double N = sto_norm(n, zeta);
  if (what == 2) {
    /* Potential of N r^{n-1} e^{-zeta r} Y_lm by the multipole expansion of a single (l,m) density:
     * V = 4 pi/(2l+1) N zeta^{-(n+1)} Y_lm [x^{-l-1} gamma(n+l+2, x) + x^l Gamma(n-l+1, x)], x = zeta r. */
    double x = zeta * r;
    double pre = 4.0 * PI / (2.0 * l + 1.0) * N * pow(zeta, -(n + 1.0)) * Y;
    if (r == 0.0) return l == 0 ? pre * factorial(n) : 0.0;
    double inner = pow(x, -(l + 1.0)) * orc_lower_gamma(n + l + 2, x);
    double outer = pow(x, (double)l) * orc_upper_gamma(n - l + 1, x);
    return pre * (inner + outer);
  }
  double chi = N * pow(r, n - 1.0) * exp(-zeta * r) * Y;
  if (what == 0) return chi;
  /* lap chi / chi = zeta^2 - 2 zeta n / r + (n(n-1) - l(l+1)) / r^2 */
  double f = zeta * zeta - 2.0 * zeta * n / r + (n * (n - 1.0) - l * (l + 1.0)) / (r * r);
  return -0.5 * f * chi;
}

static int fn_valid(const double* fn, int n_atoms) {
  int atom = (int)fn[0], n = (int)fn[1], l = (int)fn[2], m = (int)fn[3];
  if (atom < 0 || atom >= n_atoms) return 0;
  if (n < 1 || l < 0 || l >= n || m < -l || m > l) return 0;
  if (!(fn[4] > 0.0) || !isfinite(fn[4])) return 0;
  return 1;
}

int orc_eval(int32_t what, const double* fn, const double* center, int64_t npts, const double* x,
             const double* y, const double* z, double* out) {
  int n = (int)fn[1], l = (int)fn[2], m = (int)fn[3];
  if (n < 1 || l < 0 || l >= n || m < -l || m > l || !(fn[4] > 0.0)) return -1;
  for (int64_t i = 0; i < npts; ++i)
    out[i] = eval_one(what, n, l, m, fn[4], x[i] - center[0], y[i] - center[1], z[i] - center[2]);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Routing of integrals to grids (3-atom subsets; the paper builds polyatomics from them).     */
/* Readings: N = 2 uses one unrefined grid.  N >= 3 uses G(A,B|C) for every pair and every     */
/* third atom; the "pair grid" of (X,Y) is G(X,Y|C*) with C* the atom nearest the midpoint;    */
/* one-centre blocks of X live on the pair grid of X and its nearest neighbour nn(X).  "Nearest" */
/* counts distances equal within 1e-10 bohr as ties, broken by the lower atom index.            */
/* ------------------------------------------------------------------------------------------ */

static int nearest_atom(const orc_job* J, int X) {
  int best = -1;
  double bd = 0.0;
  for (int c = 0; c < J->n_atoms; ++c) {
    if (c == X) continue;
    double d = dist3(J->xyz + 3 * X, J->xyz + 3 * c);
    if (best < 0 || d < bd - 1e-10) { best = c; bd = d; }
  }
  return best;
}

static int nearest_to_midpoint(const orc_job* J, int A, int B) {
  double M[3];
  for (int d = 0; d < 3; ++d) M[d] = 0.5 * (J->xyz[3 * A + d] + J->xyz[3 * B + d]);
  int best = -1;
  double bd = 0.0;
  for (int c = 0; c < J->n_atoms; ++c) {
    if (c == A || c == B) continue;
    double d = dist3(M, J->xyz + 3 * c);
    if (best < 0 || d < bd - 1e-10) { best = c; bd = d; }
  }
  return best;
}

typedef struct { int A, B, C; } gkey;

static gkey pair_grid(const orc_job* J, int X, int Y) {
  gkey k;
  k.A = X < Y ? X : Y;
  k.B = X < Y ? Y : X;
  k.C = J->n_atoms >= 3 ? nearest_to_midpoint(J, k.A, k.B) : -1;
  return k;
}

static gkey third_grid(int X, int Y, int Z) {
  gkey k;
  k.A = X < Y ? X : Y;
  k.B = X < Y ? Y : X;
  k.C = Z;
  return k;
}

int64_t orc_grid_list(const orc_job* J, int32_t* abc, int64_t cap) {
  int64_t cnt = 0;
  int N = J->n_atoms;
  for (int A = 0; A < N; ++A)
    for (int B = A + 1; B < N; ++B) {
      if (N == 2) {
        if (abc && cnt < cap) { abc[3 * cnt] = A; abc[3 * cnt + 1] = B; abc[3 * cnt + 2] = -1; }
        ++cnt;
        continue;
      }
      for (int C = 0; C < N; ++C) {
        if (C == A || C == B) continue;
        if (abc && cnt < cap) { abc[3 * cnt] = A; abc[3 * cnt + 1] = B; abc[3 * cnt + 2] = C; }
        ++cnt;
      }
    }
  return cnt;
}

/* One contribution of an element: grid + operator details.  nuc = list of nuclei for V. */
typedef struct {
  gkey g;
  int n_nuc;
  int nuc[2];
} contrib;

/* Fill the contributions of one element; returns their count (<= 2 + n_atoms). */
static int route(const orc_job* J, int kind, int i, int j, int k, contrib* out) {
  int N = J->n_atoms, c = 0;
  if (kind == ORC_S || kind == ORC_T) {
    int X = (int)J->bf[5 * i], Y = (int)J->bf[5 * j];
    out[0].g = (X != Y) ? pair_grid(J, X, Y) : pair_grid(J, X, nearest_atom(J, X));
    out[0].n_nuc = 0;
    return 1;
  }
  if (kind == ORC_V) {
    int X = (int)J->bf[5 * i], Y = (int)J->bf[5 * j];
    if (X != Y) {
      out[c].g = pair_grid(J, X, Y);
      out[c].n_nuc = 2;
      out[c].nuc[0] = X;
      out[c].nuc[1] = Y;
      ++c;
      for (int C = 0; C < N; ++C) {
        if (C == X || C == Y) continue;
        out[c].g = third_grid(X, Y, C);
        out[c].n_nuc = 1;
        out[c].nuc[0] = C;
        ++c;
      }
    } else {
      int nn = nearest_atom(J, X);
      out[c].g = pair_grid(J, X, nn);
      out[c].n_nuc = 2;
      out[c].nuc[0] = X;
      out[c].nuc[1] = nn;
      ++c;
      for (int C = 0; C < N; ++C) {
        if (C == X || C == nn) continue;
        out[c].g = pair_grid(J, X, C);
        out[c].n_nuc = 1;
        out[c].nuc[0] = C;
        ++c;
      }
    }
    return c;
  }
  if (kind == ORC_PQ) {
    int X = (int)J->aux[5 * i], Y = (int)J->aux[5 * j];
    out[0].g = (X != Y) ? pair_grid(J, X, Y) : pair_grid(J, X, nearest_atom(J, X));
    out[0].n_nuc = 0;
    return 1;
  }
  /* ORC_ABP: a = i, b = j, P = k */
  {
    int X = (int)J->bf[5 * i], Y = (int)J->bf[5 * j], Zp = (int)J->aux[5 * k];
    if (X != Y)
      out[0].g = (Zp == X || Zp == Y) ? pair_grid(J, X, Y) : third_grid(X, Y, Zp);
    else
      out[0].g = (Zp == X) ? pair_grid(J, X, nearest_atom(J, X)) : pair_grid(J, X, Zp);
    out[0].n_nuc = 0;
    return 1;
  }
}

int orc_route(const orc_job* J, int32_t kind, int32_t i, int32_t j, int32_t k, int32_t* out,
              int32_t cap) {
  if (!J || kind < ORC_S || kind > ORC_ABP) return -1;
  int nmax1 = (kind == ORC_PQ) ? J->n_aux : J->n_bf;
  if (i < 0 || i >= nmax1 || j < 0 || j >= nmax1) return -1;
  if (kind == ORC_ABP && (k < 0 || k >= J->n_aux)) return -1;
  contrib* cb = (contrib*)malloc(sizeof(contrib) * (size_t)(2 + J->n_atoms));
  if (!cb) return -3;
  int n = route(J, kind, i, j, k, cb);
  for (int c = 0; c < n && c < cap; ++c) {
    int32_t* o = out + 6 * c;
    o[0] = cb[c].g.A;
    o[1] = cb[c].g.B;
    o[2] = cb[c].g.C;
    o[3] = cb[c].n_nuc;
    o[4] = cb[c].n_nuc > 0 ? cb[c].nuc[0] : -1;
    o[5] = cb[c].n_nuc > 1 ? cb[c].nuc[1] : -1;
  }
  free(cb);
  return n;
}

static const double* spec_for(const orc_job* J, int A, int B) {
  for (int p = 0; p < J->n_pair_specs; ++p) {
    int a = J->pair_ab[2 * p], b = J->pair_ab[2 * p + 1];
    if ((a == A && b == B) || (a == B && b == A)) return J->pair_spec + 7 * p;
  }
  return J->spec;
}

static int job_valid(const orc_job* J) {
  if (J->n_atoms < 2) return 0;
  for (int a = 0; a < J->n_atoms; ++a)
    for (int b = a + 1; b < J->n_atoms; ++b)
      if (!(dist3(J->xyz + 3 * a, J->xyz + 3 * b) > 1e-3)) return 0;
  for (int f = 0; f < J->n_bf; ++f)
    if (!fn_valid(J->bf + 5 * f, J->n_atoms)) return 0;
  for (int f = 0; f < J->n_aux; ++f)
    if (!fn_valid(J->aux + 5 * f, J->n_atoms)) return 0;
  if (!spec_valid(J->spec)) return 0;
  for (int p = 0; p < J->n_pair_specs; ++p)
    if (!spec_valid(J->pair_spec + 7 * p)) return 0;
  return 1;
}

/* Columns of function values on the points of one grid, computed on demand. */
typedef struct {
  int64_t np;
  const double *x, *y, *z;
  double** bval;  /* chi_a          [n_bf]   */
  double** kval;  /* -1/2 lap chi_a [n_bf]   */
  double** aval;  /* chi_P          [n_aux]  */
  double** vval;  /* V_P            [n_aux]  */
  double** rinv;  /* 1/|r - R_C|    [n_atoms] */
} columns;

static double* col_eval(const orc_job* J, const columns* c, int what, const double* fn) {
  double* out = (double*)malloc(sizeof(double) * (size_t)c->np);
  if (!out) return NULL;
  const double* R = J->xyz + 3 * (int)fn[0];
  int n = (int)fn[1], l = (int)fn[2], m = (int)fn[3];
  double zeta = fn[4];
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < c->np; ++g)
    out[g] = eval_one(what, n, l, m, zeta, c->x[g] - R[0], c->y[g] - R[1], c->z[g] - R[2]);
  return out;
}

static double* col_rinv(const orc_job* J, const columns* c, int C) {
  double* out = (double*)malloc(sizeof(double) * (size_t)c->np);
  if (!out) return NULL;
  const double* R = J->xyz + 3 * C;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < c->np; ++g) {
    double dx = c->x[g] - R[0], dy = c->y[g] - R[1], dz = c->z[g] - R[2];
    out[g] = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  }
  return out;
}

int orc_compute_elements(const orc_job* J, int64_t n_el, const int32_t* kind, const int32_t* I,
                         const int32_t* Jx, const int32_t* K, double* out, double* work_pp) {
  if (!job_valid(J)) return -1;
  for (int64_t e = 0; e < n_el; ++e) {
    int kd = kind[e];
    if (kd < ORC_S || kd > ORC_ABP) return -1;
    int nmax1 = (kd == ORC_PQ) ? J->n_aux : J->n_bf;
    if (I[e] < 0 || I[e] >= nmax1 || Jx[e] < 0 || Jx[e] >= nmax1) return -1;
    if (kd == ORC_ABP && (K[e] < 0 || K[e] >= J->n_aux)) return -1;
    out[e] = 0.0;
  }
  double wpp = 0.0;
  int64_t ng = orc_grid_list(J, NULL, 0);
  int32_t* glist = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)ng);
  orc_grid_list(J, glist, ng);
  int maxc = 2 + J->n_atoms;
  contrib* cb = (contrib*)malloc(sizeof(contrib) * (size_t)maxc);
  /* per-element contribution lists, precomputed */
  contrib* all = (contrib*)malloc(sizeof(contrib) * (size_t)maxc * (size_t)(n_el > 0 ? n_el : 1));
  int* nall = (int*)malloc(sizeof(int) * (size_t)(n_el > 0 ? n_el : 1));
  for (int64_t e = 0; e < n_el; ++e) {
    nall[e] = route(J, kind[e], I[e], Jx[e], K ? K[e] : 0, all + (size_t)maxc * e);
  }
  int rc = 0;
  for (int64_t gi = 0; gi < ng && rc == 0; ++gi) {
    gkey key = {glist[3 * gi], glist[3 * gi + 1], glist[3 * gi + 2]};
    /* which elements touch this grid? */
    int any = 0;
    for (int64_t e = 0; e < n_el && !any; ++e)
      for (int c = 0; c < nall[e]; ++c) {
        contrib* p = all + (size_t)maxc * e + c;
        if (p->g.A == key.A && p->g.B == key.B && p->g.C == key.C) { any = 1; break; }
      }
    if (!any) continue;
    orc_grid G;
    if (grid_build(J->xyz, J->n_atoms, key.A, key.B, key.C, spec_for(J, key.A, key.B), &G)) {
      rc = -1;
      break;
    }
    int64_t np = grid_count(&G);
    double* X = (double*)malloc(sizeof(double) * (size_t)np * 4);
    if (!X) { grid_free(&G); rc = -3; break; }
    double *Y = X + np, *Zc = X + 2 * np, *W = X + 3 * np;
    grid_points(&G, X, Y, Zc, W);
    grid_free(&G);
    columns cols;
    cols.np = np;
    cols.x = X;
    cols.y = Y;
    cols.z = Zc;
    cols.bval = (double**)calloc((size_t)J->n_bf, sizeof(double*));
    cols.kval = (double**)calloc((size_t)J->n_bf, sizeof(double*));
    cols.aval = (double**)calloc((size_t)(J->n_aux > 0 ? J->n_aux : 1), sizeof(double*));
    cols.vval = (double**)calloc((size_t)(J->n_aux > 0 ? J->n_aux : 1), sizeof(double*));
    cols.rinv = (double**)calloc((size_t)J->n_atoms, sizeof(double*));
    /* pass 1: evaluate every column this grid needs (serial over columns, parallel over points) */
    for (int64_t e = 0; e < n_el; ++e)
      for (int c = 0; c < nall[e]; ++c) {
        contrib* p = all + (size_t)maxc * e + c;
        if (!(p->g.A == key.A && p->g.B == key.B && p->g.C == key.C)) continue;
        int kd = kind[e], i = I[e], j = Jx[e];
        if (kd == ORC_S || kd == ORC_V || kd == ORC_T || kd == ORC_ABP) {
          if (!cols.bval[i]) cols.bval[i] = col_eval(J, &cols, 0, J->bf + 5 * i);
          if (!cols.bval[j]) cols.bval[j] = col_eval(J, &cols, 0, J->bf + 5 * j);
        }
        if (kd == ORC_T) {
          if (!cols.kval[i]) cols.kval[i] = col_eval(J, &cols, 1, J->bf + 5 * i);
          if (!cols.kval[j]) cols.kval[j] = col_eval(J, &cols, 1, J->bf + 5 * j);
        }
        if (kd == ORC_V)
          for (int t = 0; t < p->n_nuc; ++t)
            if (!cols.rinv[p->nuc[t]]) cols.rinv[p->nuc[t]] = col_rinv(J, &cols, p->nuc[t]);
        if (kd == ORC_PQ) {
          if (!cols.aval[i]) cols.aval[i] = col_eval(J, &cols, 0, J->aux + 5 * i);
          if (!cols.aval[j]) cols.aval[j] = col_eval(J, &cols, 0, J->aux + 5 * j);
          if (!cols.vval[i]) cols.vval[i] = col_eval(J, &cols, 2, J->aux + 5 * i);
          if (!cols.vval[j]) cols.vval[j] = col_eval(J, &cols, 2, J->aux + 5 * j);
        }
        if (kd == ORC_ABP) {
          int P = K[e];
          if (!cols.vval[P]) cols.vval[P] = col_eval(J, &cols, 2, J->aux + 5 * P);
        }
      }
    /* pass 2: the quadrature sums of eq. 9, one element at a time */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : wpp)
    for (int64_t e = 0; e < n_el; ++e) {
      int counted = 0;
      for (int c = 0; c < nall[e]; ++c) {
        contrib* p = all + (size_t)maxc * e + c;
        if (!(p->g.A == key.A && p->g.B == key.B && p->g.C == key.C)) continue;
        if (!counted) { wpp += (double)np; counted = 1; }
        int kd = kind[e], i = I[e], j = Jx[e];
        double s = 0.0;
        if (kd == ORC_S) {
          const double *fa = cols.bval[i], *fb = cols.bval[j];
          for (int64_t g = 0; g < np; ++g) s += W[g] * fa[g] * fb[g];
        } else if (kd == ORC_T) {
          const double *fa = cols.bval[i], *fb = cols.bval[j], *ka = cols.kval[i], *kb = cols.kval[j];
          for (int64_t g = 0; g < np; ++g) s += W[g] * 0.5 * (fa[g] * kb[g] + ka[g] * fb[g]);
        } else if (kd == ORC_V) {
          const double *fa = cols.bval[i], *fb = cols.bval[j];
          for (int64_t g = 0; g < np; ++g) {
            double pot = 0.0;
            for (int t = 0; t < p->n_nuc; ++t) pot -= J->Z[p->nuc[t]] * cols.rinv[p->nuc[t]][g];
            s += W[g] * fa[g] * fb[g] * pot;
          }
        } else if (kd == ORC_PQ) {
          const double *ai = cols.aval[i], *aj = cols.aval[j], *vi = cols.vval[i], *vj = cols.vval[j];
          for (int64_t g = 0; g < np; ++g) s += W[g] * 0.5 * (vi[g] * aj[g] + vj[g] * ai[g]);
        } else {
          const double *fa = cols.bval[i], *fb = cols.bval[j], *vp = cols.vval[K[e]];
          for (int64_t g = 0; g < np; ++g) s += W[g] * fa[g] * fb[g] * vp[g];
        }
        out[e] += s;
      }
    }
    for (int f = 0; f < J->n_bf; ++f) { free(cols.bval[f]); free(cols.kval[f]); }
    for (int f = 0; f < J->n_aux; ++f) { free(cols.aval[f]); free(cols.vval[f]); }
    for (int a = 0; a < J->n_atoms; ++a) free(cols.rinv[a]);
    free(cols.bval);
    free(cols.kval);
    free(cols.aval);
    free(cols.vval);
    free(cols.rinv);
    free(X);
  }
  free(glist);
  free(cb);
  free(all);
  free(nall);
  if (work_pp) *work_pp = wpp;
  return rc;
}

/* A pivot no larger than 1e-14 times the original diagonal entry is taken as zero: the metric is
 * then singular to working precision (e.g. duplicated auxiliary functions) and reported as not
 * positive definite. */
int orc_cholesky(int32_t n, const double* A, double* L) {
  for (int64_t i = 0; i < (int64_t)n * n; ++i) L[i] = A[i];
  for (int k = 0; k < n; ++k) {
    double d = L[(int64_t)k * n + k];
    if (!(d > 1e-14 * A[(int64_t)k * n + k])) return -5;
    d = sqrt(d);
    L[(int64_t)k * n + k] = d;
    for (int i = k + 1; i < n; ++i) L[(int64_t)i * n + k] /= d;
    for (int j = k + 1; j < n; ++j)
      for (int i = j; i < n; ++i)
        L[(int64_t)i * n + j] -= L[(int64_t)i * n + k] * L[(int64_t)j * n + k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) L[(int64_t)i * n + j] = 0.0;
  return 0;
}

int orc_compute_full(const orc_job* J, double* S, double* T, double* V, double* PQ, double* PQ_chol,
                     double* abP, double* work_pp) {
  if (!job_valid(J)) return -1;
  int nb = J->n_bf, na = J->n_aux;
  int64_t nsym = (int64_t)nb * (nb + 1) / 2, nasym = (int64_t)na * (na + 1) / 2;
  int64_t total = 0;
  if (S) total += nsym;
  if (T) total += nsym;
  if (V) total += nsym;
  if (PQ || PQ_chol) total += nasym;
  if (abP) total += nsym * na;
  int32_t* kd = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1) * 4);
  double* val = (double*)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
  if (!kd || !val) { free(kd); free(val); return -3; }
  int32_t *ii = kd + total, *jj = kd + 2 * total, *kk = kd + 3 * total;
  int64_t e = 0;
  int kinds[3] = {ORC_S, ORC_T, ORC_V};
  double* mats[3] = {S, T, V};
  for (int t = 0; t < 3; ++t) {
    if (!mats[t]) continue;
    for (int i = 0; i < nb; ++i)
      for (int j = i; j < nb; ++j) { kd[e] = kinds[t]; ii[e] = i; jj[e] = j; kk[e] = 0; ++e; }
  }
  if (PQ || PQ_chol)
    for (int i = 0; i < na; ++i)
      for (int j = i; j < na; ++j) { kd[e] = ORC_PQ; ii[e] = i; jj[e] = j; kk[e] = 0; ++e; }
  if (abP)
    for (int P = 0; P < na; ++P)
      for (int i = 0; i < nb; ++i)
        for (int j = i; j < nb; ++j) { kd[e] = ORC_ABP; ii[e] = i; jj[e] = j; kk[e] = P; ++e; }
  int rc = orc_compute_elements(J, total, kd, ii, jj, kk, val, work_pp);
  if (rc) { free(kd); free(val); return rc; }
  double* pq = PQ;
  double* tmp = NULL;
  if (!pq && PQ_chol) { tmp = (double*)malloc(sizeof(double) * (size_t)na * na); pq = tmp; }
  for (int64_t q = 0; q < total; ++q) {
    int i = ii[q], j = jj[q];
    switch (kd[q]) {
      case ORC_S: case ORC_T: case ORC_V: {
        double* M = kd[q] == ORC_S ? S : (kd[q] == ORC_T ? T : V);
        M[(int64_t)i * nb + j] = val[q];
        M[(int64_t)j * nb + i] = val[q];
        break;
      }
      case ORC_PQ:
        pq[(int64_t)i * na + j] = val[q];
        pq[(int64_t)j * na + i] = val[q];
        break;
      default: {
        int64_t base = (int64_t)kk[q] * nb * nb;
        abP[base + (int64_t)i * nb + j] = val[q];
        abP[base + (int64_t)j * nb + i] = val[q];
      }
    }
  }
  if (PQ_chol) rc = orc_cholesky(na, pq, PQ_chol);
  free(tmp);
  free(kd);
  free(val);
  return rc;
}
