// Host planner.  See plan.h.  Everything here is FP64 host arithmetic on O(lines + functions) data;
// per-point work happens on the device.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

namespace psint {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

double dist(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

bool spec_ok(const ps_grid_spec& s, std::string* err) {
  if (s.n_mu < 2 || s.n_nu < 2 || s.n_phi < 2) { *err = "grid spec: n_mu, n_nu, n_phi must be >= 2"; return false; }
  if (s.q < 1 || s.q > 16) { *err = "grid spec: q must be in 1..16"; return false; }
  if (s.n_sp < 1 || s.n_sp > 8) { *err = "grid spec: n_sp must be in 1..8"; return false; }
  if (!(s.c1_scale > 0.0) || !std::isfinite(s.c1_scale) || !std::isfinite(s.c1_exp)) {
    *err = "grid spec: c1_scale must be > 0 and finite";
    return false;
  }
  return true;
}

int32_t fn_check(const ps_sto& f, int n_atoms, const char* what, int idx, std::string* err) {
  char buf[160];
  if (f.atom < 0 || f.atom >= n_atoms) {
    snprintf(buf, sizeof buf, "%s %d: atom index %d out of range", what, idx, f.atom);
    *err = buf;
    return PS_E_INVALID;
  }
  if (f.n < 1 || f.l < 0 || f.l >= f.n || f.m < -f.l || f.m > f.l || !(f.zeta > 0.0) || !std::isfinite(f.zeta)) {
    snprintf(buf, sizeof buf, "%s %d: invalid (n=%d, l=%d, m=%d, zeta=%g)", what, idx, f.n, f.l, f.m, f.zeta);
    *err = buf;
    return PS_E_INVALID;
  }
  if (f.l > LMAX || f.n > NMAX) {
    snprintf(buf, sizeof buf, "%s %d: l=%d or n=%d beyond the built kernels (l<=%d, n<=%d)", what, idx, f.l,
             f.n, LMAX, NMAX);
    *err = buf;
    return PS_E_UNSUPPORTED;
  }
  return PS_OK;
}

// Nearest other atom; distances equal within 1e-10 bohr count as ties, broken by the lower index.
int nearest_atom(const std::vector<ps_atom>& at, int X) {
  int best = -1;
  double bd = 0.0;
  for (int c = 0; c < (int)at.size(); ++c) {
    if (c == X) continue;
    double d = dist(at[X].xyz, at[c].xyz);
    if (best < 0 || d < bd - 1e-10) { best = c; bd = d; }
  }
  return best;
}

// Atom other than A, B nearest the A-B midpoint (same tie rule); -1 for a diatomic.
int nearest_to_mid(const std::vector<ps_atom>& at, int A, int B) {
  double M[3];
  for (int d = 0; d < 3; ++d) M[d] = 0.5 * (at[A].xyz[d] + at[B].xyz[d]);
  int best = -1;
  double bd = 0.0;
  for (int c = 0; c < (int)at.size(); ++c) {
    if (c == A || c == B) continue;
    double d = dist(M, at[c].xyz);
    if (best < 0 || d < bd - 1e-10) { best = c; bd = d; }
  }
  return best;
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Shells of one atom's functions (caller order preserved in column order).  Functions sharing
// (n, l, zeta) form one shell, at most one function per m; each entry keeps its m and output column.
struct ShellBuild {
  int n, l;
  double zeta;
  std::vector<std::pair<int, int>> ms;  // (m, column)
};

std::vector<ShellBuild> make_shells(const std::vector<ps_sto>& fns, const std::vector<int>& idx) {
  std::vector<ShellBuild> out;
  for (int c = 0; c < (int)idx.size(); ++c) {
    const ps_sto& f = fns[idx[c]];
    bool placed = false;
    for (auto& s : out) {
      // one column per m in a shell (a repeated function starts another shell)
      bool has_m = false;
      for (auto& mc : s.ms) has_m = has_m || mc.first == f.m;
      if (s.n == f.n && s.l == f.l && s.zeta == f.zeta && !has_m) {
        s.ms.push_back({f.m, c});
        placed = true;
        break;
      }
    }
    if (!placed) out.push_back({f.n, f.l, f.zeta, {{f.m, c}}});
  }
  return out;
}

}  // namespace

// Gauss-Legendre rule by the Golub-Welsch eigenproblem of the Jacobi matrix of the Legendre
// recurrence (nodes = eigenvalues, weights = 2 * first eigenvector component^2), solved with cyclic
// Jacobi rotations.
void gauss_legendre(int q, double* x, double* w) {
  double J[16][16] = {}, V[16][16] = {};
  for (int i = 0; i < q; ++i) V[i][i] = 1.0;
  for (int k = 1; k < q; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    J[k - 1][k] = J[k][k - 1] = b;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < q; ++i)
      for (int j = i + 1; j < q; ++j) off += J[i][j] * J[i][j];
    if (off < 1e-34) break;
    for (int p = 0; p < q; ++p)
      for (int r = p + 1; r < q; ++r) {
        if (J[p][r] == 0.0) continue;
        double theta = (J[r][r] - J[p][p]) / (2.0 * J[p][r]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < q; ++k) {  // J <- J G
          double jkp = J[k][p], jkr = J[k][r];
          J[k][p] = c * jkp - s * jkr;
          J[k][r] = s * jkp + c * jkr;
        }
        for (int k = 0; k < q; ++k) {  // J <- G^T J
          double jpk = J[p][k], jrk = J[r][k];
          J[p][k] = c * jpk - s * jrk;
          J[r][k] = s * jpk + c * jrk;
        }
        for (int k = 0; k < q; ++k) {
          double vkp = V[k][p], vkr = V[k][r];
          V[k][p] = c * vkp - s * vkr;
          V[k][r] = s * vkp + c * vkr;
        }
      }
  }
  std::vector<std::pair<double, double>> nw(q);
  for (int i = 0; i < q; ++i) nw[i] = {J[i][i], 2.0 * V[0][i] * V[0][i]};
  std::sort(nw.begin(), nw.end());
  // One Newton polish of each node on P_q (the eigenvalues are already accurate to rounding).
  for (int i = 0; i < q; ++i) {
    double t = nw[i].first;
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = q * (p0 - t * p1) / (1.0 - t * t);
    if (q > 1) t -= p1 / dp;
    x[i] = t;
    w[i] = nw[i].second;
  }
}

int32_t validate_job(const ps_job* job, std::string* err) {
  if (!job) { *err = "null job"; return PS_E_INVALID; }
  if (job->n_atoms < 2 || !job->atoms) { *err = "need at least two atoms"; return PS_E_INVALID; }
  if (job->n_bf < 0 || job->n_aux < 0) { *err = "negative function count"; return PS_E_INVALID; }
  if ((job->n_bf > 0 && !job->basis) || (job->n_aux > 0 && !job->aux)) { *err = "null function array"; return PS_E_INVALID; }
  if (job->precision != PS_PREC_FP64 && job->precision != PS_PREC_MIXED) { *err = "unknown precision"; return PS_E_INVALID; }
  if (job->out_location != PS_OUT_HOST && job->out_location != PS_OUT_DEVICE) { *err = "unknown output location"; return PS_E_INVALID; }
  for (int a = 0; a < job->n_atoms; ++a) {
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(job->atoms[a].xyz[d])) { *err = "non-finite coordinate"; return PS_E_INVALID; }
    if (!(job->atoms[a].Z >= 0.0) || !std::isfinite(job->atoms[a].Z)) { *err = "nuclear charge must be >= 0"; return PS_E_INVALID; }
    for (int b = a + 1; b < job->n_atoms; ++b)
      if (!(dist(job->atoms[a].xyz, job->atoms[b].xyz) > 1e-3)) {
        *err = "atoms closer than 1e-3 bohr";
        return PS_E_INVALID;
      }
  }
  for (int i = 0; i < job->n_bf; ++i) {
    int32_t rc = fn_check(job->basis[i], job->n_atoms, "basis function", i, err);
    if (rc) return rc;
  }
  for (int i = 0; i < job->n_aux; ++i) {
    int32_t rc = fn_check(job->aux[i], job->n_atoms, "aux function", i, err);
    if (rc) return rc;
  }
  if (!spec_ok(job->grid, err)) return PS_E_INVALID;
  if (job->n_pair_grids < 0 || (job->n_pair_grids > 0 && !job->pair_grids)) { *err = "bad pair grid list"; return PS_E_INVALID; }
  for (int p = 0; p < job->n_pair_grids; ++p) {
    const ps_pair_grid& pg = job->pair_grids[p];
    if (pg.atom_a < 0 || pg.atom_b < 0 || pg.atom_a >= job->n_atoms || pg.atom_b >= job->n_atoms ||
        pg.atom_a == pg.atom_b) {
      *err = "pair grid: bad atom pair";
      return PS_E_INVALID;
    }
    if (!spec_ok(pg.spec, err)) return PS_E_INVALID;
  }
  return PS_OK;
}

int32_t build_grid(const ps_atom* atoms, int n_atoms, int A, int B, int C, const ps_grid_spec& spec,
                   GridHost* g, std::string* err) {
  if (A < 0 || B < 0 || A >= n_atoms || B >= n_atoms || A == B || C >= n_atoms || C == A || C == B) {
    *err = "bad grid atoms";
    return PS_E_INVALID;
  }
  if (!spec_ok(spec, err)) return PS_E_INVALID;
  const double* RA = atoms[A].xyz;
  const double* RB = atoms[B].xyz;
  double R = dist(RA, RB);
  if (!(R > 1e-3)) { *err = "grid atoms coincide"; return PS_E_INVALID; }
  g->A = A;
  g->B = B;
  g->C = C;
  g->spec = spec;
  GridDev& d = g->dev;
  std::memset(&d, 0, sizeof d);
  d.a = 0.5 * R;
  double M[3];
  for (int k = 0; k < 3; ++k) {
    M[k] = 0.5 * (RA[k] + RB[k]);
    d.ez[k] = (RA[k] - RB[k]) / R;  // A at local +a
  }
  // Local x axis: towards the third centre's perpendicular offset (third centre at phi = 0), or,
  // without one, the global axis least aligned with ez (near-ties within 1e-12 go to x, y, z).
  bool have = false;
  double cperp = 0.0, cpar = 0.0;
  if (C >= 0) {
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = atoms[C].xyz[k] - M[k];
    cpar = v[0] * d.ez[0] + v[1] * d.ez[1] + v[2] * d.ez[2];
    for (int k = 0; k < 3; ++k) v[k] -= cpar * d.ez[k];
    double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (n > 1e-10) {
      for (int k = 0; k < 3; ++k) d.ex[k] = v[k] / n;
      cperp = n;
      have = true;
    }
  }
  if (!have) {
    int best = 0;
    for (int k = 1; k < 3; ++k)
      if (std::fabs(d.ez[k]) < std::fabs(d.ez[best]) - 1e-12) best = k;
    double u[3] = {0, 0, 0};
    u[best] = 1.0;
    double s = d.ez[best];
    for (int k = 0; k < 3; ++k) u[k] -= s * d.ez[k];
    double n = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int k = 0; k < 3; ++k) d.ex[k] = u[k] / n;
  }
  d.ey[0] = d.ez[1] * d.ex[2] - d.ez[2] * d.ex[1];
  d.ey[1] = d.ez[2] * d.ex[0] - d.ez[0] * d.ex[2];
  d.ey[2] = d.ez[0] * d.ex[1] - d.ez[1] * d.ex[0];
  d.nmu = spec.n_mu;
  d.nnu = spec.n_nu;
  d.nphi = spec.n_phi;
  d.q = spec.q;
  d.nsp = spec.n_sp;
  // Lines (eqs. 7, 12, 17): mu_i = C1 atanh(i / (N_mu + 1)); nu, phi uniform.
  double C1 = spec.c1_scale * std::pow(d.a, spec.c1_exp);
  g->mu.resize(d.nmu + 1);
  g->nu.resize(d.nnu + 1);
  g->phi.resize(d.nphi + 1);
  for (int i = 0; i <= d.nmu; ++i) g->mu[i] = C1 * std::atanh((double)i / (d.nmu + 1));
  for (int j = 0; j <= d.nnu; ++j) g->nu[j] = kPi * j / d.nnu;
  for (int k = 0; k <= d.nphi; ++k) g->phi[k] = 2.0 * kPi * k / d.nphi;
  bool mmu = false, mnu = false;
  if (C >= 0) {
    d.has_c = 1;
    d.cx = cperp;
    d.cz = cpar;
    // Third centre in (mu, nu): cosh mu = (r_A + r_B)/2a, cos nu = (r_B - r_A)/2a (eqs. 5-6).
    double rp = dist(atoms[C].xyz, RA), rm = dist(atoms[C].xyz, RB);
    double ch = std::max(1.0, (rp + rm) / (2.0 * d.a));
    double muC = std::acosh(ch);
    double cn = std::min(1.0, std::max(-1.0, (rm - rp) / (2.0 * d.a)));
    double nuC = std::acos(cn);
    // Move the nearest interior lines onto the third centre (Sections 2.2-2.3).
    if (muC > 0.0 && muC < g->mu[d.nmu]) {
      int best = 1;
      for (int i = 2; i < d.nmu; ++i)
        if (std::fabs(g->mu[i] - muC) < std::fabs(g->mu[best] - muC)) best = i;
      g->mu[best] = muC;
      d.istar = best;
      mmu = true;
    }
    if (nuC > 0.0 && nuC < kPi) {
      int best = 1;
      for (int j = 2; j < d.nnu; ++j)
        if (std::fabs(g->nu[j] - nuC) < std::fabs(g->nu[best] - nuC)) best = j;
      g->nu[best] = nuC;
      d.jstar = best;
      mnu = true;
    }
  }
  d.split = (mmu && mnu && d.nsp >= 2) ? 1 : 0;
  d.n_reg = (int64_t)d.nmu * d.nnu * d.nphi;
  int64_t cells = d.n_reg + (d.split ? 8 * ((int64_t)d.nsp * d.nsp * d.nsp - 1) : 0);
  d.npts = cells * d.q * d.q * d.q;
  d.npad = (d.npts + PAD_POINTS - 1) / PAD_POINTS * PAD_POINTS;
  return PS_OK;
}

// Launch order of a pass's tiles.  Work-groups are dispatched round-robin over the 8 XCDs
// (blockIdx mod 8), each with its own L2.  Tiles that stage the same Y columns over the same point
// range (same task, column tile and split; different pair-row tiles) form a group; a group is placed
// on one XCD's queue and its members get consecutive slots there, so they run together and share
// the Y columns in that XCD's L2.  Groups go to the least-loaded queue; the queues are then
// interleaved into blockIdx order.
// A tile's length in MFMA steps: its chunks times the MFMA blocks per wave of its shape (tiles of one
// single-shape launch all weigh 16 per chunk, so only their chunk counts order them).
static double tile_weight(const TileDev& t) {
  const int* m = kMergedShapes[t.shape & 7];
  return (double)t.nkc * m[0] * m[1];
}

static void xcd_order(std::vector<TileDev>& tiles, int t0, int t1) {
  constexpr int NX = 8;
  if (t1 - t0 <= NX) return;
  std::map<std::tuple<int, int, int64_t>, std::vector<int>> groups;
  std::vector<std::tuple<int, int, int64_t>> order_keys;
  for (int i = t0; i < t1; ++i) {
    const TileDev& t = tiles[i];
    auto key = std::make_tuple(t.task, t.p0, t.kc0);
    auto it = groups.find(key);
    if (it == groups.end()) {
      order_keys.push_back(key);
      groups[key] = {i};
    } else {
      it->second.push_back(i);
    }
  }
  // longest groups first (a group's tiles share one K range, so one length): each queue then runs
  // its longest tiles first and the short ones fill the end of the launch
  std::stable_sort(order_keys.begin(), order_keys.end(), [&](const auto& a, const auto& b) {
    return tile_weight(tiles[groups[a][0]]) > tile_weight(tiles[groups[b][0]]);
  });
  std::vector<std::vector<int>> q(NX);
  std::vector<double> load(NX, 0.0);
  for (auto& key : order_keys) {
    auto& g = groups[key];
    int best = 0;
    for (int x = 1; x < NX; ++x)
      if (load[x] < load[best]) best = x;
    for (int i : g) {
      q[best].push_back(i);
      load[best] += tile_weight(tiles[i]);
    }
  }
  std::vector<TileDev> out;
  out.reserve(t1 - t0);
  std::vector<size_t> pos(NX, 0);
  while ((int)out.size() < t1 - t0) {
    for (int x = 0; x < NX; ++x) {
      if (pos[x] < q[x].size()) {
        out.push_back(tiles[q[x][pos[x]++]]);
      } else {
        // this queue ran dry: take from the longest remaining one to keep blockIdx dense
        int lx = -1;
        size_t rem = 0;
        for (int y = 0; y < NX; ++y)
          if (q[y].size() - pos[y] > rem) { rem = q[y].size() - pos[y]; lx = y; }
        if (lx >= 0) out.push_back(tiles[q[lx][pos[lx]++]]);
      }
    }
  }
  std::copy(out.begin(), out.end(), tiles.begin() + t0);
}

int32_t build_plan(const ps_job* job, const TileShape& shape, int ksplit_override, size_t budget,
                   Plan* P, std::string* err, bool share_third, bool overlap_passes) {
  int32_t rc = validate_job(job, err);
  if (rc) return rc;
  Plan& p = *P;
  p = Plan();
  p.tile = shape;
  p.tile2 = shape;
  p.tile2.wm = 2;
  p.tile2.wn = 2;
  p.tile2.slots = shape.slots2;
  p.ksplit_override = ksplit_override;
  p.atoms.assign(job->atoms, job->atoms + job->n_atoms);
  if (job->n_bf) p.basis.assign(job->basis, job->basis + job->n_bf);
  if (job->n_aux) p.aux.assign(job->aux, job->aux + job->n_aux);
  p.n_atoms = job->n_atoms;
  p.n_bf = job->n_bf;
  p.n_aux = job->n_aux;
  p.precision = job->precision;
  const int N = p.n_atoms, nb = p.n_bf, na = p.n_aux;

  // internal FP64 output buffer: [S | T | V | PQ | abP | L]
  p.off_S = 0;
  p.off_T = p.off_S + (int64_t)nb * nb;
  p.off_V = p.off_T + (int64_t)nb * nb;
  p.off_PQ = p.off_V + (int64_t)nb * nb;
  p.off_abP = p.off_PQ + (int64_t)na * na;
  p.off_L = p.off_abP + (int64_t)na * nb * nb;
  p.out_elems = p.off_L + (int64_t)na * na;

  // per-atom function lists in caller order
  std::vector<std::vector<int>> bf_of(N), ax_of(N);
  for (int i = 0; i < nb; ++i) bf_of[p.basis[i].atom].push_back(i);
  for (int i = 0; i < na; ++i) ax_of[p.aux[i].atom].push_back(i);
  std::vector<int> nn(N);
  for (int X = 0; X < N; ++X) nn[X] = nearest_atom(p.atoms, X);

  auto spec_for = [&](int A, int B) -> ps_grid_spec {
    for (int k = 0; k < job->n_pair_grids; ++k) {
      const ps_pair_grid& pg = job->pair_grids[k];
      if ((pg.atom_a == A && pg.atom_b == B) || (pg.atom_a == B && pg.atom_b == A)) return pg.spec;
    }
    return job->grid;
  };

  // GL tables per distinct q, in the line buffer
  std::map<int, int> gl_off;
  auto gl_for = [&](int q) {
    auto it = gl_off.find(q);
    if (it != gl_off.end()) return it->second;
    int off = (int)p.lines.size();
    double x[16], w[16];
    gauss_legendre(q, x, w);
    for (int i = 0; i < q; ++i) p.lines.push_back(x[i]);
    for (int i = 0; i < q; ++i) p.lines.push_back(w[i]);
    gl_off[q] = off;
    return off;
  };

  // ---- grids (canonical order: A < B, then C ascending) ----
  for (int A = 0; A < N; ++A)
    for (int B = A + 1; B < N; ++B) {
      int cs = N >= 3 ? nearest_to_mid(p.atoms, A, B) : -1;
      for (int C = (N == 2 ? -1 : 0); C < N; ++C) {
        if (N >= 3 && (C == A || C == B)) continue;
        GridHost g;
        rc = build_grid(job->atoms, N, A, B, C, spec_for(A, B), &g, err);
        if (rc) return rc;
        g.pair_grid = (N == 2) || (C == cs);
        g.dev.lines = (int)p.lines.size();
        p.lines.insert(p.lines.end(), g.mu.begin(), g.mu.end());
        p.lines.insert(p.lines.end(), g.nu.begin(), g.nu.end());
        p.lines.insert(p.lines.end(), g.phi.begin(), g.phi.end());
        g.dev.gl = gl_for(g.dev.q);
        p.grids.push_back(g);
        if (N == 2) break;
      }
    }

  // ---- per-grid arrays, segments and tasks ----
  std::map<std::tuple<int, int, int, int>, int> phase_count;  // (kind, X, Y, Z) -> tasks so far
  auto add_array = [&](int grid, int nf, std::vector<int32_t> map) {
    ArrayHost a;
    a.grid = grid;
    a.nf = nf;
    a.es = p.precision == PS_PREC_MIXED ? 4 : 8;
    a.offset = 0;
    a.map = std::move(map);
    a.map_off = -1;
    p.arrays.push_back(a);
    return (int)p.arrays.size() - 1;
  };
  auto push_ints = [&](const std::vector<int32_t>& v) {
    int64_t off = (int64_t)p.ints.size();
    p.ints.insert(p.ints.end(), v.begin(), v.end());
    return off;
  };
  auto add_shell_seg = [&](int grid, int mode, int centre, const std::vector<ps_sto>& fns,
                           const std::vector<int>& idx, int arr0, int arr1, int col0) {
    if (idx.empty()) return;
    std::vector<ShellBuild> sh = make_shells(fns, idx);
    std::stable_sort(sh.begin(), sh.end(), [](const ShellBuild& a, const ShellBuild& b) { return a.l < b.l; });
    SegHost s;
    std::memset(&s.dev, 0, sizeof s.dev);
    s.dev.grid = grid;
    s.dev.mode = mode;
    s.dev.centre = centre;
    s.dev.nf = p.arrays[arr0].nf;
    s.dev.item_off = (int)p.shells.size();
    s.dev.n_items = (int)sh.size();
    for (int l = 0; l <= LMAX + 1; ++l) {
      int cnt = 0;
      for (auto& x : sh)
        if (x.l < l) ++cnt;
      s.dev.l_off[l] = s.dev.item_off + cnt;
    }
    for (auto& x : sh) {
      ShellDev d;
      d.zeta = x.zeta;
      d.norm = std::pow(2.0 * x.zeta, x.n + 0.5) / std::sqrt(factorial(2 * x.n));
      d.n = x.n;
      d.l = x.l;
      d.m_off = (int)p.ments.size();
      d.nm = 2 * x.l + 1;
      d.pre = 4.0 * kPi / (2.0 * x.l + 1.0) * d.norm * std::pow(x.zeta, -(x.n + 1.0));
      // dense in m = -l..l (entry l + m); a component the basis does not hold has col -1
      for (int m = -x.l; m <= x.l; ++m) {
        MEntry me;
        const int am = std::abs(m);
        me.f = std::sqrt((2.0 * x.l + 1.0) / (4.0 * kPi) * factorial(x.l - am) / factorial(x.l + am)) *
               (am ? std::sqrt(2.0) : 1.0);
        me.m = m;
        me.col = -1;
        for (auto& mc : x.ms)
          if (mc.first == m) me.col = mc.second + col0;
        p.ments.push_back(me);
      }
      p.shells.push_back(d);
    }
    s.arr0 = arr0;
    s.arr1 = arr1;
    p.segs.push_back(s);
  };

  struct TaskSpec {
    int U, V, Y;
    std::vector<int32_t> pairs;        // (u, v) columns
    std::vector<int32_t> mapU, mapV, mapY;  // per column of U, V, Y
    int y0, ny;
    int kind;                           // output kind for offsets
    int64_t out_off, outm_off;
    int64_t s1, s2, s3, t1, t2, t3;
    double alpha;
    int skip_diag;
    std::vector<std::tuple<int, int, int, int>> keys;
    double work_elems;                  // unique output elements
  };

  for (int gi = 0; gi < (int)p.grids.size(); ++gi) {
    GridHost& g = p.grids[gi];
    const int A = g.A, B = g.B, C = g.C;
    const bool pg = g.pair_grid;
    const std::vector<int>& bA = bf_of[A];
    const std::vector<int>& bB = bf_of[B];
    const int nA = (int)bA.size(), nB = (int)bB.size();
    // which one-centre blocks live here
    bool oneA = pg && nn[A] == B, oneB = pg && nn[B] == A;

    // arrays
    int aBA = add_array(gi, nA, std::vector<int32_t>(bA.begin(), bA.end()));
    int aBB = add_array(gi, nB, std::vector<int32_t>(bB.begin(), bB.end()));
    int aKA = -1, aKB = -1, aXAB = -1;
    if (pg) {
      aKA = add_array(gi, nA, std::vector<int32_t>(bA.begin(), bA.end()));
      aKB = add_array(gi, nB, std::vector<int32_t>(bB.begin(), bB.end()));
      // values of the auxiliary functions of A and B, one array [aux of A | aux of B]
      std::vector<int32_t> xm(ax_of[A].begin(), ax_of[A].end());
      xm.insert(xm.end(), ax_of[B].begin(), ax_of[B].end());
      aXAB = add_array(gi, (int)xm.size(), xm);
    }
    // potential columns: pair grid [aux A | aux B | aux C]; other grids [aux C]
    std::vector<int32_t> ymap;
    int yA0 = 0, yB0 = 0, yC0 = 0;
    int nyA = 0, nyB = 0, nyC = 0;
    if (pg) {
      yA0 = 0;
      nyA = (int)ax_of[A].size();
      ymap.insert(ymap.end(), ax_of[A].begin(), ax_of[A].end());
      yB0 = (int)ymap.size();
      nyB = (int)ax_of[B].size();
      ymap.insert(ymap.end(), ax_of[B].begin(), ax_of[B].end());
    }
    if (C >= 0) {
      yC0 = (int)ymap.size();
      nyC = (int)ax_of[C].size();
      ymap.insert(ymap.end(), ax_of[C].begin(), ax_of[C].end());
    }
    int aY = add_array(gi, (int)ymap.size(), ymap);
    // weight columns
    std::vector<WColDev> wc;
    auto add_w = [&](int kind, double zA, double zB, double zC) {
      WColDev w;
      w.kind = kind;
      w.zA = zA;
      w.zB = zB;
      w.zC = zC;
      w.col = (int)wc.size();
      wc.push_back(w);
      return w.col;
    };
    int cw = -1, cone = -1, cOAB = -1, cOAA = -1, cOBB = -1, cOC = -1;
    double ZA = p.atoms[A].Z, ZB = p.atoms[B].Z, ZC = C >= 0 ? p.atoms[C].Z : 0.0;
    if (pg) {
      cw = add_w(0, 0, 0, 0);
      cone = add_w(1, 0, 0, 0);
      cOAB = add_w(2, ZA, ZB, ZC);                       // nuclei A, B (and C* when present)
      cOAA = add_w(2, oneA ? ZA : 0.0, ZB, 0.0);         // nucleus B, plus A if B = nn(A)
      cOBB = add_w(2, ZA, oneB ? ZB : 0.0, 0.0);         // nucleus A, plus B if A = nn(B)
    } else {
      cOC = add_w(2, 0.0, 0.0, ZC);
    }
    int aW = add_array(gi, (int)wc.size(), std::vector<int32_t>(wc.size(), 0));

    // evaluation segments
    int mode_basis = pg ? EV_CHI_KIN : EV_CHI;
    if (pg) {
      add_shell_seg(gi, mode_basis, CEN_A, p.basis, bA, aBA, aKA, 0);
      add_shell_seg(gi, mode_basis, CEN_B, p.basis, bB, aBB, aKB, 0);
      add_shell_seg(gi, EV_CHI, CEN_A, p.aux, ax_of[A], aXAB, -1, 0);
      add_shell_seg(gi, EV_CHI, CEN_B, p.aux, ax_of[B], aXAB, -1, (int)ax_of[A].size());
      add_shell_seg(gi, EV_POT_W, CEN_A, p.aux, ax_of[A], aY, -1, yA0);
      add_shell_seg(gi, EV_POT_W, CEN_B, p.aux, ax_of[B], aY, -1, yB0);
    } else {
      add_shell_seg(gi, EV_CHI, CEN_A, p.basis, bA, aBA, -1, 0);
      add_shell_seg(gi, EV_CHI, CEN_B, p.basis, bB, aBB, -1, 0);
    }
    if (C >= 0) add_shell_seg(gi, EV_POT_W, CEN_C, p.aux, ax_of[C], aY, -1, yC0);
    {
      SegHost s;
      std::memset(&s.dev, 0, sizeof s.dev);
      s.dev.grid = gi;
      s.dev.mode = EV_WEIGHTS;
      s.dev.centre = CEN_A;
      s.dev.nf = (int)wc.size();
      s.dev.item_off = (int)p.wcols.size();
      s.dev.n_items = (int)wc.size();
      p.wcols.insert(p.wcols.end(), wc.begin(), wc.end());
      s.arr0 = aW;
      s.arr1 = -1;
      p.segs.push_back(s);
    }

    // ---- tasks ----
    const int64_t NB = nb, NA = na, NB2 = (int64_t)nb * nb;
    std::vector<TaskSpec> ts;
    auto iota_map = [](const std::vector<int>& v) { return std::vector<int32_t>(v.begin(), v.end()); };
    auto rect_pairs = [](int nu, const std::vector<int>& vcols) {
      std::vector<int32_t> pr;
      for (int u = 0; u < nu; ++u)
        for (int v : vcols) { pr.push_back(u); pr.push_back(v); }
      return pr;
    };
    auto rect_uv = [](int nu, int nv) {
      std::vector<int32_t> pr;
      for (int u = 0; u < nu; ++u)
        for (int v = 0; v < nv; ++v) { pr.push_back(u); pr.push_back(v); }
      return pr;
    };
    auto tri_pairs = [](int n) {
      std::vector<int32_t> pr;
      for (int u = 0; u < n; ++u)
        for (int v = u; v < n; ++v) { pr.push_back(u); pr.push_back(v); }
      return pr;
    };
    // 2-index task on S/V/T/PQ raw matrices: rows = (u, weight column), cols = Y columns.
    auto two_index = [&](int U, const std::vector<int32_t>& mapU, std::vector<int> wcols_used,
                         std::vector<int32_t> wsel, int Yarr, const std::vector<int32_t>& mapY, int y0,
                         int ny, int64_t base, int64_t sel_stride, int64_t ld, bool mirror,
                         std::vector<std::tuple<int, int, int, int>> keys, double work) {
      TaskSpec t;
      t.U = U;
      t.V = aW;
      t.Y = Yarr;
      t.pairs = rect_pairs((int)mapU.size(), wcols_used);
      t.mapU = mapU;
      t.mapV.assign(wc.size(), 0);
      for (size_t k = 0; k < wcols_used.size(); ++k) t.mapV[wcols_used[k]] = wsel[k];
      t.mapY.assign(p.arrays[Yarr].nf, 0);
      for (int k = 0; k < ny; ++k) t.mapY[y0 + k] = mapY[k];
      t.y0 = y0;
      t.ny = ny;
      t.out_off = base;
      t.s1 = ld;
      t.s2 = sel_stride;
      t.s3 = 1;
      t.outm_off = mirror ? base : -1;
      t.t1 = 1;
      t.t2 = sel_stride;
      t.t3 = ld;
      t.alpha = 1.0;
      t.skip_diag = 0;
      t.keys = keys;
      t.work_elems = work;
      t.kind = 0;
      if (t.pairs.empty() || ny == 0) return;
      ts.push_back(t);
    };
    auto abp_task = [&](int U, int V, bool tri, const std::vector<int32_t>& mapU,
                        const std::vector<int32_t>& mapV, int y0, int ny, bool mirror,
                        std::vector<std::tuple<int, int, int, int>> keys, double work) {
      TaskSpec t;
      t.U = U;
      t.V = V;
      t.Y = aY;
      t.pairs = tri ? tri_pairs((int)mapU.size()) : rect_uv((int)mapU.size(), (int)mapV.size());
      t.mapU = mapU;
      t.mapV = mapV;
      t.mapY = ymap;
      t.y0 = y0;
      t.ny = ny;
      t.out_off = p.off_abP;
      t.s1 = NB;
      t.s2 = 1;
      t.s3 = NB2;
      t.outm_off = mirror ? p.off_abP : -1;
      t.t1 = 1;
      t.t2 = NB;
      t.t3 = NB2;
      t.alpha = 1.0;
      t.skip_diag = tri ? 1 : 0;
      t.keys = keys;
      t.work_elems = work;
      t.kind = 4;
      if (t.pairs.empty() || ny == 0) return;
      ts.push_back(t);
    };
    std::vector<int32_t> mA = iota_map(bA), mB = iota_map(bB);
    const int64_t dSV = p.off_V - p.off_S;
    const double dA = nA, dB = nB;
    if (pg) {
      // S_AB and V_AB (rows: a x {w, w O_AB}); mirrored into the (B, A) block
      two_index(aBA, mA, {cw, cOAB}, {0, 1}, aBB, mB, 0, nB, p.off_S, dSV, NB, true,
                {{0, A, B, -1}, {0, B, A, -1}, {2, A, B, -1}, {2, B, A, -1}}, 2 * dA * dB);
      // T raw, both orders (symmetrised at the end)
      two_index(aBA, mA, {cw}, {0}, aKB, mB, 0, nB, p.off_T, 0, NB, false, {{1, A, B, -1}}, dA * dB);
      two_index(aBB, mB, {cw}, {0}, aKA, mA, 0, nA, p.off_T, 0, NB, false, {{1, B, A, -1}}, 0);
      // (P|Q) raw[P][Q] = sum w V_P chi_Q over the blocks this grid carries (A x B and B x A always,
      // A x A and B x B when it is that atom's one-centre grid), as at most two rectangles of
      // rows (Y column of V_P, weight column "ones") x columns (aux values [A | B])
      {
        const int pA = (int)ax_of[A].size(), pB = (int)ax_of[B].size();
        auto pq_task = [&](int y_lo, int y_n, int x_lo, int x_n, std::vector<std::tuple<int, int, int, int>> keys,
                           double work) {
          if (y_n <= 0 || x_n <= 0) return;
          TaskSpec t;
          t.U = aY; t.V = aW; t.Y = aXAB;
          std::vector<int32_t> mapUy(p.arrays[aY].nf, 0);
          for (int k = 0; k < y_n; ++k) {
            mapUy[y_lo + k] = ymap[y_lo + k];
            t.pairs.push_back(y_lo + k);
            t.pairs.push_back(cone);
          }
          t.mapU = mapUy; t.mapV.assign(wc.size(), 0); t.mapY = p.arrays[aXAB].map;
          t.y0 = x_lo; t.ny = x_n;
          t.out_off = p.off_PQ; t.s1 = NA; t.s2 = 0; t.s3 = 1;
          t.outm_off = -1; t.t1 = t.t2 = t.t3 = 0; t.alpha = 1.0; t.skip_diag = 0;
          t.keys = keys; t.work_elems = work; t.kind = 3;
          ts.push_back(t);
        };
        const double wAB = pA * pB, wAA = pA * (pA + 1) / 2.0, wBB = pB * (pB + 1) / 2.0;
        const std::tuple<int, int, int, int> kAB{3, A, B, -1}, kBA{3, B, A, -1}, kAA{3, A, A, -1}, kBB{3, B, B, -1};
        if (oneA && oneB) {
          pq_task(yA0, nyA + nyB, 0, pA + pB, {kAB, kBA, kAA, kBB}, wAB + wAA + wBB);
        } else if (oneA) {
          pq_task(yA0, nyA + nyB, 0, pA, {kAA, kBA}, wAA);  // rows A and B x columns A
          pq_task(yA0, nyA, pA, pB, {kAB}, wAB);            // rows A x columns B
        } else if (oneB) {
          pq_task(yA0, nyA + nyB, pA, pB, {kAB, kBB}, wAB + wBB);  // rows A and B x columns B
          pq_task(yB0, nyB, 0, pA, {kBA}, 0.0);                      // rows B x columns A
        } else {
          pq_task(yA0, nyA, pA, pB, {kAB}, wAB);
          pq_task(yB0, nyB, 0, pA, {kBA}, 0.0);
        }
      }
      // (ab|P), a on A, b on B, P on A, B (and C*)
      abp_task(aBA, aBB, false, mA, mB, 0, p.arrays[aY].nf, true,
               {{4, A, B, A}, {4, B, A, A}, {4, A, B, B}, {4, B, A, B}, {4, A, B, C}, {4, B, A, C}},
               dA * dB * p.arrays[aY].nf);
      // one-centre blocks of A and B
      for (int side = 0; side < 2; ++side) {
        const int X = side == 0 ? A : B, Yo = side == 0 ? B : A;
        const bool one = side == 0 ? oneA : oneB;
        const int aBX = side == 0 ? aBA : aBB, aKX = side == 0 ? aKA : aKB;
        const std::vector<int32_t>& mX = side == 0 ? mA : mB;
        const int cO = side == 0 ? cOAA : cOBB;
        const double n = mX.size();
        const double tri = n * (n + 1) / 2;
        const int yO0 = side == 0 ? yB0 : yA0, nyO = side == 0 ? nyB : nyA;
        if (one) {
          two_index(aBX, mX, {cw, cO}, {0, 1}, aBX, mX, 0, (int)mX.size(), p.off_S, dSV, NB, false,
                    {{0, X, X, -1}, {2, X, X, -1}}, 2 * tri);
          two_index(aBX, mX, {cw}, {0}, aKX, mX, 0, (int)mX.size(), p.off_T, 0, NB, false,
                    {{1, X, X, -1}}, tri);
          // (xx'|P), P on X and on the other focus: Y columns [A | B] are contiguous
          abp_task(aBX, aBX, true, mX, mX, 0, nyA + nyB, true, {{4, X, X, X}, {4, X, X, Yo}},
                   tri * (nyA + nyB));
        } else {
          two_index(aBX, mX, {cO}, {0}, aBX, mX, 0, (int)mX.size(), p.off_V, 0, NB, false,
                    {{2, X, X, -1}}, tri);
          abp_task(aBX, aBX, true, mX, mX, yO0, nyO, true, {{4, X, X, Yo}}, tri * nyO);
        }
      }
    } else {
      two_index(aBA, mA, {cOC}, {0}, aBB, mB, 0, nB, p.off_V, 0, NB, true, {{2, A, B, -1}, {2, B, A, -1}},
                dA * dB);
      abp_task(aBA, aBB, false, mA, mB, 0, nyC, true, {{4, A, B, C}, {4, B, A, C}}, dA * dB * nyC);
    }

    // register tasks with phases
    for (auto& t : ts) {
      int ph = 0;
      for (auto& k : t.keys) ph = std::max(ph, phase_count[k]);
      for (auto& k : t.keys) phase_count[k] = ph + 1;
      TaskHost th;
      std::memset(&th.dev, 0, sizeof th.dev);
      th.grid = gi;
      th.U = t.U;
      th.V = t.V;
      th.Y = t.Y;
      th.pairs_off = push_ints(t.pairs);
      th.dev.npairs = (int)t.pairs.size() / 2;
      th.dev.y0 = t.y0;
      th.dev.ny = t.ny;
      th.dev.s1 = t.s1;
      th.dev.s2 = t.s2;
      th.dev.s3 = t.s3;
      th.dev.t1 = t.t1;
      th.dev.t2 = t.t2;
      th.dev.t3 = t.t3;
      th.dev.alpha = t.alpha;
      th.dev.skip_diag = t.skip_diag;
      th.out_kind = t.kind;
      th.out_off = t.out_off;
      th.outm_off = t.outm_off;
      th.phase = ph;
      th.pair_points = t.work_elems * (double)g.dev.npts;
      // maps stored after the pair list
      int64_t mu = push_ints(t.mapU), mv = push_ints(t.mapV), my = push_ints(t.mapY);
      // stash map offsets in the (host-only) pointer fields as integers until binding
      th.dev.mapU = reinterpret_cast<const int32_t*>(mu);
      th.dev.mapV = reinterpret_cast<const int32_t*>(mv);
      th.dev.mapY = reinterpret_cast<const int32_t*>(my);
      p.tasks.push_back(th);
      p.pair_points += th.pair_points;
    }
    p.n_points += g.dev.npts;
  }

  // ---- mixed precision: the two-index tasks (S, T, V, (P|Q)) keep FP64 operands ----
  // An array read only by two-index tasks is held in FP64; one read by (ab|P) tasks as well gets an
  // FP64 twin beside its FP32 copy.  The FP32 evaluation computes every value in FP64 and writes
  // both copies; the two-index tasks read the FP64 arrays and run in FP64 contraction launches.
  const bool mixed = p.precision == PS_PREC_MIXED;
  if (mixed) {
    const size_t n0 = p.arrays.size();
    std::vector<char> need32(n0, 0), need64(n0, 0);
    for (const auto& th : p.tasks) {
      std::vector<char>& nd = th.out_kind == 4 ? need32 : need64;
      nd[th.U] = nd[th.V] = nd[th.Y] = 1;
    }
    std::vector<int> f64(n0, -1);  // FP64 array holding the values of array a
    for (size_t a = 0; a < n0; ++a) {
      if (!need64[a]) continue;
      if (need32[a]) {
        ArrayHost t = p.arrays[a];
        t.es = 8;
        p.arrays.push_back(t);
        f64[a] = (int)p.arrays.size() - 1;
      } else {
        p.arrays[a].es = 8;
        f64[a] = (int)a;
      }
    }
    for (auto& th : p.tasks)
      if (th.out_kind != 4) {
        th.U = f64[th.U];
        th.V = f64[th.V];
        th.Y = f64[th.Y];
      }
    for (auto& sg : p.segs) {
      for (int* a : {&sg.arr0, &sg.arr1}) {
        int* d = a == &sg.arr0 ? &sg.arr0d : &sg.arr1d;
        if (*a < 0 || f64[*a] < 0) continue;
        *d = f64[*a];
        if (f64[*a] == *a) *a = -1;  // FP64 only
      }
    }
  }

  // ---- cross-third-centre reuse (optional) ----
  // The grids G(A,B|C) of one pair other than its pair grid differ only by a rotation about the A-B
  // axis (each puts its own C at phi = 0) and by the lines moved onto their C.  In the regular cells
  // no member's moved lines touch, their points share (mu, nu, phi) and the distances to A and B:
  // one shared segment per atom evaluates those cells for all members (radial factors once), and
  // the members' own basis segments skip them.  Needs Q = 4 (a cell is one wave) and at most 128
  // cells per axis (the skip masks).
  if (share_third && N >= 4) {
    std::map<std::pair<int, int>, std::vector<int>> members_of;
    for (int gi = 0; gi < (int)p.grids.size(); ++gi)
      if (!p.grids[gi].pair_grid && p.grids[gi].C >= 0) members_of[{p.grids[gi].A, p.grids[gi].B}].push_back(gi);
    for (auto& kv : members_of) {
      const std::vector<int>& mg = kv.second;
      if (mg.size() < 2) continue;
      const GridDev& g0 = p.grids[mg[0]].dev;
      if (g0.q != 4 || g0.nmu > 128 || g0.nnu > 128) continue;
      std::vector<char> mu_ok(g0.nmu, 1), nu_ok(g0.nnu, 1);
      for (int gi : mg) {
        const GridDev& d = p.grids[gi].dev;
        if (d.istar > 0) mu_ok[d.istar - 1] = mu_ok[d.istar] = 0;  // cells on either side of a moved line
        if (d.jstar > 0) nu_ok[d.jstar - 1] = nu_ok[d.jstar] = 0;
      }
      std::vector<int32_t> cells;
      uint64_t mmask[2] = {0, 0}, nmask[2] = {0, 0};
      for (int i = 0; i < g0.nmu; ++i)
        if (mu_ok[i]) {
          cells.push_back(i);
          mmask[i >> 6] |= 1ull << (i & 63);
        }
      const int n_si = (int)cells.size();
      for (int j = 0; j < g0.nnu; ++j)
        if (nu_ok[j]) {
          cells.push_back(j);
          nmask[j >> 6] |= 1ull << (j & 63);
        }
      const int n_sj = (int)cells.size() - n_si;
      if (n_si == 0 || n_sj == 0) continue;
      const int64_t cells_off = push_ints(cells);
      for (int side = 0; side < 2; ++side) {
        const int centre = side == 0 ? CEN_A : CEN_B;
        ShareHost sh;
        for (int gi : mg)
          for (int si = 0; si < (int)p.segs.size(); ++si) {
            const SegHost& sg = p.segs[si];
            if (sg.dev.grid == gi && sg.dev.mode == EV_CHI && sg.dev.centre == centre) {
              sh.grids.push_back(gi);
              sh.segs.push_back(si);
              sh.arr0.push_back(sg.arr0);
              sh.arr0d.push_back(sg.arr0d);
            }
          }
        if (sh.segs.size() != mg.size()) continue;
        const SegDev& d0 = p.segs[sh.segs[0]].dev;
        std::memset(&sh.dev, 0, sizeof sh.dev);
        sh.dev.centre = centre;
        sh.dev.nf = d0.nf;
        sh.dev.n_members = (int)mg.size();
        sh.dev.n_si = n_si;
        sh.dev.n_sj = n_sj;
        sh.dev.item_off = d0.item_off;  // every member lists the same shells
        sh.dev.n_items = d0.n_items;
        for (int l = 0; l <= LMAX + 1; ++l) sh.dev.l_off[l] = d0.l_off[l];
        sh.cells_off = cells_off;
        for (int si : sh.segs) {
          SegDev& d = p.segs[si].dev;
          d.skip = 1;
          d.skip_mu[0] = mmask[0];
          d.skip_mu[1] = mmask[1];
          d.skip_nu[0] = nmask[0];
          d.skip_nu[1] = nmask[1];
        }
        p.shares.push_back(sh);
      }
    }
  }

  // ---- passes: group grids so that arrays + workspace fit the budget ----
  const TileShape& shape2 = p.tile2;
  // row tiles of a task: BM consecutive pairs, halved until their staged U + V columns fit
  auto row_tiles = [&](const TaskHost& th, const TileShape& sh) {
    const int BM = sh.bm(), MAXUV = sh.maxuv();
    const int32_t* pr = p.ints.data() + th.pairs_off;
    const int npairs = th.dev.npairs;
    std::vector<std::pair<int, int>> rows;
    for (int r0 = 0; r0 < npairs; r0 += BM) {
      std::vector<std::pair<int, int>> stack = {{r0, std::min(BM, npairs - r0)}};
      while (!stack.empty()) {
        auto [a0, n] = stack.back();
        stack.pop_back();
        int umin = 1 << 30, umax = -1, vmin = 1 << 30, vmax = -1;
        for (int r = a0; r < a0 + n; ++r) {
          umin = std::min(umin, pr[2 * r]);
          umax = std::max(umax, pr[2 * r]);
          vmin = std::min(vmin, pr[2 * r + 1]);
          vmax = std::max(vmax, pr[2 * r + 1]);
        }
        if ((umax - umin + 1) + (vmax - vmin + 1) <= MAXUV || n == 1) {
          rows.push_back({a0, n});
        } else {
          int h = n / 2;
          stack.push_back({a0 + h, n - h});
          stack.push_back({a0, h});
        }
      }
    }
    std::sort(rows.begin(), rows.end());
    return rows;
  };
  // Two-index tasks always take the second (64 x 64) shape.  An (ab|P) task takes it too when that
  // issues less than 90% of the FLOPs of the main shape (short row ranges); 64 x 64 tiles run about
  // 10% slower per FLOP.  Either shape's last column tile is narrowed to a multiple of 32 columns
  // (below), so one third atom's auxiliary set (e.g. 165 = 128 + 37 columns) issues 192 columns
  // in both and stays on the main shape.
  std::vector<char> small_task(p.tasks.size(), 1);
  for (size_t t = 0; t < p.tasks.size(); ++t) {
    const TaskHost& th = p.tasks[t];
    if (th.out_kind != 4) continue;
    auto issued = [&](const TileShape& sh) {
      const int full = th.dev.ny / sh.bn() * sh.bn();
      const int cols = full + (th.dev.ny - full + 31) / 32 * 32;
      return (double)row_tiles(th, sh).size() * sh.bm() * (double)cols;
    };
    small_task[t] = issued(shape2) < 0.9 * issued(shape) ? 1 : 0;
  }
  auto shape_of = [&](const TaskHost& th) -> const TileShape& {
    return small_task[&th - p.tasks.data()] ? shape2 : shape;
  };
  // per grid: its arrays, and one partial tile per (row tile, column tile) item of its tasks
  std::vector<size_t> grid_bytes(p.grids.size(), 0);
  for (auto& a : p.arrays) grid_bytes[a.grid] += ((size_t)a.nf * p.grids[a.grid].dev.npad * a.es + 255) / 256 * 256;
  for (auto& th : p.tasks) {
    const TileShape& sh = shape_of(th);
    const size_t items = row_tiles(th, sh).size() * (size_t)((th.dev.ny + sh.bn() - 1) / sh.bn());
    grid_bytes[th.grid] += items * (size_t)sh.bm() * sh.bn() * 8;
  }
  // reserve the K-split workspace (up to 8192 extra partial tiles per launch), the output buffer and
  // the job's tables; the rest holds the arrays and per-item partial tiles of the pass's grids
  const size_t out_bytes = (size_t)p.out_elems * 8;
  const size_t ws_cap1 = std::min<size_t>((size_t)8192 * shape.bm() * shape.bn() * 8, budget / 8);
  const size_t ws_cap2 = std::min<size_t>((size_t)8192 * shape2.bm() * shape2.bn() * 8, budget / 16);
  const size_t ws_cap3 = std::min<size_t>((size_t)4 * 8192 * shape.bm() * shape.bn() * 8, budget / 16);
  const size_t ws_cap = ws_cap1 + ws_cap2 + ws_cap3;
  // tables (grids, shells, tasks, tiles, pair lists): the pair lists plus a small allowance
  const size_t tables = ((size_t)1 << 20) + budget / 256 + p.ints.size() * 4;
  size_t arr_budget = budget > ws_cap + out_bytes + tables ? budget - ws_cap - out_bytes - tables : 0;
  // Overlapped passes: each of the two regions holds one pass's arrays, partial tiles and K-split
  // extras, so a pass gets half of what remains after a second workspace reservation; only for jobs
  // that need more than one pass anyway, and whose largest grid fits such a pass.
  {
    size_t total = 0, largest = 0;
    for (size_t b : grid_bytes) {
      total += b;
      largest = std::max(largest, b);
    }
    const size_t half = arr_budget > ws_cap ? (arr_budget - ws_cap) / 2 : 0;
    if (overlap_passes && total > arr_budget && largest <= half) {
      p.overlap = true;
      arr_budget = half;
    }
  }
  {
    int g0 = 0;
    while (g0 < (int)p.grids.size()) {
      size_t acc = 0;
      int g1 = g0;
      while (g1 < (int)p.grids.size() && (g1 == g0 || acc + grid_bytes[g1] <= arr_budget)) {
        acc += grid_bytes[g1];
        ++g1;
      }
      if (acc > arr_budget) {
        char buf[200];
        snprintf(buf, sizeof buf, "grid %d needs %.2f GB of device arrays, beyond the budget", g0, acc / 1e9);
        *err = buf;
        return PS_E_NOMEM;
      }
      Pass ps;
      ps.grid0 = g0;
      ps.grid1 = g1;
      ps.array_bytes = acc;
      p.passes.push_back(ps);
      g0 = g1;
    }
  }
  // array offsets within each pass's region
  for (auto& ps : p.passes) {
    size_t off = 0;
    for (auto& a : p.arrays) {
      if (a.grid < ps.grid0 || a.grid >= ps.grid1) continue;
      a.offset = (int64_t)off;
      off += (size_t)a.nf * p.grids[a.grid].dev.npad * a.es;
      off = (off + 255) / 256 * 256;
    }
    ps.array_bytes = off;
  }
  // shared segments: kept only when all members are in one pass; block offsets per pass
  {
    std::vector<int> pass_of(p.grids.size(), -1);
    for (int k = 0; k < (int)p.passes.size(); ++k)
      for (int gi = p.passes[k].grid0; gi < p.passes[k].grid1; ++gi) pass_of[gi] = k;
    for (auto& sh : p.shares)
      for (int gi : sh.grids)
        if (pass_of[gi] != pass_of[sh.grids[0]]) sh.dropped = true;
    for (auto& sh : p.shares)
      if (sh.dropped)
        for (int si : sh.segs) {
          SegDev& d = p.segs[si].dev;
          d.skip = 0;
          d.skip_mu[0] = d.skip_mu[1] = d.skip_nu[0] = d.skip_nu[1] = 0;
        }
    for (int k = 0; k < (int)p.passes.size(); ++k) {
      Pass& ps = p.passes[k];
      ps.sseg0 = (int)p.ssegs.size();
      int64_t blk = 0;
      for (int h = 0; h < (int)p.shares.size(); ++h) {
        ShareHost& sh = p.shares[h];
        if (sh.dropped || pass_of[sh.grids[0]] != k) continue;
        sh.dev.block0 = blk;
        blk += ((int64_t)sh.dev.n_si * sh.dev.n_sj * p.grids[sh.grids[0]].dev.nphi + 3) / 4;
        p.ssegs.push_back(h);
      }
      ps.sseg1 = (int)p.ssegs.size();
      ps.shared_blocks = blk;
    }
  }
  // segments: block offsets per pass
  {
    size_t si = 0;
    for (auto& ps : p.passes) {
      ps.seg0 = (int)si;
      int64_t blk = 0;
      while (si < p.segs.size() && p.segs[si].dev.grid < ps.grid1) {
        p.segs[si].dev.block0 = blk;
        blk += p.grids[p.segs[si].dev.grid].dev.npad / 256;
        ++si;
      }
      ps.seg1 = (int)si;
      ps.eval_blocks = blk;
    }
  }
  // tiles and reduction items per pass
  {
    size_t ti = 0;
    for (auto& ps : p.passes) {
      ps.task0 = (int)ti;
      while (ti < p.tasks.size() && p.tasks[ti].grid < ps.grid1) ++ti;
      ps.task1 = (int)ti;
      // row x column tiles of each task; group 0 = (ab|P) tasks (main shape), group 1 = two-index
      // tasks (second shape), each group one contraction launch
      struct Item {
        int task, row0, nrows, p0, np, ulo, nu, vlo, nv;
        double cost;
      };
      // groups (one launch each): 0 the main shape, 1 the 64 x 64 shape, 2 + w for w = 1..3 the
      // main shape narrowed to 32 w columns, which takes the last column tile of a main-shape task
      // when that tile is at most 32 w wide (e.g. 345 columns = 128 + 128 + 96 instead of 3 x 128)
      // (group 5: the 64 x 64 shape narrowed to 32 columns, likewise for its tasks' last tiles;
      // groups 6 and 7: the 64 x 64 and 64 x 32 shapes in FP64, for the two-index tasks of a mixed job)
      // groups: 0 main shape, 1 the 64 x 64 shape, 2-4 the main shape narrowed to 32, 64, 96 columns,
      // 5 the 64 x 32 shape, 6-7 the FP64 64 x 64 and 64 x 32 shapes of a mixed job, 8-11 32-row
      // shapes 32 x (32, 64, 96, 128) for short row tiles, 12-13 FP64 32 x (32, 64) for the short row
      // tiles of a mixed job's FP64 tasks, 14-17 the 4 x 1 arrangement 128 x (16, 48, 80, 112) for
      // last column tiles of an odd number of 16-column blocks
      constexpr int NG = 18;
      TileShape gshape[NG] = {shape, shape2, shape, shape, shape, shape2, shape2, shape2, shape,
                              shape, shape, shape, shape2, shape2, shape, shape, shape, shape};
      for (int w = 1; w <= 3; ++w) {
        gshape[1 + w].wn = w;
        gshape[1 + w].slots = shape.slots_n[w];
      }
      for (int w = 1; w <= 4; ++w) {
        gshape[7 + w].wm = 1;
        gshape[7 + w].wn = w;
        gshape[7 + w].slots = shape.slots_short[w];
      }
      for (int w = 1; w <= 2; ++w) {
        gshape[11 + w].wm = 1;
        gshape[11 + w].wn = w;
        gshape[11 + w].slots = shape.slots_short_f64[w];
      }
      for (int k = 0; k < 4; ++k) {
        gshape[14 + k].wm = 2;
        gshape[14 + k].wn = 2 * k + 1;
        gshape[14 + k].wr = 4;
        gshape[14 + k].slots = shape.slots_tall[k];
      }
      const bool tall_ok = shape.wr == 2 && shape.bm() == 128;
      gshape[5].wn = 1;
      gshape[5].slots = shape.slots2n;
      gshape[6].slots = shape.slots2_f64;
      gshape[7].wn = 1;
      gshape[7].slots = shape.slots2n_f64;
      std::vector<Item> items[NG];
      double total_cost[NG] = {};
      for (int t = ps.task0; t < ps.task1; ++t) {
        TaskHost& th = p.tasks[t];
        const int grp0 = (mixed && th.out_kind != 4) ? 6 : (small_task[t] ? 1 : 0);
        const TileShape& sh = gshape[grp0];
        const int BN = sh.bn();
        const int32_t* pr = p.ints.data() + th.pairs_off;
        const int64_t nch = p.grids[th.grid].dev.npad / KC;
        const std::vector<std::pair<int, int>> rows = row_tiles(th, sh);
        for (auto& rw : rows) {
          int umin = 1 << 30, umax = -1, vmin = 1 << 30, vmax = -1;
          for (int r = rw.first; r < rw.first + rw.second; ++r) {
            umin = std::min(umin, pr[2 * r]);
            umax = std::max(umax, pr[2 * r]);
            vmin = std::min(vmin, pr[2 * r + 1]);
            vmax = std::max(vmax, pr[2 * r + 1]);
          }
          for (int c0 = 0; c0 < th.dev.ny; c0 += BN) {
            Item it;
            it.task = t;
            it.row0 = rw.first;
            it.nrows = rw.second;
            it.p0 = c0;
            it.np = std::min(BN, th.dev.ny - c0);
            it.ulo = umin;
            it.nu = umax - umin + 1;
            it.vlo = vmin;
            it.nv = vmax - vmin + 1;
            it.cost = (double)nch;
            int grp = grp0;
            const int w = (it.np + 31) / 32;
            if (grp0 == 0 && w < shape.wn) grp = 1 + w;
            // a last column tile of an odd number of 16-column blocks (e.g. 37 columns: 48, not 64)
            const int b16 = (it.np + 15) / 16;
            if (grp0 == 0 && tall_ok && b16 % 2 == 1 && b16 < 2 * shape.wn) grp = 14 + b16 / 2;
            if (grp0 == 1 && w < shape2.wn) grp = 5;
            if (grp0 == 6 && w < shape2.wn) grp = 7;
            // a task's last row tile when it holds a quarter of the main shape's rows or fewer (e.g. 4
            // of 128), or half of the 64-row shape's: a 32-row shape issues a quarter (a half) of the
            // MFMAs
            const int short_grp = grp0 == 6 ? 11 + w : 7 + w;
            const bool short_rows = grp0 == 0 ? shape.wm > 1 && 4 * it.nrows <= shape.bm()
                                              : 2 * it.nrows <= shape2.bm();
            if (short_rows && w <= (grp0 == 6 ? 2 : 4) && it.nu + it.nv <= gshape[short_grp].maxuv())
              grp = short_grp;
            total_cost[grp] += it.cost;
            items[grp].push_back(it);
          }
        }
      }
      int64_t ws = 0;
      ps.red_by_phase.clear();
      ps.launches.clear();
      ps.tile0 = (int)p.tiles.size();
      int n_narrow = 0, n_second = 0;
      for (int grp : {2, 3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17}) n_narrow += items[grp].empty() ? 0 : 1;
      for (int grp : {1, 6}) n_second += items[grp].empty() ? 0 : 1;
      // launch order: main, narrow main, tall, 32-row, 64 x 64, narrow 64 x 64, then the FP64 ones of
      // a mixed job (64 x 64, 64 x 32, 32-row)
      const int order[NG] = {0, 2, 3, 4, 14, 15, 16, 17, 8, 9, 10, 11, 1, 5, 6, 7, 12, 13};
      for (int oi = 0; oi < NG; ++oi) {
        const int grp = order[oi];
        if (items[grp].empty()) continue;
        const TileShape& sh = gshape[grp];
        const int BM = sh.bm(), BN = sh.bn();
        // K splits: at least 2048 work-groups per launch (8 per CU over 256 CUs); launches of long tiles
        // up to 6 per item while tiles keep 8192 chunks or more, so that the dispatch balances (a
        // tile's fixed cost, its first stage and its partial-tile write, stays small against its
        // length); all within the group's workspace reservation (one BM x BN FP64 partial tile per
        // work-group)
        const size_t cap = grp == 0 ? ws_cap1
                           : (grp == 1 || grp == 6) ? ws_cap2 / std::max(1, n_second)
                                                    : ws_cap3 / std::max(1, n_narrow);
        const double ws_tiles = (double)cap / ((double)BM * BN * 8);
        const double want_tiles =
            std::max(2048.0, std::min(6.0 * (double)items[grp].size(), total_cost[grp] / 8192.0));
        const double target = std::max((double)items[grp].size(), std::min(want_tiles, ws_tiles));
        const int tg0 = (int)p.tiles.size();
        const size_t nit = items[grp].size();
        std::vector<int64_t> nsv(nit), nstv(nit);
        const bool fill_ws = (double)nit >= ws_tiles;
        // tile length bound: the smallest L for which ceil(cost / L) splits per item total at most the
        // target, so that no tile of the launch is longer than L (splitting each item in proportion
        // to its cost and rounding left one launch's tiles up to twice as long as others)
        double len_bound = 1.0;
        if (p.ksplit_override <= 0 && !fill_ws && nit > 0) {
          double hi = 0.0;
          for (const Item& it : items[grp]) hi = std::max(hi, it.cost);
          double lo = std::min(hi, total_cost[grp] / target);
          auto splits = [&](double L) {
            double n = 0.0;
            for (const Item& it : items[grp]) n += std::ceil(it.cost / L - 1e-9);
            return n;
          };
          for (int k = 0; k < 60; ++k) {
            const double mid = 0.5 * (lo + hi);
            if (splits(mid) <= target) hi = mid; else lo = mid;
          }
          len_bound = hi;
        }
        int64_t total_ns = 0;
        for (size_t ii = 0; ii < nit; ++ii) {
          const Item& it = items[grp][ii];
          const int64_t nch = p.grids[p.tasks[it.task].grid].dev.npad / KC;
          int64_t ns;
          if (p.ksplit_override > 0)
            ns = p.ksplit_override;
          else if (fill_ws)
            ns = 1;  // the items alone fill the K-split allowance: one partial tile each
          else
            ns = (int64_t)std::ceil(it.cost / len_bound - 1e-9);
          const int64_t nst = nch / TileShape::SC_MAX;  // whole stages (nch is a multiple of 16)
          ns = std::max<int64_t>(1, std::min<int64_t>(ns, std::max<int64_t>(1, nst / 8)));
          nsv[ii] = ns;
          nstv[ii] = nst;
          total_ns += ns;
        }
        // round the launch up to whole waves of resident work-groups: split the items with the
        // longest tiles once more until the last wave is full (its tiles would otherwise leave CUs
        // idle while the launch drains)
        if (sh.slots > 0 && p.ksplit_override <= 0 && !fill_ws && total_ns > 0) {
          int64_t want = (total_ns + sh.slots - 1) / sh.slots * sh.slots;
          if ((double)want > ws_tiles) want = total_ns;  // beyond the workspace reservation: no rounding
          while (total_ns < want) {
            int64_t best = -1;
            double best_len = 0.0;
            for (size_t ii = 0; ii < nit; ++ii) {
              if (nsv[ii] >= std::max<int64_t>(1, nstv[ii] / 8)) continue;
              const double len = (double)nstv[ii] / (double)nsv[ii];
              if (len > best_len) {
                best_len = len;
                best = (int64_t)ii;
              }
            }
            if (best < 0) break;
            ++nsv[best];
            ++total_ns;
          }
        }
        for (size_t ii = 0; ii < nit; ++ii) {
          const Item& it = items[grp][ii];
          TaskHost& th = p.tasks[it.task];
          const int64_t ns = nsv[ii], nst = nstv[ii];
          RedDev rd;
          rd.task = it.task;
          rd.row0 = it.row0;
          rd.nrows = it.nrows;
          rd.p0 = it.p0;
          rd.np = it.np;
          rd.nsplit = (int)ns;
          rd.bm = BM;
          rd.bn = BN;
          rd.ws = ws;
          for (int64_t sp = 0; sp < ns; ++sp) {
            TileDev td;
            std::memset(&td, 0, sizeof td);
            td.task = it.task;
            td.row0 = it.row0;
            td.nrows = it.nrows;
            td.ulo = it.ulo;
            td.nu = it.nu;
            td.vlo = it.vlo;
            td.nv = it.nv;
            td.p0 = it.p0;
            td.np = it.np;
            td.kc0 = TileShape::SC_MAX * (nst * sp / ns);
            td.nkc = TileShape::SC_MAX * (nst * (sp + 1) / ns) - td.kc0;
            td.ws = ws + sp * (int64_t)BM * BN;
            p.issued_flops += 2.0 * BM * BN * (double)td.nkc * KC;
            p.tiles.push_back(td);
          }
          ws += ns * (int64_t)BM * BN;
          int phase = th.phase;
          if ((int)ps.red_by_phase.size() <= phase) ps.red_by_phase.resize(phase + 1);
          ps.red_by_phase[phase].push_back((int)p.reds.size());
          p.reds.push_back(rd);
        }
        xcd_order(p.tiles, tg0, (int)p.tiles.size());
        ps.launches.push_back({tg0, (int)p.tiles.size(), sh, grp == 6 || grp == 7 || grp == 12 || grp == 13});
      }
      // The 128-row launches (the main shape, its narrowed and tall last-column shapes; consecutive,
      // first in the launch order, one precision) become one launch whose tiles name their shapes:
      // one drain of the device per pass instead of one per shape.  Its tiles are ordered again,
      // longest first by MFMA steps, across all of them.
      {
        auto merged_id = [](const TileShape& s) {
          for (int k = 0; k < 8; ++k)
            if (s.wm == kMergedShapes[k][0] && s.wn == kMergedShapes[k][1] && s.wr == kMergedShapes[k][2]) return k;
          return -1;
        };
        std::vector<Pass::Launch> kept;
        int m0 = -1, m1 = -1;
        for (const auto& l : ps.launches) {
          const int id = merged_id(l.shape);
          if (id >= 0 && !l.f64 && l.shape.sc == shape.sc && (m1 < 0 || l.tile0 == m1)) {
            for (int i = l.tile0; i < l.tile1; ++i) p.tiles[i].shape = id;
            if (m0 < 0) m0 = l.tile0;
            m1 = l.tile1;
          } else {
            kept.push_back(l);
          }
        }
        if (m0 >= 0) {
          xcd_order(p.tiles, m0, m1);
          TileShape merged = shape;
          merged.wm = 0;  // marks the merged launch
          kept.insert(kept.begin(), Pass::Launch{m0, m1, merged, false});
        }
        ps.launches = kept;
      }
      ps.tile1 = (int)p.tiles.size();
      ps.ws_elems = (size_t)ws;
      // the pass's partial tiles follow its arrays in the shared region
      ps.ws_offset = (ps.array_bytes + 255) / 256 * 256;
      p.max_array_bytes = std::max(p.max_array_bytes, ps.ws_offset + (size_t)ws * 8);
      p.max_ws_bytes = std::max(p.max_ws_bytes, (size_t)ws * 8);
    }
  }
  if (p.overlap) {
    // even passes at the start of the array area, odd passes after the largest even one
    size_t r0 = 0, r1 = 0;
    for (size_t k = 0; k < p.passes.size(); ++k) {
      const Pass& ps = p.passes[k];
      size_t& r = k % 2 ? r1 : r0;
      r = std::max(r, ps.ws_offset + ps.ws_elems * 8);
    }
    r0 = (r0 + 255) / 256 * 256;
    for (size_t k = 1; k < p.passes.size(); k += 2) {
      Pass& ps = p.passes[k];
      ps.region_off = r0;
      ps.ws_offset += r0;
      for (auto& a : p.arrays)
        if (a.grid >= ps.grid0 && a.grid < ps.grid1) a.offset += (int64_t)r0;
    }
    p.max_array_bytes = r0 + r1;
  }
  p.contract_flops = 2.0 * p.pair_points;
  return PS_OK;
}

}  // namespace psint
