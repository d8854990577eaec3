// gfx950 kernels for prolate-spheroidal quadrature of Slater integrals.
//
//   eval_kernel      one thread per grid point: PS coordinates -> focus-relative displacements and
//                    weight (FP64), then Slater values, kinetic values, w * aux potentials or weight
//                    columns into chunked-SoA arrays (coalesced 128-byte lines per column chunk).
//   contract_f64     C[(u,v)][y] = sum_g U[u][g] V[v][g] Y[y][g]: the pair product is formed in
//                    registers from LDS-staged columns and fed to v_mfma_f64_16x16x4; each
//                    work-group owns one (pair-rows x columns) tile over a range of point chunks and
//                    writes an FP64 partial tile.
//   contract_mixed   the same with FP32 operands and v_mfma_f32_16x16x4f32, each stage's FP32 sums
//                    folded into FP64 accumulators.
//   reduce_kernel    sums the partial tiles of a tile in split order (deterministic) and scatters
//                    into the FP64 output buffer, with an optional mirrored write.
//   symmetrize / cholesky / fill / copy helpers.
//   mfma_rate_kernel a probe of the matrix pipe's sustained FP64 / FP32 rate (independent MFMAs on
//                    register operands), for reading roofline fractions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "psint_internal.h"

namespace psint {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------------
// Grid geometry.  Point g of grid G: cell c = g / q^3 with GL node indices (p, q, r); cells past
// n_reg are the extra subcells of the 8 cells around the third centre (subcell 0 of each of those
// 8 cells keeps the cell's own slot in the regular enumeration).
// ------------------------------------------------------------------------------------------------
struct Geo {
  double w;
  double d[3][3];  // displacement point - centre (A, B, C), global orientation
  double r[3];
};

__device__ __forceinline__ void point_geo(const GridDev& G, const double* __restrict__ lines, int64_t g,
                                          Geo& o) {
  const int q = G.q, q2 = q * q, q3 = q2 * q;
  const int64_t c = g / q3;
  const int rem = (int)(g - c * q3);
  const int ip = rem / q2, iq = (rem / q) % q, ir = rem % q;
  int i, j, k, ns = 1, si = 0, sj = 0, sk = 0;
  if (c < G.n_reg) {
    const int64_t plane = (int64_t)G.nnu * G.nphi;
    i = (int)(c / plane);
    const int64_t r2 = c - (int64_t)i * plane;
    j = (int)(r2 / G.nphi);
    k = (int)(r2 - (int64_t)j * G.nphi);
    if (G.split && (i == G.istar - 1 || i == G.istar) && (j == G.jstar - 1 || j == G.jstar) &&
        (k == G.nphi - 1 || k == 0))
      ns = G.nsp;
  } else {
    const int s3m = G.nsp * G.nsp * G.nsp - 1;
    const int64_t e = c - G.n_reg;
    const int which = (int)(e / s3m);
    const int sub = (int)(e - (int64_t)which * s3m) + 1;
    i = G.istar - 1 + (which >> 2);
    j = G.jstar - 1 + ((which >> 1) & 1);
    k = (which & 1) ? 0 : G.nphi - 1;
    ns = G.nsp;
    si = sub / (G.nsp * G.nsp);
    sj = (sub / G.nsp) % G.nsp;
    sk = sub % G.nsp;
  }
  const double* mu = lines + G.lines;
  const double* nu = mu + G.nmu + 1;
  const double* ph = nu + G.nnu + 1;
  const double* glx = lines + G.gl;
  const double* glw = glx + q;
  const double inv = 1.0 / ns;
  const double hm = (mu[i + 1] - mu[i]) * inv, hn = (nu[j + 1] - nu[j]) * inv, hp = (ph[k + 1] - ph[k]) * inv;
  const double m = mu[i] + hm * (si + 0.5 * (1.0 + glx[ip]));
  const double n = nu[j] + hn * (sj + 0.5 * (1.0 + glx[iq]));
  const double f = ph[k] + hp * (sk + 0.5 * (1.0 + glx[ir]));
  const double wq = (0.5 * hm * glw[ip]) * (0.5 * hn * glw[iq]) * (0.5 * hp * glw[ir]);
  // half-angle forms keep distances to the foci free of cancellation
  const double shh = sinh(0.5 * m);
  const double s2 = shh * shh;
  const double chh = sqrt(1.0 + s2);
  double sn2, cs2, sf, cf;
  sincos(0.5 * n, &sn2, &cs2);
  sincos(f, &sf, &cf);
  const double sh = 2.0 * shh * chh, ch = 1.0 + 2.0 * s2;
  const double sn = 2.0 * sn2 * cs2, cs = (cs2 - sn2) * (cs2 + sn2);
  const double a = G.a;
  o.w = wq * a * a * a * sh * sn * (sh * sh + sn * sn);
  const double rho = a * sh * sn;
  const double lx = rho * cf, ly = rho * sf;
  const double lz[3] = {a * (2.0 * s2 * cs - 2.0 * sn2 * sn2), a * (2.0 * s2 * cs + 2.0 * cs2 * cs2),
                        a * ch * cs - G.cz};
  const double lxs[3] = {lx, lx, lx - G.cx};
  o.r[0] = 2.0 * a * (s2 + sn2 * sn2);
  o.r[1] = 2.0 * a * (s2 + cs2 * cs2);
  o.r[2] = sqrt(lxs[2] * lxs[2] + ly * ly + lz[2] * lz[2]);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    o.d[t][0] = lxs[t] * G.ex[0] + ly * G.ey[0] + lz[t] * G.ez[0];
    o.d[t][1] = lxs[t] * G.ex[1] + ly * G.ey[1] + lz[t] * G.ez[1];
    o.d[t][2] = lxs[t] * G.ex[2] + ly * G.ey[2] + lz[t] * G.ez[2];
  }
}

// ------------------------------------------------------------------------------------------------
// Slater radial parts and the Coulomb potential of an auxiliary Slater function.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

__constant__ double kFact[24] = {1.0,
                                 1.0,
                                 2.0,
                                 6.0,
                                 24.0,
                                 120.0,
                                 720.0,
                                 5040.0,
                                 40320.0,
                                 362880.0,
                                 3628800.0,
                                 39916800.0,
                                 479001600.0,
                                 6227020800.0,
                                 87178291200.0,
                                 1307674368000.0,
                                 20922789888000.0,
                                 355687428096000.0,
                                 6402373705728000.0,
                                 121645100408832000.0,
                                 2432902008176640000.0,
                                 51090942171709440000.0,
                                 1124000727777607680000.0,
                                 25852016738884976640000.0};

// 1/j for j = 1..255 (entry 0 unused): the series below and the harmonic recurrence multiply by
// these instead of dividing (an FP64 division is a ten-instruction sequence; the index is uniform
// across a wave, so each entry is a scalar load).
struct InvTable {
  double v[256];
};
constexpr InvTable make_inv_table() {
  InvTable t{};
  t.v[0] = 0.0;
  for (int j = 1; j < 256; ++j) t.v[j] = 1.0 / j;
  return t;
}
__constant__ InvTable kInv = make_inv_table();

// Integer-order incomplete gamma functions from the terms t_j = x^j / j!:
//   Gamma(k, x) = (k-1)! e^-x sum_{j<k} t_j,   gamma(k, x) = (k-1)! e^-x sum_{j>=k} t_j.
// The lower one is (k-1)! (1 - e^-x head) unless the regularised P(k, x) = e^-x sum_{j>=k} t_j is
// small, where that difference would cancel: its relative rounding error is about 1e-16 / P.  For
// x < k/2 the tail terms fall at least by half each step, so e^-x t_k <= P <= 2 e^-x t_k; the tail is
// summed directly when x < k/2 and e^-x t_k < 1e-3 (there its terms fall fast), else the complement
// is used (relative error at most 3e-13 for k <= 24).  Both head sums come from one pass (k_up < k_lo).
__device__ __forceinline__ void inc_gamma_pair(int k_lo, int k_up, double x, double ex, double* lower,
                                               double* upper) {
  double t = 1.0, head = 1.0, h2 = 1.0;
  for (int j = 1; j < k_lo; ++j) {
    t *= x * kInv.v[j];
    h2 += t;
    if (j < k_up) head = h2;
  }
  *upper = kFact[k_up - 1] * ex * head;
  const double tk = t * x * kInv.v[k_lo];  // t_{k_lo}
  if (x < 0.5 * k_lo && ex * tk < 1e-3) {
    double tail = 0.0, tj = tk;
    for (int j = k_lo; j < k_lo + 200; ++j) {
      tail += tj;
      if (tj < 1e-17 * tail) break;
      tj *= x * kInv.v[j + 1];
    }
    *lower = kFact[k_lo - 1] * ex * tail;
  } else {
    *lower = kFact[k_lo - 1] * (1.0 - ex * h2);
  }
}

// ------------------------------------------------------------------------------------------------
// Real solid harmonics of the unit displacement (x, y, z) at degree l from degree l - 1 (Cm1, Sm1),
// written over degree l - 2 in (C, Sv): entry m of degree l needs entry m of degree l - 2 and entries
// m, m - 1 of degree l - 1 only (the recurrences below), so two register sets alternate by the
// parity of l.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void harmonic_level(int l, double x, double y, double z, const double* Cm1,
                                               const double* Sm1, double* C, double* Sv) {
  if (l == 0) {
#pragma unroll
    for (int m = 0; m <= LMAX; ++m) C[m] = Sv[m] = 0.0;
    C[0] = 1.0;
    return;
  }
  const double tl = 2.0 * l - 1.0;
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    double cn = 0.0, sn = 0.0;
    if (m == l) {
      if (m >= 1) {
        cn = tl * (x * Cm1[m >= 1 ? m - 1 : 0] - y * Sm1[m >= 1 ? m - 1 : 0]);
        sn = tl * (y * Cm1[m >= 1 ? m - 1 : 0] + x * Sm1[m >= 1 ? m - 1 : 0]);
      }
    } else if (m == l - 1) {
      cn = tl * z * Cm1[m];
      sn = tl * z * Sm1[m];
    } else if (m < l - 1) {
      const double inv = kInv.v[l - m];
      cn = (tl * z * Cm1[m] - (l + m - 1.0) * C[m]) * inv;
      sn = (tl * z * Sm1[m] - (l + m - 1.0) * Sv[m]) * inv;
    }
    C[m] = cn;
    Sv[m] = sn;
  }
}

// ------------------------------------------------------------------------------------------------
// Evaluation kernel.  Real solid harmonics of the unit displacement by the Cartesian recurrences
//   C_l^l = (2l-1)(x C_{l-1}^{l-1} - y S_{l-1}^{l-1}),  S_l^l = (2l-1)(y C_{l-1}^{l-1} + x S_{l-1}^{l-1}),
//   C_l^{l-1} = (2l-1) z C_{l-1}^{l-1},  (l-m) C_l^m = (2l-1) z C_{l-1}^m - (l+m-1) C_{l-2}^m,
// (same for S), which give P_l^m(cos t) cos(m phi) and sin(m phi) without the Condon-Shortley phase;
// Y_lm = f * C_l^m (m >= 0) or f * S_l^|m| (m < 0) with f from the host.
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void eval_kernel(const SegDev* __restrict__ segs, int nseg,
                                                   const GridDev* __restrict__ grids,
                                                   const double* __restrict__ lines,
                                                   const ShellDev* __restrict__ shells,
                                                   const MEntry* __restrict__ ments,
                                                   const WColDev* __restrict__ wcols) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const SegDev& S = segs[lo];
  const GridDev& G = grids[S.grid];
  // A wave's 64 points are 4 whole chunks of one grid (grids are padded to multiples of 256 points),
  // so the output offset splits into a wave-uniform part (chunk g/16 starts at (g/16) * nf * 16 =
  // gw * nf elements for the wave's first point gw, plus col * 16 for a column) and a fixed per-lane
  // part below 4 * nf * 16: each store is a scalar base plus one 32-bit lane offset.
  const int lane = threadIdx.x & 63;
  const int64_t gw = (b - S.block0) * 256 + __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
  const int64_t g = gw + lane;
  typedef __attribute__((address_space(1))) T GT;
  typedef __attribute__((address_space(1))) double GD;
  GT* __restrict__ w0 = (GT*)S.arr0 + gw * S.nf;
  GT* __restrict__ w1 = (GT*)S.arr1 + gw * S.nf;
  const uint32_t loff = (uint32_t)((lane >> 4) * S.nf * KC + (lane & 15));
  // FP32 evaluation (mixed jobs): a column may go to the FP32 array, to its FP64 twin, or both
  // (the pointers are uniform over the segment); FP64 evaluation: the FP64 array alone
  constexpr bool F32 = sizeof(T) == 4;
  GD* __restrict__ d0 = (GD*)S.arr0d + gw * S.nf;
  GD* __restrict__ d1 = (GD*)S.arr1d + gw * S.nf;
  const bool has0 = !F32 || S.arr0 != nullptr, has1 = !F32 || S.arr1 != nullptr;
  const bool has0d = F32 && S.arr0d != nullptr, has1d = F32 && S.arr1d != nullptr;
  auto put0 = [&](int col, double v) {
    if (has0) w0[(int64_t)col * KC + loff] = (T)v;
    if (has0d) d0[(int64_t)col * KC + loff] = v;
  };
  auto put1 = [&](int col, double v) {
    if (has1) w1[(int64_t)col * KC + loff] = (T)v;
    if (has1d) d1[(int64_t)col * KC + loff] = v;
  };
  if (g >= G.npts) {  // padding points: every column exactly zero
    if (S.mode == EV_WEIGHTS) {
      for (int it = 0; it < S.n_items; ++it) put0(wcols[S.item_off + it].col, 0.0);
    } else {
      for (int s = S.item_off; s < S.item_off + S.n_items; ++s) {
        const ShellDev sh = shells[s];
        for (int e = 0; e < sh.nm; ++e) {
          const int col = ments[sh.m_off + e].col;
          if (col < 0) continue;
          put0(col, 0.0);
          if (S.mode == EV_CHI_KIN) put1(col, 0.0);
        }
      }
    }
    return;
  }
  if (S.skip) {
    // cells a shared segment writes (Q = 4: a wave's 64 points are one cell, so whole waves leave)
    const int64_t c = g >> 6;
    if (c < G.n_reg) {
      const int64_t plane = (int64_t)G.nnu * G.nphi;
      const int i = (int)(c / plane), j = (int)((c - (int64_t)i * plane) / G.nphi);
      if (((S.skip_mu[i >> 6] >> (i & 63)) & 1) && ((S.skip_nu[j >> 6] >> (j & 63)) & 1)) return;
    }
  }
  Geo geo;
  point_geo(G, lines, g, geo);
  if (S.mode == EV_WEIGHTS) {
    for (int it = 0; it < S.n_items; ++it) {
      const WColDev W = wcols[S.item_off + it];
      double v;
      if (W.kind == 0) v = geo.w;
      else if (W.kind == 1) v = 1.0;
      else {
        double pot = W.zA / geo.r[0] + W.zB / geo.r[1];
        if (W.zC != 0.0) pot += W.zC / geo.r[2];
        v = -geo.w * pot;
      }
      put0(W.col, v);
    }
    return;
  }
  // select the segment's centre without dynamic indexing (keeps Geo in registers)
  const int cen = S.centre;
  const double r = cen == 0 ? geo.r[0] : (cen == 1 ? geo.r[1] : geo.r[2]);
  const double dx = cen == 0 ? geo.d[0][0] : (cen == 1 ? geo.d[1][0] : geo.d[2][0]);
  const double dy = cen == 0 ? geo.d[0][1] : (cen == 1 ? geo.d[1][1] : geo.d[2][1]);
  const double dz = cen == 0 ? geo.d[0][2] : (cen == 1 ? geo.d[1][2] : geo.d[2][2]);
  const double ir = 1.0 / r;
  const double x = dx * ir, y = dy * ir, z = dz * ir;
  // harmonics of even degrees in (Pc, Ps), odd degrees in (Qc, Qs)
  double Pc[LMAX + 1], Ps[LMAX + 1], Qc[LMAX + 1], Qs[LMAX + 1];
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) Pc[m] = Ps[m] = Qc[m] = Qs[m] = 0.0;
  int lmax_seg = 0;
  for (int l = 0; l <= LMAX; ++l)
    if (S.l_off[l + 1] > S.l_off[l]) lmax_seg = l;
  // the shells of degree l, whose harmonics are (C, Sv)
  auto shells_of = [&](int l, const double* C, const double* Sv) __attribute__((always_inline)) {
    for (int s = S.l_off[l]; s < S.l_off[l + 1]; ++s) {
      const ShellDev sh = shells[s];
      const double ex = exp(-sh.zeta * r);
      double rad, kin = 0.0;
      if (S.mode == EV_POT_W) {
        const double xx = sh.zeta * r;
        double lower, upper;
        inc_gamma_pair(sh.n + l + 2, sh.n - l + 1, xx, ex, &lower, &upper);
        const double ixx = 1.0 / xx;
        rad = geo.w * sh.pre * (ipow(ixx, l + 1) * lower + ipow(xx, l) * upper);
      } else {
        rad = sh.norm * ipow(r, sh.n - 1) * ex;
        if (S.mode == EV_CHI_KIN) {
          const double f = sh.zeta * sh.zeta - 2.0 * sh.zeta * sh.n * ir +
                           (sh.n * (sh.n - 1.0) - l * (l + 1.0)) * ir * ir;
          kin = -0.5 * f * rad;
        }
      }
      // components m = +mm (C) and -mm (S) for each |m| = mm <= l: the entries are dense in m, so
      // the harmonic is a fixed register for each unrolled mm
      // (all of the shell's entries are loaded before its first store)
      const MEntry* __restrict__ me0 = ments + sh.m_off + l;  // m = 0
      MEntry ep[LMAX + 1], en[LMAX + 1];
#pragma unroll
      for (int mm = 0; mm <= LMAX; ++mm) {
        if (mm > l) break;
        ep[mm] = me0[mm];
        en[mm] = me0[-mm];
      }
#pragma unroll
      for (int mm = 0; mm <= LMAX; ++mm) {
        if (mm > l) break;
        if (ep[mm].col >= 0) {
          const double Yh = C[mm] * ep[mm].f;
          put0(ep[mm].col, rad * Yh);
          if (S.mode == EV_CHI_KIN) put1(ep[mm].col, kin * Yh);
        }
        if (mm > 0 && en[mm].col >= 0) {
          const double Yh = Sv[mm] * en[mm].f;
          put0(en[mm].col, rad * Yh);
          if (S.mode == EV_CHI_KIN) put1(en[mm].col, kin * Yh);
        }
      }
    }
  };
  for (int l = 0; l <= lmax_seg; l += 2) {
    harmonic_level(l, x, y, z, Qc, Qs, Pc, Ps);
    shells_of(l, Pc, Ps);
    if (l + 1 > lmax_seg) break;
    harmonic_level(l + 1, x, y, z, Pc, Ps, Qc, Qs);
    shells_of(l + 1, Qc, Qs);
  }
}

// ------------------------------------------------------------------------------------------------
// Shared evaluation (ShareSegDev): one wave per shared cell (Q = 4), one thread per point.  The
// local coordinates and the distance to the segment's centre follow point_geo for a regular cell;
// the displacement in each member's frame is that grid's own (lx ex + ly ey + lz ez).  Per shell the
// radial factor is computed once for all members; the harmonics of each degree are rebuilt per member
// from degree 0 (a few multiply-adds against the exp and power the members share).
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void eval_shared_kernel(const ShareSegDev* __restrict__ segs, int nseg,
                                                          const GridDev* __restrict__ grids,
                                                          const double* __restrict__ lines,
                                                          const ShellDev* __restrict__ shells,
                                                          const MEntry* __restrict__ ments) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const ShareSegDev& S = segs[lo];
  const ShareMember* __restrict__ mem = S.members;
  const GridDev& G0 = grids[mem[0].grid];
  const int lane = threadIdx.x & 63;
  const int64_t wv = (b - S.block0) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ncell = (int64_t)S.n_si * S.n_sj * G0.nphi;
  if (wv >= ncell) return;
  const int k = (int)(wv % G0.nphi);
  const int64_t t2 = wv / G0.nphi;
  const int i = S.cells[t2 / S.n_sj], j = S.cells[S.n_si + (int)(t2 % S.n_sj)];
  const int64_t gw = (((int64_t)i * G0.nnu + j) * G0.nphi + k) * 64;  // the cell's first point
  // point (p, q, r) = lane of the cell, as point_geo maps a regular cell (no split)
  const int ip = lane >> 4, iq = (lane >> 2) & 3, ir = lane & 3;
  const double* mu = lines + G0.lines;
  const double* nu = mu + G0.nmu + 1;
  const double* ph = nu + G0.nnu + 1;
  const double* glx = lines + G0.gl;
  const double inv = 1.0;
  const double hm = (mu[i + 1] - mu[i]) * inv, hn = (nu[j + 1] - nu[j]) * inv, hp = (ph[k + 1] - ph[k]) * inv;
  const double m = mu[i] + hm * (0 + 0.5 * (1.0 + glx[ip]));
  const double n = nu[j] + hn * (0 + 0.5 * (1.0 + glx[iq]));
  const double f = ph[k] + hp * (0 + 0.5 * (1.0 + glx[ir]));
  const double shh = sinh(0.5 * m);
  const double s2 = shh * shh;
  const double chh = sqrt(1.0 + s2);
  double sn2, cs2, sf, cf;
  sincos(0.5 * n, &sn2, &cs2);
  sincos(f, &sf, &cf);
  const double sh = 2.0 * shh * chh;
  const double sn = 2.0 * sn2 * cs2, cs = (cs2 - sn2) * (cs2 + sn2);
  const double a = G0.a;
  const double rho = a * sh * sn;
  const double lx = rho * cf, ly = rho * sf;
  const bool onA = S.centre == CEN_A;
  const double lz = onA ? a * (2.0 * s2 * cs - 2.0 * sn2 * sn2) : a * (2.0 * s2 * cs + 2.0 * cs2 * cs2);
  const double r = onA ? 2.0 * a * (s2 + sn2 * sn2) : 2.0 * a * (s2 + cs2 * cs2);
  const double ir_ = 1.0 / r;
  typedef __attribute__((address_space(1))) T GT;
  typedef __attribute__((address_space(1))) double GD;
  const uint32_t loff = (uint32_t)((lane >> 4) * S.nf * KC + (lane & 15));
  int lmax_seg = 0;
  for (int l = 0; l <= LMAX; ++l)
    if (S.l_off[l + 1] > S.l_off[l]) lmax_seg = l;
  constexpr int GROUP = 8;  // shells of one degree whose radial factors are held at once
  for (int l = 0; l <= lmax_seg; ++l) {
    for (int s0 = S.l_off[l]; s0 < S.l_off[l + 1]; s0 += GROUP) {
      const int ns = min(GROUP, S.l_off[l + 1] - s0);
      double rad[GROUP];
#pragma unroll
      for (int u = 0; u < GROUP; ++u) {
        rad[u] = 0.0;
        if (u < ns) {
          const ShellDev shl = shells[s0 + u];
          const double ex = exp(-shl.zeta * r);
          rad[u] = shl.norm * ipow(r, shl.n - 1) * ex;
        }
      }
      for (int c = 0; c < S.n_members; ++c) {
        const GridDev& G = grids[mem[c].grid];
        const double dx = lx * G.ex[0] + ly * G.ey[0] + lz * G.ez[0];
        const double dy = lx * G.ex[1] + ly * G.ey[1] + lz * G.ez[1];
        const double dz = lx * G.ex[2] + ly * G.ey[2] + lz * G.ez[2];
        const double x = dx * ir_, y = dy * ir_, z = dz * ir_;
        // even degrees in (Pc, Ps), odd degrees in (Qc, Qs); degree l ends in the set of its parity
        double Pc[LMAX + 1], Ps[LMAX + 1], Qc[LMAX + 1], Qs[LMAX + 1];
#pragma unroll
        for (int mm = 0; mm <= LMAX; ++mm) Pc[mm] = Ps[mm] = Qc[mm] = Qs[mm] = 0.0;
        for (int ll = 0; ll <= l; ll += 2) {
          harmonic_level(ll, x, y, z, Qc, Qs, Pc, Ps);
          if (ll + 1 > l) break;
          harmonic_level(ll + 1, x, y, z, Pc, Ps, Qc, Qs);
        }
        const bool odd = (l & 1) != 0;
        GT* __restrict__ w0 = (GT*)mem[c].arr0 + gw * S.nf;
        GD* __restrict__ d0 = (GD*)mem[c].arr0d + gw * S.nf;
        const bool has0 = mem[c].arr0 != nullptr, has0d = sizeof(T) == 4 && mem[c].arr0d != nullptr;
#pragma unroll
        for (int u = 0; u < GROUP; ++u) {
          if (u >= ns) break;
          const ShellDev shl = shells[s0 + u];
          const MEntry* __restrict__ me0 = ments + shl.m_off + l;
#pragma unroll
          for (int mm = 0; mm <= LMAX; ++mm) {
            if (mm > l) break;
            const MEntry ep = me0[mm], en = me0[-mm];
            if (ep.col >= 0) {
              const double v = rad[u] * ((odd ? Qc[mm] : Pc[mm]) * ep.f);
              if (has0) w0[(int64_t)ep.col * KC + loff] = (T)v;
              if (has0d) d0[(int64_t)ep.col * KC + loff] = v;
            }
            if (mm > 0 && en.col >= 0) {
              const double v = rad[u] * ((odd ? Qs[mm] : Ps[mm]) * en.f);
              if (has0) w0[(int64_t)en.col * KC + loff] = (T)v;
              if (has0d) d0[(int64_t)en.col * KC + loff] = v;
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Contraction kernels.  256 threads = 4 waves, WR along the rows and 4 / WR along the columns (2 x 2,
// or 4 x 1 for tiles whose width is an odd number of 16-column blocks); wave (wm, wn) owns WM x WN
// MFMA blocks of 16 x 16.  Points are consumed in stages of SC storage chunks (SC * 16 points).  Each
// stage's U, V and Y columns sit in LDS as padded rows of SC * 16 values (bank-conflict-free operand
// reads); two LDS buffers alternate, so one barrier per stage suffices: while the MFMAs of stage s run
// on one buffer, direct global->LDS copies fill the other with stage s+1, issued between the MFMA
// steps.
//
// Operand layouts (probed on gfx950): A lane l = A[l%16][l/16], B lane l = B[l/16][l%16];
// v_mfma_f64_16x16x4 result register r of lane l = D[4r + l/16][l%16];
// v_mfma_f32_16x16x4f32 result register r of lane l = D[4(l/16) + r][l%16].
// ------------------------------------------------------------------------------------------------
template <typename T, int WM, int WN, int SC_, int WR = 2>
struct ContractCfg {
  static constexpr int WC = 4 / WR;                     // waves along the columns
  static constexpr int BM = 16 * WM * WR, BN = 16 * WN * WC;
  static constexpr int SC = SC_;                        // storage chunks per stage
  static constexpr int KS = SC * KC;                    // points per stage
  // padded LDS row: FP64 rows 34 doubles (68 words: 16 consecutive rows at the same k fall in distinct
  // banks within a half-wave), FP32 rows 36 floats (same property)
  static constexpr int LDK = KS + (sizeof(T) == 8 ? 2 : 4);
  static constexpr int SLOTS = LDK * (int)sizeof(T) / 16;       // 16-byte slots per row
  static constexpr int DSLOTS = KS * (int)sizeof(T) / 16;       // slots holding data
  static constexpr int VN = 16 / (int)sizeof(T);                // values per slot
  static constexpr int OVER = (63 + SLOTS - 1) / SLOTS;         // rows a 64-slot copy can overshoot
  static constexpr int MAXUV = BM + 4 + OVER;           // the host keeps nu + nv <= BM + 4
  static constexpr int ROWS = MAXUV + BN + OVER;
  static constexpr int BUF = ROWS * LDK;                // elements per stage buffer
  static constexpr int LDS_BYTES = 2 * BUF * (int)sizeof(T);
};

// Instruction classes of __builtin_amdgcn_sched_group_barrier (LLVM AMDGPU scheduling groups).
constexpr int SG_VALU = 0x002, SG_MFMA = 0x008, SG_DSR = 0x100;

// One work-group's tile: C[(u,v)][y] partial over chunks [kc0, kc0 + nkc) (nkc a multiple of SC).
//
// Staging uses direct global->LDS copies (global_load_lds_dwordx4): one wave instruction fills 64
// consecutive 16-byte LDS slots (lane i -> slot base + i) of a region of contiguous rows, the U+V
// rows [0, nu+nv) or the Y rows [MAXUV, MAXUV+np).  Each thread's source offset for every copy it
// issues is computed once per tile; per stage only the chunk base moves.  The copies of stage s+1
// are spread between the MFMA steps of stage s so their address work hides under the matrix pipe.
template <typename T, int WM, int WN, int SC_, int WR>
__device__ __forceinline__ void contract_body(const TaskDev& __restrict__ Tk, const TileDev& t,
                                              __attribute__((address_space(3))) T* lds, double* __restrict__ ws) {
  typedef ContractCfg<T, WM, WN, SC_, WR> Cf;
  constexpr int BN = Cf::BN, LDK = Cf::LDK, MAXUV = Cf::MAXUV, KS = Cf::KS, SC = Cf::SC, BUF = Cf::BUF;
  constexpr int SLOTS = Cf::SLOTS, DSLOTS = Cf::DSLOTS, VN = Cf::VN;
  constexpr int NCUV = (MAXUV * SLOTS + 255) / 256;  // copies per thread per stage, U+V region (max)
  constexpr int NCY = (BN * SLOTS + 255) / 256;      // Y region (max)
  constexpr int KSTEPS = KS / 4;
  // FP64: MFMA steps over which the next stage's copies are issued (steps are long enough to hide
  // them in the first two); the FP32 paths spread them over all of the stage's step pairs
  constexpr int CSPREAD = KSTEPS > 2 ? 2 : KSTEPS;
  constexpr bool F64 = sizeof(T) == 8;
  // FP32 tiles of more than 8 blocks per wave: stage sums kept per row block (row-block-outer step
  // order) rather than for the whole tile, which keeps a 4 x 4 tile within two waves per SIMD
  constexpr bool ROWOUTER = !F64 && WM * WN > 8;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform, lets tests below be scalar
  const int wm = wave / Cf::WC, wn = wave % Cf::WC;
  const int kl = lane >> 4;

  // Rows beyond nrows and columns beyond np are computed on whatever their (in-bounds) LDS rows hold
  // and never read back: an MFMA output row depends only on its A row and an output column only on
  // its B column, and the reduction skips both.  So the operands need no masking.
  // Points of a stage per MFMA step: FP64, step kk takes point 4 kk + kl from lane group kl; FP32,
  // steps 2m and 2m + 1 take points 8m + 2 kl and 8m + 2 kl + 1, which one 8-byte LDS read per lane
  // fetches for both steps (16 rows at the 36-float row stride read 4 bytes per lane fall into the
  // same LDS bank in pairs, rows j and j + 8; read as 8-byte pairs they do not, and half as many
  // read instructions move the same bytes).  A and B use the same assignment, so every point enters
  // every sum once.
  const int koff = F64 ? kl : 2 * kl;
  int offU[WM], offV[WM];
#pragma unroll
  for (int mb = 0; mb < WM; ++mb) {
    const int row = wm * 16 * WM + mb * 16 + (lane & 15);
    int u = t.ulo, v = t.vlo;
    if (row < t.nrows) {
      u = Tk.pairs[2 * (t.row0 + row)];
      v = Tk.pairs[2 * (t.row0 + row) + 1];
    }
    offU[mb] = (u - t.ulo) * LDK + koff;
    offV[mb] = (t.nu + v - t.vlo) * LDK + koff;
  }
  int offY[WN];
#pragma unroll
  for (int nb = 0; nb < WN; ++nb) {
    const int col = wn * 16 * WN + nb * 16 + (lane & 15);
    offY[nb] = (MAXUV + col) * LDK + koff;
  }

  const T* __restrict__ Ub = (const T*)Tk.U + (int64_t)t.ulo * KC;
  const T* __restrict__ Vb = (const T*)Tk.V + (int64_t)t.vlo * KC;
  const T* __restrict__ Yb = (const T*)Tk.Y + (int64_t)(Tk.y0 + t.p0) * KC;
  const int64_t sU = (int64_t)Tk.nfU * KC, sV = (int64_t)Tk.nfV * KC, sY = (int64_t)Tk.nfY * KC;
  const int nstage = (int)(t.nkc / SC);
  const int nslot_uv = (t.nu + t.nv) * SLOTS, nslot_y = t.np * SLOTS;

  // per-thread copy descriptors: element offset from the stage's chunk base; bit 30 marks a V source
  int cuv[NCUV], cy[NCY];
#pragma unroll
  for (int i = 0; i < NCUV; ++i) {
    const int slot = wave * 64 + 256 * i + lane;
    const int row = slot / SLOTS, q = slot - row * SLOTS;
    int d = 0;
    if (slot < nslot_uv && q < DSLOTS) {
      const int e = q * VN, j = e / KC, k = e - j * KC;
      d = row < t.nu ? (int)(j * sU) + row * KC + k : ((int)(j * sV) + (row - t.nu) * KC + k) | (1 << 30);
    }
    cuv[i] = d;
  }
#pragma unroll
  for (int i = 0; i < NCY; ++i) {
    const int slot = wave * 64 + 256 * i + lane;
    const int row = slot / SLOTS, q = slot - row * SLOTS;
    int d = 0;
    if (slot < nslot_y && q < DSLOTS) {
      const int e = q * VN, j = e / KC, k = e - j * KC;
      d = (int)(j * sY) + row * KC + k;
    }
    cy[i] = d;
  }
  // copy i of the U+V region (i < NCUV) or Y region (NCUV <= i < NCUV + NCY) of stage s
  auto copy = [&](int s, int i) {
    __attribute__((address_space(3))) T* b = lds + (s & 1) * BUF;
    const int64_t c = t.kc0 + (int64_t)s * SC;
    if (i < NCUV) {
      const int base = wave * 64 + 256 * i;
      if (base < nslot_uv) {
        const int d = cuv[i];
        const T* src = (d & (1 << 30)) ? Vb + c * sV + (d & ~(1 << 30)) : Ub + c * sU + d;
        __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)(b + base * VN),
                                         16, 0, 0);
      }
    } else {
      const int ii = i - NCUV;
      const int base = wave * 64 + 256 * ii;
      if (base < nslot_y) {
        const T* src = Yb + c * sY + cy[ii];
        __builtin_amdgcn_global_load_lds((const void*)src,
                                         (__attribute__((address_space(3))) void*)(b + MAXUV * LDK + base * VN), 16,
                                         0, 0);
      }
    }
  };

  d4_t acc[WM][WN];
#pragma unroll
  for (int mb = 0; mb < WM; ++mb)
#pragma unroll
    for (int nb = 0; nb < WN; ++nb) acc[mb][nb] = (d4_t){0.0, 0.0, 0.0, 0.0};

  // Operand registers, two slots: the next step's operands are read from LDS while the current
  // step's MFMAs run (FP32: the next step pair's).  The barrier that ends stage s sits before the
  // MFMAs of its last step (step pair), whose operands are already in registers; the first operands
  // of stage s + 1 are read right after it, into the slot the last step leaves free, so those MFMAs
  // cover the LDS latency at the stage boundary.
  T uA[2][WM], vA[2][WM], yB[2][WN];  // FP64 whole-tile step order
  typedef float f2_t __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(3))) f2_t* L2p;
  f2_t uP[2][WM], vP[2][WM], yP[2][WN];  // FP32 whole-tile order, one step pair per slot
  f2_t ru[2], rv[2], ry[2][WN];          // FP32 row-block-outer order, one step pair per slot
  // FP32: operands of step pair m (steps 2m, 2m + 1) as 8-byte reads
  auto fetchp = [&](const __attribute__((address_space(3))) T* cur, int m, int slot) {
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      uP[slot][mb] = *(L2p)(cur + offU[mb] + 8 * m);
      vP[slot][mb] = *(L2p)(cur + offV[mb] + 8 * m);
    }
#pragma unroll
    for (int nb = 0; nb < WN; ++nb) yP[slot][nb] = *(L2p)(cur + offY[nb] + 8 * m);
  };
  auto fetch = [&](const __attribute__((address_space(3))) T* cur, int kk, int slot) {
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      uA[slot][mb] = cur[offU[mb] + 4 * kk];
      vA[slot][mb] = cur[offV[mb] + 4 * kk];
    }
#pragma unroll
    for (int nb = 0; nb < WN; ++nb) yB[slot][nb] = cur[offY[nb] + 4 * kk];
  };
  // FP32 row-block-outer: iteration it = (row block mb, step pair m)
  constexpr int NPAIR = KSTEPS / 2;
  auto fetch1 = [&](const __attribute__((address_space(3))) T* cur, int it, int slot) {
    const int mb = it / NPAIR, m = it - mb * NPAIR;
    ru[slot] = *(L2p)(cur + offU[mb] + 8 * m);
    rv[slot] = *(L2p)(cur + offV[mb] + 8 * m);
#pragma unroll
    for (int nb = 0; nb < WN; ++nb) ry[slot][nb] = *(L2p)(cur + offY[nb] + 8 * m);
  };
  // FP64, before the last step's MFMAs of stage s (uniform): wait for this wave's copies of stage
  // s + 1, barrier, then read the first operands of stage s + 1 into slot 0
  auto boundary = [&](int s) {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    fetch(lds + ((s + 1) & 1) * BUF, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };

  if (nstage > 0) {
#pragma unroll
    for (int i = 0; i < NCUV + NCY; ++i) copy(0, i);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if constexpr (F64) {
    if (nstage > 0) fetch(lds, 0, 0);
  } else if constexpr (ROWOUTER) {
    if (nstage > 0) fetch1(lds, 0, 0);
  } else {
    if (nstage > 0) fetchp(lds, 0, 0);
  }
  // FP32 row-block-outer order: the stage sums of the row block in progress.  They are carried
  // from one row block to the next, and from one stage to the next, until the first step of the
  // following row block folds them into that block's FP64 accumulators (zeros before the first stage).
  f4_t s32[WN];
#pragma unroll
  for (int nb = 0; nb < WN; ++nb) s32[nb] = f4_t{};
  // FP32 whole-tile order: the stage sums of every block, folded during the next stage's first
  // step pair (zeros before the first stage)
  f4_t a32[WM][WN];
#pragma unroll
  for (int mb = 0; mb < WM; ++mb)
#pragma unroll
    for (int nb = 0; nb < WN; ++nb) a32[mb][nb] = f4_t{};
  // one stage: MFMAs on the current buffer, copies of the next stage into the other
  auto run_stage = [&](int s) {
    const bool more = s + 1 < nstage;
    const __attribute__((address_space(3))) T* cur = lds + (s & 1) * BUF;
    if constexpr (ROWOUTER) {
      // FP32: one row block at a time over the stage's steps, so only WN blocks of FP32 stage sums
      // are live.  The Y operands are read from LDS once per row block.  A row block's sums go into
      // its FP64 accumulators during the first step of the next row block, block by block just
      // before the MFMA that restarts that block's sums: the MFMAs that produced them completed a
      // whole step earlier, so the fold waits on nothing and runs beside the matrix pipe.
      constexpr int NIT = WM * NPAIR;  // even: the first operands of a stage are always in slot 0
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int mb = it / NPAIR, m = it % NPAIR, sl = it & 1;
        if (it + 1 < NIT) fetch1(cur, it + 1, sl ^ 1);
        const float av0 = ru[sl].x * rv[sl].x, av1 = ru[sl].y * rv[sl].y;
        f2_t bv[WN];
#pragma unroll
        for (int nb = 0; nb < WN; ++nb) bv[nb] = ry[sl][nb];
        if (it + 1 == NIT && more) {
          // before the stage's last MFMAs: wait for this wave's copies of stage s + 1, barrier, then
          // read its first operands, which those MFMAs cover
          __builtin_amdgcn_sched_barrier(0);
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          __syncthreads();
          fetch1(lds + ((s + 1) & 1) * BUF, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (m == 0) {
          const int pb = (mb + WM - 1) % WM;  // the previous row block (of the previous stage at mb = 0)
#pragma unroll
          for (int nb = 0; nb < WN; ++nb) {
            d4_t a = acc[pb][nb];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] += (double)s32[nb][r];
            asm volatile("" : "+v"(a));  // keeps the fold here rather than sunk to the end of the stage
            acc[pb][nb] = a;
            s32[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, bv[nb].x, f4_t{}, 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int nb = 0; nb < WN; ++nb)
            s32[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, bv[nb].x, s32[nb], 0, 0, 0);
        }
#pragma unroll
        for (int nb = 0; nb < WN; ++nb)
          s32[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1, bv[nb].y, s32[nb], 0, 0, 0);
        // issue order (left to itself the compiler's scheduler issues the next step pair's LDS reads
        // right before their use and waits for them there): the pair products, then the first WN
        // MFMAs with the next operands' reads two at a time between them (each block's fold before
        // its MFMA when a row block starts), then the second WN MFMAs
        constexpr int NRD = 2 + WN;  // LDS reads of the next step pair
        __builtin_amdgcn_sched_group_barrier(SG_VALU, 2, 0);
#pragma unroll
        for (int nb = 0; nb < WN; ++nb) {
          if (m == 0) __builtin_amdgcn_sched_group_barrier(SG_VALU, 8, 0);
          __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
          if (2 * nb + 1 < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 2, 0);
          else if (2 * nb < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(SG_MFMA, WN, 0);
        if constexpr (2 * WN < NRD) __builtin_amdgcn_sched_group_barrier(SG_DSR, NRD - 2 * WN, 0);
        __builtin_amdgcn_sched_barrier(0);
        // the next stage's copies, over every iteration but the last (whose barrier they precede)
        if (more) {
#pragma unroll
          for (int i = 0; i < NCUV + NCY; ++i)
            if (i % (NIT - 1) == it) copy(s + 1, i);
        }
      }
      return;
    }
    if constexpr (!F64) {
      // FP32 whole tile, one step pair per iteration.  The previous stage's sums go into the FP64
      // accumulators during this stage's first step pair, each block's just before the MFMA that
      // restarts it (as in the row-block-outer order).
#pragma unroll
      for (int m = 0; m < NPAIR; ++m) {
        const int sl = m & 1;  // NPAIR is even: the first operands of a stage are in slot 0
        if (m + 1 < NPAIR) fetchp(cur, m + 1, sl ^ 1);
        float av[2][WM];
#pragma unroll
        for (int mb = 0; mb < WM; ++mb) {
          av[0][mb] = uP[sl][mb].x * vP[sl][mb].x;
          av[1][mb] = uP[sl][mb].y * vP[sl][mb].y;
        }
        if (m + 1 == NPAIR && more) {
          __builtin_amdgcn_sched_barrier(0);
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          __syncthreads();
          fetchp(lds + ((s + 1) & 1) * BUF, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int mb = 0; mb < WM; ++mb)
#pragma unroll
          for (int nb = 0; nb < WN; ++nb) {
            if (m == 0) {
              d4_t a = acc[mb][nb];
#pragma unroll
              for (int r = 0; r < 4; ++r) a[r] += (double)a32[mb][nb][r];
              asm volatile("" : "+v"(a));  // keeps the fold here rather than sunk to the end of the stage
              acc[mb][nb] = a;
            }
            a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][mb], yP[sl][nb].x,
                                                               m == 0 ? f4_t{} : a32[mb][nb], 0, 0, 0);
          }
#pragma unroll
        for (int mb = 0; mb < WM; ++mb)
#pragma unroll
          for (int nb = 0; nb < WN; ++nb)
            a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][mb], yP[sl][nb].y, a32[mb][nb], 0, 0, 0);
        // issue order: the pair products, then the first WM x WN MFMAs with the next operands' reads
        // two at a time between them (and each block's fold before its MFMA in the first step
        // pair), then the second WM x WN MFMAs
        constexpr int NRD = 2 * WM + WN;
        __builtin_amdgcn_sched_group_barrier(SG_VALU, 2 * WM, 0);
#pragma unroll
        for (int b = 0; b < WM * WN; ++b) {
          if (m == 0) __builtin_amdgcn_sched_group_barrier(SG_VALU, 8, 0);
          __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
          if (2 * b + 1 < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 2, 0);
          else if (2 * b < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(SG_MFMA, WM * WN, 0);
        if constexpr (2 * WM * WN < NRD) __builtin_amdgcn_sched_group_barrier(SG_DSR, NRD - 2 * WM * WN, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (more) {
#pragma unroll
          for (int i = 0; i < NCUV + NCY; ++i)
            if (i % (NPAIR - 1) == m) copy(s + 1, i);
        }
      }
      return;
    }
    // FP64: one step per iteration
#pragma unroll
    for (int kk = 0; kk < KSTEPS; ++kk) {
      const int sl = kk & 1;
      if (kk + 1 < KSTEPS) fetch(cur, kk + 1, sl ^ 1);
      T av[WM], bv[WN];
#pragma unroll
      for (int mb = 0; mb < WM; ++mb) av[mb] = uA[sl][mb] * vA[sl][mb];
#pragma unroll
      for (int nb = 0; nb < WN; ++nb) bv[nb] = yB[sl][nb];
      if (kk + 1 == KSTEPS && more) boundary(s);
#pragma unroll
      for (int mb = 0; mb < WM; ++mb)
#pragma unroll
        for (int nb = 0; nb < WN; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
      // issue order: the pair products, then the MFMAs with the next step's LDS reads two at a time
      // between the first ones
      {
        constexpr int NRD = 2 * WM + WN;
        __builtin_amdgcn_sched_group_barrier(SG_VALU, WM, 0);
#pragma unroll
        for (int b = 0; b < WM * WN; ++b) {
          __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
          if (2 * b + 1 < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 2, 0);
          else if (2 * b < NRD)
            __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
        }
        if constexpr (2 * WM * WN < NRD) __builtin_amdgcn_sched_group_barrier(SG_DSR, NRD - 2 * WM * WN, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the next stage's copies, spread over the steps (into the other buffer)
      if (more) {
#pragma unroll
        for (int i = 0; i < NCUV + NCY; ++i)
          if (i % CSPREAD == kk) copy(s + 1, i);
      }
    }
  };
  for (int s = 0; s < nstage; ++s) run_stage(s);
  if constexpr (ROWOUTER) {
    // the last row block's sums
#pragma unroll
    for (int nb = 0; nb < WN; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[WM - 1][nb][r] += (double)s32[nb][r];
  } else if constexpr (!F64) {
    // the last stage's sums
#pragma unroll
    for (int mb = 0; mb < WM; ++mb)
#pragma unroll
      for (int nb = 0; nb < WN; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += (double)a32[mb][nb][r];
  }
  double* __restrict__ wt = ws + t.ws;
#pragma unroll
  for (int mb = 0; mb < WM; ++mb)
#pragma unroll
    for (int nb = 0; nb < WN; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 16 * WM + mb * 16 + (F64 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r);
        const int col = wn * 16 * WN + nb * 16 + (lane & 15);
        wt[row * BN + col] = acc[mb][nb][r];
      }
}

template <int WM, int WN, int SC, int WR>
__global__ __launch_bounds__(256, 1) void contract_f64(const TaskDev* __restrict__ tasks,
                                                       const TileDev* __restrict__ tiles,
                                                       double* __restrict__ ws) {
  extern __shared__ __attribute__((aligned(16))) double smem_d[];
  const TileDev t = tiles[blockIdx.x];
  contract_body<double, WM, WN, SC, WR>(tasks[t.task], t, (__attribute__((address_space(3))) double*)smem_d, ws);
}

// The 128-row shapes of a pass in one launch: each tile runs the body of the shape it names
// (kMergedShapes).  The kernel's registers and LDS are those of its largest shape (128 x 128): two
// work-groups per CU, which the LDS of every other shape of this family allows on its own too, except
// the two narrowest (128 x 32 and the tall 128 x 16, three).  One launch instead of up to eight drains
// the device once per pass.
template <typename T, int SC>
__device__ __forceinline__ void contract_merged_body(const TaskDev* __restrict__ tasks, const TileDev& t,
                                                     __attribute__((address_space(3))) T* lds,
                                                     double* __restrict__ ws) {
  constexpr auto& M = kMergedShapes;
  const TaskDev& Tk = tasks[t.task];
  switch (t.shape) {
    case 0: contract_body<T, M[0][0], M[0][1], SC, M[0][2]>(Tk, t, lds, ws); break;
    case 1: contract_body<T, M[1][0], M[1][1], SC, M[1][2]>(Tk, t, lds, ws); break;
    case 2: contract_body<T, M[2][0], M[2][1], SC, M[2][2]>(Tk, t, lds, ws); break;
    case 3: contract_body<T, M[3][0], M[3][1], SC, M[3][2]>(Tk, t, lds, ws); break;
    case 4: contract_body<T, M[4][0], M[4][1], SC, M[4][2]>(Tk, t, lds, ws); break;
    case 5: contract_body<T, M[5][0], M[5][1], SC, M[5][2]>(Tk, t, lds, ws); break;
    case 6: contract_body<T, M[6][0], M[6][1], SC, M[6][2]>(Tk, t, lds, ws); break;
    default: contract_body<T, M[7][0], M[7][1], SC, M[7][2]>(Tk, t, lds, ws); break;
  }
}

template <int SC>
__global__ __launch_bounds__(256, 1) void contract_f64_merged(const TaskDev* __restrict__ tasks,
                                                              const TileDev* __restrict__ tiles,
                                                              double* __restrict__ ws) {
  extern __shared__ __attribute__((aligned(16))) double smem_md[];
  const TileDev t = tiles[blockIdx.x];
  contract_merged_body<double, SC>(tasks, t, (__attribute__((address_space(3))) double*)smem_md, ws);
}

template <int SC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void contract_mixed_merged(
    const TaskDev* __restrict__ tasks, const TileDev* __restrict__ tiles, double* __restrict__ ws) {
  extern __shared__ __attribute__((aligned(16))) float smem_mf[];
  const TileDev t = tiles[blockIdx.x];
  contract_merged_body<float, SC>(tasks, t, (__attribute__((address_space(3))) float*)smem_mf, ws);
}

// Two waves per SIMD asked of the compiler: the widest FP32 tile then keeps its FP64 accumulators
// and operands in VGPRs rather than splitting them into AGPRs (measured 2% faster than leaving the
// allocation free).
template <int WM, int WN, int SC, int WR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void contract_mixed(const TaskDev* __restrict__ tasks,
                                                         const TileDev* __restrict__ tiles,
                                                         double* __restrict__ ws) {
  extern __shared__ __attribute__((aligned(16))) float smem_f[];
  const TileDev t = tiles[blockIdx.x];
  contract_body<float, WM, WN, SC, WR>(tasks[t.task], t, (__attribute__((address_space(3))) float*)smem_f, ws);
}

// Sum the splits of each reduction item in order and scatter into the FP64 output buffer.  Partial
// tiles are row-major with R.bn columns (a multiple of 32, every entry written by the contraction).
// A thread takes one pair row and 16 consecutive columns: per split it reads one whole 128-byte line
// of the partial tile, so no line is fetched for a single value.  Consecutive threads take
// consecutive pair rows: for (ab|P) those are consecutive b, so the output writes are contiguous.
// Each item is shared by `spread` consecutive work-groups (interleaved 256-thread slices of its
// rows), so that launches of few items still fill the device; every output element is still summed
// by one thread in split order.
__global__ __launch_bounds__(256) void reduce_kernel(const TaskDev* __restrict__ tasks,
                                                     const RedDev* __restrict__ reds,
                                                     const int32_t* __restrict__ items,
                                                     const double* __restrict__ ws, int spread) {
  const int part = blockIdx.x % spread;
  const RedDev R = reds[items[blockIdx.x / spread]];
  const TaskDev& T = tasks[R.task];
  const int64_t tile = (int64_t)R.bm * R.bn;
  const int ngrp = (R.np + 15) / 16;
  for (int e = part * 256 + threadIdx.x; e < R.nrows * ngrp; e += 256 * spread) {
    const int cg = e / R.nrows, row = e - cg * R.nrows;
    const int c0 = 16 * cg, nc = min(16, R.np - c0);
    double sum[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) sum[c] = 0.0;
    const double* p = ws + R.ws + (int64_t)row * R.bn + c0;
#pragma unroll 2
    for (int k = 0; k < R.nsplit; ++k) {
      const double2* q = (const double2*)(p + k * tile);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double2 v = q[c];
        sum[2 * c] += v.x;
        sum[2 * c + 1] += v.y;
      }
    }
    const int u = T.pairs[2 * (R.row0 + row)], v = T.pairs[2 * (R.row0 + row) + 1];
    const int64_t ia = T.mapU[u], ib = T.mapV[v];
    const bool mirror = T.outm && !(T.skip_diag && ia == ib);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c < nc) {
        const int64_t ip = T.mapY[T.y0 + R.p0 + c0 + c];
        const double val = T.alpha * sum[c];
        T.out[ia * T.s1 + ib * T.s2 + ip * T.s3] += val;
        if (mirror) T.outm[ia * T.t1 + ib * T.t2 + ip * T.t3] += val;
      }
    }
  }
}

// Matrix-pipe throughput probe: every wave runs `iters` (a multiple of 16) rounds of 8 independent
// 16 x 16 x 4 MFMAs (FP64, or FP32 inputs with FP32 sums) on register operands, and one sum per wave
// is stored so that the work is kept.  2048 FLOPs per MFMA.
template <typename T>
__global__ __launch_bounds__(256) void mfma_rate_kernel(double* __restrict__ out, int iters) {
  typedef typename std::conditional<sizeof(T) == 8, d4_t, f4_t>::type Acc;
  const int lane = threadIdx.x & 63;
  const T a = (T)(1.0 + 1e-3 * lane), b = (T)(1.0 - 1e-3 * lane);
  Acc acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = Acc{};
  // 16 rounds per loop trip: the accumulators stay in the matrix registers inside a trip
  for (int i = 0; i < iters; i += 16) {
#pragma unroll
    for (int ii = 0; ii < 16; ++ii)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (sizeof(T) == 8)
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        else
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
      }
  }
  double sum = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum += (double)acc[j][r];
  if (lane == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = sum;
}

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// X <- (X + X^T) / 2 for an n x n matrix (upper-triangle threads write both halves).
__global__ void symmetrize_kernel(double* __restrict__ X, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j <= i) continue;
    const double s = 0.5 * (X[(int64_t)i * n + j] + X[(int64_t)j * n + i]);
    X[(int64_t)i * n + j] = s;
    X[(int64_t)j * n + i] = s;
  }
}

// Blocked right-looking Cholesky in FP64, panel width CB = 32.  L starts as a copy of A.
// chol_panel: factor the CB x CB diagonal block in LDS (a pivot not larger than 1e-14 times the
// original diagonal entry of A sets *status and stops every later kernel).
// chol_trsm: the panel rows below it, L21 <- A21 L11^-T.
// chol_update: A22 <- A22 - L21 L21^T on the lower triangle, 64 x 64 tiles.
constexpr int CB = 32;

__global__ __launch_bounds__(256) void chol_panel(const double* __restrict__ A, double* __restrict__ L, int n, int k0,
                                                  int* __restrict__ status) {
  __shared__ double D[CB][CB + 1];
  __shared__ int bad;
  if (*status) return;
  const int tid = threadIdx.x;
  const int nb = min(CB, n - k0);
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    D[i][j] = (i < nb && j < nb && j <= i) ? L[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      const double d = D[k][k];
      if (!(d > 1e-14 * A[(int64_t)(k0 + k) * n + k0 + k])) bad = 1;
      else D[k][k] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    const double piv = D[k][k];
    if (tid > k && tid < nb) D[tid][k] /= piv;
    __syncthreads();
    for (int e = tid; e < CB * CB; e += 256) {
      const int i = e / CB, j = e % CB;
      if (j > k && i >= j && i < nb) D[i][j] -= D[i][k] * D[j][k];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *status = 1;
    return;
  }
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    if (i < nb && j <= i) L[(int64_t)(k0 + i) * n + k0 + j] = D[i][j];
  }
}

// Panel rows below the diagonal block: x D^T = a for each row.  Each wave solves two rows with one
// entry per lane (lanes 0-31 one row, 32-63 the next); x_p is broadcast with a lane shuffle.  A
// work-group takes TRSM_ROWS rows, so each wave runs two of the row pairs' serial chains.
constexpr int TRSM_ROWS = 16;
__global__ __launch_bounds__(256) void chol_trsm(double* __restrict__ L, int n, int k0, const int* __restrict__ status) {
  __shared__ double D[CB][CB + 1];
  if (*status) return;
  const int tid = threadIdx.x;
  const int nb = min(CB, n - k0);
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    D[i][j] = (i < nb && j < nb && j <= i) ? L[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6, half = lane >> 5, q = lane & 31;
  const int first = k0 + nb + blockIdx.x * TRSM_ROWS;
  for (int r = 0; r < TRSM_ROWS; r += 8) {
    const int i = first + r + wave * 2 + half;
    const bool live = i < n && q < nb;
    double x = live ? L[(int64_t)i * n + k0 + q] : 0.0;
    for (int p = 0; p < nb; ++p) {
      if (q == p) x /= D[p][p];
      const double xp = __shfl(x, (half << 5) + p, 64);
      if (q > p) x -= xp * D[q][p];
    }
    if (live) L[(int64_t)i * n + k0 + q] = x;
  }
}

__global__ __launch_bounds__(256) void chol_update(double* __restrict__ L, int n, int k0, const int* __restrict__ status) {
  if (*status) return;
  const int base = k0 + CB;
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (tj > ti) return;
  const int i0 = base + ti * 64, j0 = base + tj * 64;
  __shared__ double Ri[64][CB + 1], Rj[64][CB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * CB; e += 256) {
    const int r = e / CB, p = e % CB;
    Ri[r][p] = (i0 + r < n) ? L[(int64_t)(i0 + r) * n + k0 + p] : 0.0;
    Rj[r][p] = (j0 + r < n) ? L[(int64_t)(j0 + r) * n + k0 + p] : 0.0;
  }
  __syncthreads();
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4] = {};
#pragma unroll 4
  for (int p = 0; p < CB; ++p) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Ri[tr * 4 + u][p];
      b[u] = Rj[tc * 4 + u][p];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + tr * 4 + u, j = j0 + tc * 4 + v;
      if (i < n && j <= i) L[(int64_t)i * n + j] -= acc[u][v];
    }
}

__global__ void copy_lower_kernel(const double* __restrict__ A, double* __restrict__ L, int n, int zero_upper) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (zero_upper) {
      if (j > i) L[e] = 0.0;
    } else {
      L[e] = A[e];
    }
  }
}

// Grid points for the inspection hook: xyzw[4 g + 0..3] = (x, y, z, w) in the global frame.
__global__ void grid_points_kernel(GridDev G, const double* __restrict__ lines, double ax, double ay, double az,
                                   double* __restrict__ xyzw) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.npts) return;
  Geo geo;
  point_geo(G, lines, g, geo);
  xyzw[4 * g + 0] = ax + geo.d[0][0];
  xyzw[4 * g + 1] = ay + geo.d[0][1];
  xyzw[4 * g + 2] = az + geo.d[0][2];
  xyzw[4 * g + 3] = geo.w;
}

// One function at arbitrary points (inspection hook): what 0 chi, 1 -1/2 lap chi, 2 potential.
__global__ void eval_points_kernel(int what, ShellDev sh, MEntry me, double cx, double cy, double cz,
                                   const double* __restrict__ X, const double* __restrict__ Y,
                                   const double* __restrict__ Z, int64_t n, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dx = X[i] - cx, dy = Y[i] - cy, dz = Z[i] - cz;
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double ir = 1.0 / r;
  const double x = dx * ir, y = dy * ir, z = dz * ir;
  const int l = sh.l;
  double Cm2[LMAX + 1] = {}, Sm2[LMAX + 1] = {}, Cm1[LMAX + 1] = {}, Sm1[LMAX + 1] = {}, C[LMAX + 1] = {},
         Sv[LMAX + 1] = {};
  for (int ll = 0; ll <= l; ++ll) {
    if (ll == 0) {
      C[0] = 1.0;
      Sv[0] = 0.0;
    } else {
      const double tl = 2.0 * ll - 1.0;
#pragma unroll
      for (int m = 0; m <= LMAX; ++m) {
        double cn = 0.0, sn = 0.0;
        if (m == ll) {
          if (m >= 1) {
            cn = tl * (x * Cm1[m >= 1 ? m - 1 : 0] - y * Sm1[m >= 1 ? m - 1 : 0]);
            sn = tl * (y * Cm1[m >= 1 ? m - 1 : 0] + x * Sm1[m >= 1 ? m - 1 : 0]);
          }
        } else if (m == ll - 1) {
          cn = tl * z * Cm1[m];
          sn = tl * z * Sm1[m];
        } else if (m < ll - 1) {
          cn = (tl * z * Cm1[m] - (ll + m - 1.0) * Cm2[m]) / (double)(ll - m);
          sn = (tl * z * Sm1[m] - (ll + m - 1.0) * Sm2[m]) / (double)(ll - m);
        }
        C[m] = cn;
        Sv[m] = sn;
      }
    }
    if (ll < l) {
#pragma unroll
      for (int m = 0; m <= LMAX; ++m) {
        Cm2[m] = Cm1[m];
        Sm2[m] = Sm1[m];
        Cm1[m] = C[m];
        Sm1[m] = Sv[m];
      }
    }
  }
  const int am = me.m < 0 ? -me.m : me.m;
  double Yh = 0.0;
#pragma unroll
  for (int mm = 0; mm <= LMAX; ++mm)
    if (mm == am) Yh = me.m < 0 ? Sv[mm] : C[mm];
  Yh *= me.f;
  const double ex = exp(-sh.zeta * r);
  double v;
  if (what == 2) {
    const double xx = sh.zeta * r;
    double lower, upper;
    inc_gamma_pair(sh.n + l + 2, sh.n - l + 1, xx, ex, &lower, &upper);
    v = sh.pre * (ipow(1.0 / xx, l + 1) * lower + ipow(xx, l) * upper) * Yh;
  } else {
    const double rad = sh.norm * ipow(r, sh.n - 1) * ex;
    v = rad * Yh;
    if (what == 1)
      v *= -0.5 * (sh.zeta * sh.zeta - 2.0 * sh.zeta * sh.n * ir + (sh.n * (sh.n - 1.0) - l * (l + 1.0)) * ir * ir);
  }
  out[i] = v;
}

// ------------------------------------------------------------------------------------------------
// Launch wrappers (host).
// ------------------------------------------------------------------------------------------------
hipError_t launch_eval(bool fp32, const SegDev* segs, int nseg, int64_t nblocks, const GridDev* grids,
                       const double* lines, const ShellDev* shells, const MEntry* ments, const WColDev* wcols,
                       hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(eval_kernel<float>, dim3((unsigned)nblocks), dim3(256), 0, st, segs, nseg, grids, lines,
                       shells, ments, wcols);
  else
    hipLaunchKernelGGL(eval_kernel<double>, dim3((unsigned)nblocks), dim3(256), 0, st, segs, nseg, grids, lines,
                       shells, ments, wcols);
  return hipGetLastError();
}

hipError_t launch_eval_shared(bool fp32, const ShareSegDev* segs, int nseg, int64_t nblocks, const GridDev* grids,
                              const double* lines, const ShellDev* shells, const MEntry* ments, hipStream_t st) {
  if (nblocks <= 0 || nseg <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(eval_shared_kernel<float>, dim3((unsigned)nblocks), dim3(256), 0, st, segs, nseg, grids, lines,
                       shells, ments);
  else
    hipLaunchKernelGGL(eval_shared_kernel<double>, dim3((unsigned)nblocks), dim3(256), 0, st, segs, nseg, grids,
                       lines, shells, ments);
  return hipGetLastError();
}

template <typename T, int WM, int WN, int SC, int WR>
static hipError_t launch_contract_t(const TaskDev* tasks, const TileDev* tiles, int ntiles, double* ws,
                                    hipStream_t st) {
  constexpr int lds = ContractCfg<T, WM, WN, SC, WR>::LDS_BYTES;
  static_assert(lds <= 160 * 1024, "LDS budget");
  const void* fn = sizeof(T) == 8 ? (const void*)contract_f64<WM, WN, SC, WR>
                                  : (const void*)contract_mixed<WM, WN, SC, WR>;
  // once per instantiation (a function-local static is initialised once, also with concurrent callers)
  static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (attr != hipSuccess) return attr;
  if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL((contract_f64<WM, WN, SC, WR>), dim3(ntiles), dim3(256), lds, st, tasks, tiles, ws);
  else
    hipLaunchKernelGGL((contract_mixed<WM, WN, SC, WR>), dim3(ntiles), dim3(256), lds, st, tasks, tiles, ws);
  return hipGetLastError();
}

// Shapes built: (wm, wn, stage chunks) in the 2 x 2 wave arrangement, and the 4 x 1 arrangement with
// wm = 2 (128 rows) and odd wn (16 to 112 columns).
#define PS_SHAPES(X)                                                                            \
  X(4, 4, 1, 2) X(4, 4, 2, 2) X(2, 2, 1, 2) X(2, 2, 2, 2) X(4, 2, 1, 2) X(4, 2, 2, 2) X(2, 4, 1, 2) \
  X(2, 4, 2, 2) X(4, 1, 1, 2) X(4, 1, 2, 2) X(4, 3, 1, 2) X(4, 3, 2, 2) X(2, 1, 1, 2) X(2, 1, 2, 2) \
  X(2, 3, 1, 2) X(2, 3, 2, 2) X(1, 1, 1, 2) X(1, 1, 2, 2) X(1, 2, 1, 2) X(1, 2, 2, 2) X(1, 3, 1, 2) \
  X(1, 3, 2, 2) X(1, 4, 1, 2) X(1, 4, 2, 2) X(2, 1, 1, 4) X(2, 1, 2, 4) X(2, 3, 1, 4) X(2, 3, 2, 4) \
  X(2, 5, 1, 4) X(2, 5, 2, 4) X(2, 7, 1, 4) X(2, 7, 2, 4)

// A merged launch (wm == 0): LDS of its largest shape.
template <typename T, int SC, int I>
constexpr int merged_lds() {
  return ContractCfg<T, kMergedShapes[I][0], kMergedShapes[I][1], SC, kMergedShapes[I][2]>::LDS_BYTES;
}

template <typename T, int SC>
static hipError_t launch_merged_t(const TaskDev* tasks, const TileDev* tiles, int ntiles, double* ws,
                                  hipStream_t st) {
  constexpr int lds = std::max({merged_lds<T, SC, 0>(), merged_lds<T, SC, 1>(), merged_lds<T, SC, 2>(),
                                merged_lds<T, SC, 3>(), merged_lds<T, SC, 4>(), merged_lds<T, SC, 5>(),
                                merged_lds<T, SC, 6>(), merged_lds<T, SC, 7>()});
  static_assert(lds <= 160 * 1024, "LDS budget");
  const void* fn = sizeof(T) == 8 ? (const void*)contract_f64_merged<SC> : (const void*)contract_mixed_merged<SC>;
  static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (attr != hipSuccess) return attr;
  if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL((contract_f64_merged<SC>), dim3(ntiles), dim3(256), lds, st, tasks, tiles, ws);
  else
    hipLaunchKernelGGL((contract_mixed_merged<SC>), dim3(ntiles), dim3(256), lds, st, tasks, tiles, ws);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_contract_any(int wm, int wn, int sc, int wr, const TaskDev* tasks, const TileDev* tiles,
                                      int ntiles, double* ws, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (wm == 0) {
    if (sc == 1) return launch_merged_t<T, 1>(tasks, tiles, ntiles, ws, st);
    if (sc == 2) return launch_merged_t<T, 2>(tasks, tiles, ntiles, ws, st);
    return hipErrorInvalidValue;
  }
#define PS_SHAPE(a, b, c, d) \
  if (wm == a && wn == b && sc == c && wr == d) return launch_contract_t<T, a, b, c, d>(tasks, tiles, ntiles, ws, st);
  PS_SHAPES(PS_SHAPE)
#undef PS_SHAPE
  return hipErrorInvalidValue;
}

// Work-groups of one contraction shape resident on the current device at once (occupancy x CUs),
// 0 when the runtime cannot tell.
template <typename T, int WM, int WN, int SC, int WR>
static int resident_t() {
  constexpr int lds = ContractCfg<T, WM, WN, SC, WR>::LDS_BYTES;
  const void* fn = sizeof(T) == 8 ? (const void*)contract_f64<WM, WN, SC, WR>
                                  : (const void*)contract_mixed<WM, WN, SC, WR>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

int contract_resident_workgroups(bool mixed, int wm, int wn, int sc, int wr) {
#define PS_SHAPE(a, b, c, d)                        \
  if (wm == a && wn == b && sc == c && wr == d)     \
    return mixed ? resident_t<float, a, b, c, d>() : resident_t<double, a, b, c, d>();
  PS_SHAPES(PS_SHAPE)
#undef PS_SHAPE
  return 0;
}
#undef PS_SHAPES

hipError_t launch_contract_f64(int wm, int wn, int sc, int wr, const TaskDev* tasks, const TileDev* tiles,
                               int ntiles, double* ws, hipStream_t st) {
  return launch_contract_any<double>(wm, wn, sc, wr, tasks, tiles, ntiles, ws, st);
}

hipError_t launch_contract_mixed(int wm, int wn, int sc, int wr, const TaskDev* tasks, const TileDev* tiles,
                                 int ntiles, double* ws, hipStream_t st) {
  return launch_contract_any<float>(wm, wn, sc, wr, tasks, tiles, ntiles, ws, st);
}

hipError_t launch_reduce(const TaskDev* tasks, const RedDev* reds, const int32_t* items, int nitems,
                         const double* ws, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  // up to four work-groups per item while the launch has fewer than 1024 items
  const int spread = nitems >= 1024 ? 1 : std::min(4, (1023 + nitems) / nitems);
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)(nitems * spread)), dim3(256), 0, st, tasks, reds, items, ws,
                     spread);
  return hipGetLastError();
}

// blocks x 256 threads; out holds 4 doubles per block
hipError_t launch_mfma_rate(bool fp64, int blocks, int iters, double* out, hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL(mfma_rate_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, out, iters);
  else
    hipLaunchKernelGGL(mfma_rate_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, out, iters);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* X, int n, hipStream_t st) {
  if (n <= 1) return hipSuccess;
  int64_t blocks = ((int64_t)n * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, n);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* A, double* L, int n, int* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = ((int64_t)n * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(copy_lower_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, L, n, 0);
  for (int k0 = 0; k0 < n; k0 += CB) {
    hipLaunchKernelGGL(chol_panel, dim3(1), dim3(256), 0, st, A, L, n, k0, status);
    const int m = n - k0 - CB;
    if (m > 0) {
      hipLaunchKernelGGL(chol_trsm, dim3((m + TRSM_ROWS - 1) / TRSM_ROWS), dim3(256), 0, st, L, n, k0, status);
      const int t = (m + 63) / 64;
      hipLaunchKernelGGL(chol_update, dim3(t, t), dim3(256), 0, st, L, n, k0, status);
    }
  }
  hipLaunchKernelGGL(copy_lower_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, L, n, 1);
  return hipGetLastError();
}

hipError_t launch_grid_points(const GridDev& G, const double* lines, const double* RA, double* xyzw, hipStream_t st) {
  int64_t blocks = (G.npts + 255) / 256;
  hipLaunchKernelGGL(grid_points_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G, lines, RA[0], RA[1], RA[2],
                     xyzw);
  return hipGetLastError();
}

hipError_t launch_eval_points(int what, const ShellDev& sh, const MEntry& me, const double* c, const double* X,
                              const double* Y, const double* Z, int64_t n, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(eval_points_kernel, dim3((unsigned)blocks), dim3(256), 0, st, what, sh, me, c[0], c[1], c[2], X,
                     Y, Z, n, out);
  return hipGetLastError();
}

}  // namespace psint
