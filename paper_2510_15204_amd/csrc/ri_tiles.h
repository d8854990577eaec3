// Order in which the work-groups of the RI product kernel take their output tiles (internal).
#pragma once
#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define RI_HD __host__ __device__
#else
#define RI_HD
#endif

namespace psint {

// The product's nt x nt grid of 128 x 128 tiles is symmetric: only tiles (i, j) with i <= j are
// computed.  Listed row by row they form T = nt (nt + 1) / 2 tiles; that list is cut into 8
// contiguous runs (run x starts at floor(T x / 8)) and the runs are interleaved, one tile of each
// run in turn, so that work-group t (which the hardware places on XCD t mod 8) takes the next tile
// of run t mod 8 while whole runs last: the tiles of one run share their row block in that XCD's L2.
// Position t of that order -> (i, j); O(1).
RI_HD inline void ri_syrk_tile(int64_t t, int64_t nt, int* ti, int* tj) {
  const int64_t T = nt * (nt + 1) / 2;
  const int64_t lmin = T / 8;
  int64_t r, x;
  if (t < 8 * lmin) {
    r = t / 8;
    x = t - 8 * r;
  } else {
    // the (t - 8 lmin)-th of the runs that are one tile longer, in run order
    r = lmin;
    int64_t k = t - 8 * lmin;
    for (x = 0; x < 7; ++x) {
      if (T * (x + 1) / 8 - T * x / 8 > lmin) {
        if (k == 0) break;
        --k;
      }
    }
  }
  int64_t idx = T * x / 8 + r;
  // row i of the upper triangle starts at i nt - i (i - 1) / 2
  const double b = 2.0 * (double)nt + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)idx)) / 2.0);
  if (i < 0) i = 0;
  while (i > 0 && i * nt - i * (i - 1) / 2 > idx) --i;
  while ((i + 1) * nt - (i + 1) * i / 2 <= idx) ++i;
  *ti = (int)i;
  *tj = (int)(i + idx - (i * nt - i * (i - 1) / 2));
}

}  // namespace psint
