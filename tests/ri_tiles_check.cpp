// Check of the RI product's tile order (ri_tiles.h): for every tile-grid size up to 600, position t
// of the closed-form order equals position t of the plainly built list (upper-triangle tiles row by
// row, cut into 8 contiguous runs, interleaved one tile per run in turn), so every tile on or above
// the diagonal is taken exactly once.  Prints "ok" and exits 0, else reports the first mismatch.
#include <cstdio>
#include <utility>
#include <vector>

#include "ri_tiles.h"

int main() {
  for (int nt = 1; nt <= 600; ++nt) {
    std::vector<std::pair<int, int>> rows;
    for (int i = 0; i < nt; ++i)
      for (int j = i; j < nt; ++j) rows.push_back({i, j});
    size_t beg[9];
    for (size_t x = 0; x <= 8; ++x) beg[x] = rows.size() * x / 8;
    std::vector<std::pair<int, int>> order;
    for (size_t r = 0; order.size() < rows.size(); ++r)
      for (size_t x = 0; x < 8; ++x)
        if (beg[x] + r < beg[x + 1]) order.push_back(rows[beg[x] + r]);
    for (size_t t = 0; t < order.size(); ++t) {
      int i = -1, j = -1;
      psint::ri_syrk_tile((int64_t)t, nt, &i, &j);
      if (i != order[t].first || j != order[t].second) {
        std::printf("nt=%d t=%zu: (%d,%d) instead of (%d,%d)\n", nt, t, i, j, order[t].first, order[t].second);
        return 1;
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
