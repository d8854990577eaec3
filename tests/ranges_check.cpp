// Randomised check of the device pool's free-range bookkeeping (RangeMap) against a plain model:
// taken ranges are disjoint and inside the chunk, taken + free ranges tile the chunk exactly, free
// ranges are coalesced, take() returns the lowest free range that fits, and giving everything back
// leaves one free range.  Prints "ok" and exits 0, else reports the first violation and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "ranges.h"

using psint::RangeMap;

static int fail(const char* what, int step) {
  std::printf("violation at step %d: %s\n", step, what);
  return 1;
}

static bool tiles(const RangeMap& r, const std::map<size_t, size_t>& taken) {
  std::map<size_t, size_t> all(taken.begin(), taken.end());
  for (auto& f : r.free_ranges()) {
    if (all.count(f.first)) return false;
    all[f.first] = f.second;
  }
  size_t pos = 0;
  for (auto& a : all) {
    if (a.first != pos || a.second == 0) return false;
    pos += a.second;
  }
  return pos == r.size();
}

static bool coalesced(const RangeMap& r) {
  size_t end = (size_t)-1;
  for (auto& f : r.free_ranges()) {
    if (f.first == end) return false;
    end = f.first + f.second;
  }
  return true;
}

int main() {
  std::mt19937_64 rng(15204);
  for (int trial = 0; trial < 200; ++trial) {
    const size_t size = 64 + rng() % 4096;
    RangeMap r(size);
    std::map<size_t, size_t> taken;  // offset -> length
    for (int step = 0; step < 400; ++step) {
      if (taken.empty() || rng() % 3) {
        const size_t want = 1 + rng() % (size / 4 + 1);
        size_t expect = (size_t)-1;
        for (auto& f : r.free_ranges())
          if (f.second >= want) {
            expect = f.first;
            break;
          }
        size_t off = 0;
        const bool ok = r.take(want, &off);
        if (ok != (expect != (size_t)-1)) return fail("take result differs from first fit", step);
        if (ok) {
          if (off != expect) return fail("not the lowest fitting range", step);
          if (off + want > size) return fail("range outside the chunk", step);
          taken[off] = want;
        }
      } else {
        auto it = taken.begin();
        std::advance(it, rng() % taken.size());
        r.give(it->first, it->second);
        taken.erase(it);
      }
      if (!tiles(r, taken)) return fail("taken and free ranges do not tile the chunk", step);
      if (!coalesced(r)) return fail("adjacent free ranges not merged", step);
    }
    for (auto& t : taken) r.give(t.first, t.second);
    if (!r.unused()) return fail("not one free range after giving everything back", -1);
  }
  std::printf("ok\n");
  return 0;
}
