// Host check of the library's z-order helpers (csrc/zorder.h): the next key inside a
// box (znext) against a brute-force walk over the keys, for boxes of a 32 x 32 grid,
// and the bit gather (zcompact) as the inverse of the spread on random coordinates.
#include "../paper_2412_02448_amd/csrc/zorder.h"

#include <cstdio>
#include <random>

using namespace unify;

static bool inside(uint64_t z, uint64_t x0, uint64_t x1, uint64_t y0, uint64_t y1) {
  const uint64_t x = zcompact(z >> 1), y = zcompact(z);
  return x >= x0 && x <= x1 && y >= y0 && y <= y1;
}

int main() {
  const uint64_t N = 32;
  long checks = 0, bad = 0;
  for (uint64_t x0 = 0; x0 < N; ++x0)
    for (uint64_t x1 = x0; x1 < N; ++x1)
      for (uint64_t y0 = 0; y0 < N; y0 += 3)
        for (uint64_t y1 = y0; y1 < N; y1 += 2) {
          const uint64_t lo = zkey(x0, y0), hi = zkey(x1, y1);
          for (uint64_t z = lo; z <= hi; ++z) {
            if (inside(z, x0, x1, y0, y1)) continue;
            int64_t want = -1;
            for (uint64_t t = z + 1; t <= hi; ++t)
              if (inside(t, x0, x1, y0, y1)) {
                want = (int64_t)t;
                break;
              }
            ++checks;
            if (znext(z, lo, hi) != want) ++bad;
          }
        }
  std::mt19937_64 rng(7);
  for (int i = 0; i < 200000; ++i) {
    const uint64_t a = rng() & ZTOP, b = rng() & ZTOP;
    const uint64_t z = (uint64_t)zkey(a, b);
    ++checks;
    if (zcompact(z >> 1) != a || zcompact(z) != b) ++bad;
  }
  std::printf("checks %ld bad %ld\n", checks, bad);
  return bad != 0;
}
