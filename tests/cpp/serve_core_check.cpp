// Host-only checks of the serving arena allocator and batch former (no GPU).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>

#include "../../paper_2504_19163_amd/csrc/serve_core.hpp"

using namespace bbc;

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);     \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static void arena_basic() {
  Arena a(1 << 20);
  CHECK(a.capacity() == (1u << 20));
  const size_t x = a.alloc(1000), y = a.alloc(3000), z = a.alloc(256);
  CHECK(x == 0 && y == 1024 && z == 1024 + 3072);
  CHECK(a.used() == 1024 + 3072 + 256);
  a.release(y, 3000);
  CHECK(a.n_free_ranges() == 2);
  const size_t w = a.alloc(2000);  // first fit reuses the hole
  CHECK(w == 1024);
  a.release(x, 1000);
  a.release(w, 2000);
  a.release(z, 256);
  CHECK(a.used() == 0 && a.n_free_ranges() == 1 && a.largest_free() == (1u << 20));
  CHECK(a.alloc(size_t(2) << 20) == SIZE_MAX);
  CHECK(!a.ever_fits((size_t(1) << 20) + 1) && a.ever_fits(size_t(1) << 20));
  CHECK(a.peak() == 1024 + 3072 + 256);
}

// random alloc/free against a brute-force occupancy map
static void arena_random() {
  const size_t cap = 256 * 512;
  Arena a(cap);
  std::mt19937 rng(7);
  std::vector<std::pair<size_t, size_t>> live;
  std::vector<char> occ(cap / 256, 0);
  for (int it = 0; it < 20000; ++it) {
    if (!live.empty() && (rng() % 2 == 0)) {
      const size_t k = rng() % live.size();
      const auto [off, b] = live[k];
      for (size_t g = off / 256; g < (off + Arena::round(b)) / 256; ++g) occ[g] = 0;
      a.release(off, b);
      live.erase(live.begin() + k);
    } else {
      const size_t b = 1 + rng() % 9000;
      const size_t off = a.alloc(b);
      // first fit: the result is the lowest run of free granules that is long enough
      const size_t need = Arena::round(b) / 256;
      size_t want = SIZE_MAX, run = 0;
      for (size_t g = 0; g < occ.size(); ++g) {
        run = occ[g] ? 0 : run + 1;
        if (run == need) {
          want = (g + 1 - need) * 256;
          break;
        }
      }
      CHECK(off == want);
      if (off == SIZE_MAX) continue;
      for (size_t g = off / 256; g < off / 256 + need; ++g) {
        CHECK(!occ[g]);
        occ[g] = 1;
      }
      live.push_back({off, b});
    }
    size_t used = 0;
    for (char c : occ) used += c ? 256 : 0;
    CHECK(a.used() == used);
  }
}

static void former() {
  auto need = [](int32_t, int64_t p, int32_t r) { return size_t(p) * 100 + size_t(r) * 10; };
  std::vector<PendingView> q = {{0, 10}, {1, 5}, {0, 20}, {0, 50}, {1, 1}, {0, 5}};
  // everything of scene 0 that fits 40 points: 10 + 20, skip 50, then 5
  auto pick = form_batch(q, 40, 100, need, [](size_t) { return true; });
  CHECK((pick == std::vector<size_t>{0, 2, 5}));
  // request cap
  pick = form_batch(q, 1000, 2, need, [](size_t) { return true; });
  CHECK((pick == std::vector<size_t>{0, 2}));
  // budget: at most 3500 bytes -> 10 + 20 (3020 bytes), 50 does not fit, 5 fits (3530 > 3500: no)
  pick = form_batch(q, 1000, 100, need, [](size_t b) { return b <= 3500; });
  CHECK((pick == std::vector<size_t>{0, 2}));
  // the oldest request does not fit now: nothing is taken (no overtaking)
  pick = form_batch(q, 1000, 100, need, [](size_t b) { return b <= 500; });
  CHECK(pick.empty());
  // oldest request alone exceeds the batch size
  pick = form_batch(q, 8, 100, need, [](size_t) { return true; });
  CHECK(pick.empty());
  // other scene first in line
  std::vector<PendingView> q2 = {{1, 5}, {0, 3}, {1, 7}};
  pick = form_batch(q2, 100, 100, need, [](size_t) { return true; });
  CHECK((pick == std::vector<size_t>{0, 2}));
  CHECK(form_batch({}, 10, 10, need, [](size_t) { return true; }).empty());
}

static void pct() {
  CHECK(percentile({}, 50) == 0.0);
  CHECK(percentile({3.0}, 99) == 3.0);
  CHECK(percentile({4, 1, 3, 2, 5}, 50) == 3.0);
  CHECK(std::abs(percentile({1, 2, 3, 4, 5, 6, 7, 8, 9, 10}, 99) - 9.91) < 1e-12);
}

int main() {
  arena_basic();
  arena_random();
  former();
  pct();
  if (fails) return 1;
  std::printf("serve_core ok\n");
  return 0;
}
