// Host test of the arena's first-fit bookkeeping (paper_2510_09813_amd/csrc/first_fit.h),
// built by tests/test_first_fit_sanitizers.py with the address and undefined-behaviour
// sanitizers and, separately, the thread sanitizer.
//  1. random take/give sequences against a byte map: no two live blocks overlap, every gap
//     is merged with its neighbours, gaps + used == size, first fit takes the lowest gap;
//  2. eight threads taking and giving blocks through one mutex, as the server's lanes do.
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "first_fit.h"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

struct Live {
  size_t off, len;
};

static void check_invariants(const rsv::FirstFit& ff, const std::vector<Live>& live) {
  std::vector<int> map(ff.size(), 0);
  for (const Live& b : live)
    for (size_t i = b.off; i < b.off + b.len; ++i) {
      CHECK(i < ff.size());
      CHECK(map[i] == 0);
      map[i] = 1;
    }
  size_t free_bytes = 0, prev_end = 0;
  bool first = true;
  for (const auto& g : ff.gaps()) {
    CHECK(g.second > 0);
    CHECK(first || g.first > prev_end);  // sorted and never adjacent (merged)
    for (size_t i = g.first; i < g.first + g.second; ++i) {
      CHECK(map[i] == 0);
      map[i] = 2;
    }
    free_bytes += g.second;
    prev_end = g.first + g.second;
    first = false;
  }
  size_t used = 0;
  for (const Live& b : live) used += b.len;
  CHECK(used == ff.used());
  CHECK(used + free_bytes == ff.size());
  for (int v : map) CHECK(v != 0);  // every byte is live or free
}

static void sequential() {
  std::mt19937_64 rng(12345);
  rsv::FirstFit ff;
  const size_t size = 4096;
  ff.reset(size);
  std::vector<Live> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t len = 1 + rng() % 200;
      size_t off = 0;
      // first fit: the lowest gap that holds len
      size_t want = size;
      for (const auto& g : ff.gaps())
        if (g.second >= len) {
          want = g.first;
          break;
        }
      if (ff.take(len, &off)) {
        CHECK(off == want);
        live.push_back({off, len});
      } else {
        CHECK(want == size);
      }
    } else {
      const size_t i = rng() % live.size();
      ff.give(live[i].off, live[i].len);
      live.erase(live.begin() + i);
    }
    if (step % 97 == 0) check_invariants(ff, live);
  }
  for (const Live& b : live) ff.give(b.off, b.len);
  CHECK(ff.used() == 0 && ff.gaps().size() == 1 && ff.gaps().begin()->second == size);
}

static void threaded() {
  rsv::FirstFit ff;
  std::mutex mu;
  ff.reset(1 << 20);
  std::vector<std::thread> th;
  for (int t = 0; t < 8; ++t)
    th.emplace_back([&, t] {
      std::mt19937_64 rng(t + 1);
      std::vector<Live> mine;
      for (int i = 0; i < 5000; ++i) {
        if (mine.empty() || rng() % 2) {
          const size_t len = 256 * (1 + rng() % 16);
          size_t off = 0;
          std::lock_guard<std::mutex> lk(mu);
          if (ff.take(len, &off)) mine.push_back({off, len});
        } else {
          const Live b = mine.back();
          mine.pop_back();
          std::lock_guard<std::mutex> lk(mu);
          ff.give(b.off, b.len);
        }
      }
      std::lock_guard<std::mutex> lk(mu);
      for (const Live& b : mine) ff.give(b.off, b.len);
    });
  for (auto& t : th) t.join();
  CHECK(ff.used() == 0 && ff.gaps().size() == 1);
}

int main() {
  sequential();
  threaded();
  std::puts("first_fit ok");
  return 0;
}
