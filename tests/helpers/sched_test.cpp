// Test-only driver for the serving scheduler's host logic (no GPU): the
// device-arena allocator, FIFO admission by slot and memory, the event-chunk
// rule, the choice of lane and the length of a chain. Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "vegas_sched.hpp"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

using vegas::Admission;
using vegas::Arena;

static void arena_basic() {
  Arena a(4096, 256);
  const size_t x = a.alloc(100), y = a.alloc(256), z = a.alloc(1000);
  CHECK(x == 0 && y == 256 && z == 512);
  CHECK(a.used() == 256 + 256 + 1024);
  CHECK(a.alloc(4096) == SIZE_MAX);
  CHECK(a.release(y));
  CHECK(!a.release(y));
  CHECK(a.alloc(200) == 256);  // first fit reuses the hole
  CHECK(a.release(x) && a.release(256) && a.release(z));
  CHECK(a.used() == 0 && a.largest_free() == 4096 && a.live_ranges() == 0);
  CHECK(a.alloc(0) == SIZE_MAX);
}

static void arena_random() {
  // random alloc/free never overlaps ranges and coalesces back to one block
  std::mt19937 rng(7);
  Arena a(1 << 20, 256);
  std::vector<std::pair<size_t, size_t>> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || (rng() % 3 != 0 && live.size() < 200)) {
      const size_t n = 1 + rng() % 20000;
      const size_t off = a.alloc(n);
      if (off == SIZE_MAX) continue;
      const size_t len = (n + 255) / 256 * 256;
      CHECK(off % 256 == 0 && off + len <= a.size());
      for (auto& r : live) CHECK(off + len <= r.first || r.first + r.second <= off);
      live.emplace_back(off, len);
    } else {
      const size_t i = rng() % live.size();
      CHECK(a.release(live[i].first));
      live.erase(live.begin() + (long)i);
    }
  }
  for (auto& r : live) CHECK(a.release(r.first));
  CHECK(a.used() == 0 && a.largest_free() == a.size());
}

static void admission() {
  Arena a(10000, 1);
  Admission<int> adm(2, &a);
  for (int i = 0; i < 5; ++i) adm.push(i);
  auto bytes = [](int r) { return (size_t)(r == 1 ? 8000 : 1000); };
  auto got = adm.admit(bytes);
  // slots for two; request 1 (8000 bytes) fits next to request 0
  CHECK(got.size() == 2 && std::get<0>(got[0]) == 0 && std::get<0>(got[1]) == 1);
  CHECK(adm.free_slots() == 0 && adm.pending() == 3);
  CHECK(adm.admit(bytes).empty());
  adm.finish(std::get<1>(got[0]), std::get<2>(got[0]));
  auto got2 = adm.admit(bytes);
  CHECK(got2.size() == 1 && std::get<0>(got2[0]) == 2);
  // memory-bound: free the slot but keep the memory busy with a large head
  Arena b(5000, 1);
  Admission<int> adm2(8, &b);
  adm2.push(10);
  adm2.push(11);
  adm2.push(12);
  auto big = [](int r) { return (size_t)(r == 11 ? 4500 : 1000); };
  auto g = adm2.admit(big);
  CHECK(g.size() == 1 && std::get<0>(g[0]) == 10);  // 11 does not fit, 12 waits behind it (FIFO)
  adm2.finish(std::get<1>(g[0]), std::get<2>(g[0]));
  g = adm2.admit(big);
  CHECK(g.size() == 1 && std::get<0>(g[0]) == 11);
}

static void chunks() {
  CHECK(vegas::chunk_events(10000, 0) == 256);
  CHECK(vegas::chunk_events(300000, 0) == 768);
  CHECK(vegas::chunk_events(10000000, 0) == 19712);
  CHECK(vegas::chunk_events(100000000000LL, 0) == 262144);
  CHECK(vegas::chunk_events(123, 777) == 777);
  for (long long n : {2LL, 4097LL, 1000003LL, 123456789LL}) {
    const long long c = vegas::chunk_events(n, 0);
    CHECK(c % 256 == 0 && c >= 256 && c <= 262144);
  }
}

static void lanes() {
  bool busy[4] = {true, false, false, true};
  size_t members[4] = {3, 2, 0, 0};
  CHECK(vegas::pick_lane(4, busy, members) == 2);  // idle and empty
  members[2] = 1;
  CHECK(vegas::pick_lane(4, busy, members) == 3);  // none free: fewest integrals
  busy[3] = false;
  CHECK(vegas::pick_lane(4, busy, members) == 3);  // idle and empty again
  bool all_busy[2] = {true, true};
  size_t eq[2] = {1, 1};
  CHECK(vegas::pick_lane(2, all_busy, eq) == 0);   // the first of equals
  CHECK(vegas::pick_lane(1, all_busy, eq) == 0);
}

static void chains() {
  const int rem[3] = {7, 5, 9};
  const int64_t ev[3] = {1000, 2000, 3000};
  CHECK(vegas::chain_ticks(3, rem, ev, 32, 1LL << 40) == 5);   // the first completion
  CHECK(vegas::chain_ticks(3, rem, ev, 3, 1LL << 40) == 3);    // the tick bound
  CHECK(vegas::chain_ticks(3, rem, ev, 32, 13000) == 2);       // 6000 events per tick
  CHECK(vegas::chain_ticks(3, rem, ev, 32, 100) == 1);         // one tick even if larger
  const int one[1] = {1};
  CHECK(vegas::chain_ticks(1, one, ev, 32, 1LL << 40) == 1);
}

int main() {
  arena_basic();
  arena_random();
  admission();
  chunks();
  lanes();
  chains();
  std::printf("ok\n");
  return 0;
}
