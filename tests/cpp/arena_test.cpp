// Randomised check of the device-arena allocator against a byte map: no two
// live allocations overlap, everything stays inside the arena, freed space is
// coalesced back into one range, and shrink keeps the head in place.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "../../paper_2201_13020_amd/csrc/szx_arena.hpp"

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                               \
    }                                                         \
  } while (0)

int main() {
  using szx::Arena;
  const uint64_t cap = 1 << 20;
  Arena a(cap);
  CHECK(a.capacity() == cap && a.free_ranges() == 1);
  CHECK(a.alloc(cap + 1) == Arena::kFail);
  // exact fill and drain
  uint64_t o = a.alloc(cap);
  CHECK(o == 0 && a.in_use() == cap && !a.fits(1));
  CHECK(a.release(o) && a.in_use() == 0 && a.free_ranges() == 1);
  CHECK(!a.release(o));
  // shrink keeps the head, frees the tail, coalesces with the next free range
  o = a.alloc(10000);
  const uint64_t o2 = a.alloc(100);
  CHECK(a.size_of(o) == Arena::round(10000));
  CHECK(a.shrink(o, 300) && a.size_of(o) == 512);
  CHECK(!a.shrink(o, 100000));
  // the freed tail lies between o and o2 and is reused first
  CHECK(o2 == Arena::round(10000) && a.alloc(9000) == 512);
  a.reset(cap);

  std::mt19937_64 rng(7);
  std::vector<int> owner(cap / Arena::kAlign, -1);
  struct Live { uint64_t off, n; int id; };
  std::vector<Live> live;
  int next_id = 0;
  for (int step = 0; step < 200000; ++step) {
    const int op = (int)(rng() % 10);
    if (op < 5 || live.empty()) {
      const uint64_t n = 1 + rng() % (op == 0 ? 200000 : 5000);
      const bool could = a.fits(n);
      const uint64_t off = a.alloc(n);
      CHECK((off != Arena::kFail) == could);
      if (off == Arena::kFail) continue;
      CHECK(off % Arena::kAlign == 0 && off + n <= cap);
      const uint64_t units = Arena::round(n) / Arena::kAlign;
      for (uint64_t u = 0; u < units; ++u) {
        CHECK(owner[off / Arena::kAlign + u] == -1);
        owner[off / Arena::kAlign + u] = next_id;
      }
      live.push_back({off, Arena::round(n), next_id++});
    } else if (op < 8) {
      const size_t k = rng() % live.size();
      Live l = live[k];
      for (uint64_t u = 0; u < l.n / Arena::kAlign; ++u) owner[l.off / Arena::kAlign + u] = -1;
      CHECK(a.release(l.off));
      live[k] = live.back();
      live.pop_back();
    } else {
      const size_t k = rng() % live.size();
      Live& l = live[k];
      const uint64_t keep = 1 + rng() % l.n;
      CHECK(a.shrink(l.off, keep));
      const uint64_t kept = Arena::round(keep);
      for (uint64_t u = kept / Arena::kAlign; u < l.n / Arena::kAlign; ++u) owner[l.off / Arena::kAlign + u] = -1;
      l.n = kept;
      CHECK(a.size_of(l.off) == kept);
    }
    uint64_t sum = 0;
    for (const Live& l : live) sum += l.n;
    CHECK(a.in_use() == sum && a.allocations() == live.size());
  }
  for (const Live& l : live) CHECK(a.release(l.off));
  CHECK(a.in_use() == 0 && a.free_ranges() == 1 && a.largest_free() == cap);
  CHECK(a.peak() > 0 && a.peak() <= cap);
  printf("arena ok\n");
  return 0;
}
