// CPU test of the server's range allocator (header only, no HIP).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2104_05426_amd/csrc/jefi_arena.h"

#define CHECK(c)                                             \
  do {                                                       \
    if (!(c)) {                                              \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
      return 1;                                              \
    }                                                        \
  } while (0)

int main() {
  using jefi::Arena;
  Arena a(4096);
  uint64_t o1, o2, o3, o4;
  CHECK(a.alloc(100, &o1) && o1 == 0);          // one granule
  CHECK(a.alloc(256, &o2) && o2 == 256);
  CHECK(a.alloc(1000, &o3) && o3 == 512);       // four granules
  CHECK(a.used() == 256 * 6);
  CHECK(!a.alloc(4096, &o4));                   // too big: nothing changes
  CHECK(a.used() == 256 * 6);
  a.release(o2, 256);                           // hole between o1 and o3
  CHECK(a.free_blocks() == 2);
  CHECK(a.alloc(200, &o4) && o4 == 256);        // first fit reuses the hole
  a.release(o1, 100);
  a.release(o4, 200);
  a.release(o3, 1000);
  CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == 4096);  // fully coalesced
  CHECK(a.high_water() == 256 * 6);
  // random alloc/free against a byte map: no overlap, exact accounting
  std::mt19937 rng(7);
  Arena b(1 << 20);
  std::vector<unsigned char> owner(1 << 20, 0);
  struct Blk { uint64_t off, bytes; };
  std::vector<Blk> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3) {
      const uint64_t bytes = 1 + rng() % 20000;
      uint64_t off;
      if (b.alloc(bytes, &off)) {
        const uint64_t len = Arena::round_up(bytes);
        CHECK(off % Arena::kGranule == 0 && off + len <= (1u << 20));
        for (uint64_t i = off; i < off + len; ++i) {
          CHECK(owner[i] == 0);
          owner[i] = 1;
        }
        live.push_back({off, bytes});
      } else {
        CHECK(!b.fits(bytes));
      }
    } else {
      const size_t k = rng() % live.size();
      const Blk blk = live[k];
      live.erase(live.begin() + k);
      for (uint64_t i = blk.off; i < blk.off + Arena::round_up(blk.bytes); ++i) owner[i] = 0;
      b.release(blk.off, blk.bytes);
    }
    uint64_t used = 0;
    for (auto& x : live) used += Arena::round_up(x.bytes);
    CHECK(b.used() == used);
  }
  for (auto& x : live) b.release(x.off, x.bytes);
  CHECK(b.used() == 0 && b.free_blocks() == 1);
  std::printf("arena ok\n");
  return 0;
}
