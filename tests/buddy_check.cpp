// Host check of the server arena's buddy allocator: random allocations and
// releases against a model of the live blocks (no overlap, inside the
// arena, aligned to the block size), exact capacity cases, and a complete
// merge once everything is released.  Exit status 0 when every check holds.
#include <cstdio>
#include <iterator>
#include <map>
#include <random>

#include "gx_buddy.hpp"

static int fail(const char* what) {
  std::printf("FAIL %s\n", what);
  return 1;
}

int main() {
  using gx::Buddy;
  const uint64_t MiB = uint64_t(1) << 20, GiB = uint64_t(1) << 30;
  {  // 400 MiB: top blocks of 256, 128 and 16 MiB
    Buddy b;
    b.init(400 * MiB);
    if (b.largest() != 256 * MiB) return fail("largest of 400 MiB");
    if (b.alloc(256 * MiB) != 0) return fail("first 256 MiB block");
    if (b.alloc(256 * MiB) != ~0ull) return fail("second 256 MiB block must not fit");
    if (b.alloc(128 * MiB) != 256 * MiB) return fail("128 MiB block");
    if (b.alloc(16 * MiB) != 384 * MiB) return fail("16 MiB block");
    if (b.alloc(4096) != ~0ull) return fail("arena full");
    b.release(256 * MiB, 128 * MiB);
    if (b.alloc(64 * MiB) != 256 * MiB) return fail("reuse after release");
  }
  std::mt19937_64 rng(7);
  for (uint64_t size : {400 * MiB, 200 * GiB, MiB, uint64_t(5000) * 4096 + 123}) {
    Buddy b;
    b.init(size);
    std::map<uint64_t, uint64_t> live;  // offset -> bytes asked
    for (int it = 0; it < 100000; ++it) {
      if (!live.empty() && (rng() & 1)) {
        auto x = live.begin();
        std::advance(x, rng() % live.size());
        b.release(x->first, x->second);
        live.erase(x);
        continue;
      }
      const uint64_t n = 1 + rng() % (uint64_t(1) << (rng() % 31));
      const uint64_t off = b.alloc(n);
      if (off == ~0ull) continue;
      const uint64_t bb = Buddy::block_bytes(n);
      if (bb < n || off % bb != 0) return fail("block size or alignment");
      if (off + bb > size) return fail("block outside the arena");
      auto nx = live.lower_bound(off);
      if (nx != live.end() && nx->first < off + bb) return fail("overlaps the next block");
      if (nx != live.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + Buddy::block_bytes(pv->second) > off) return fail("overlaps the previous block");
      }
      live[off] = n;
    }
    for (const auto& kv : live) b.release(kv.first, kv.second);
    if (b.alloc(b.largest()) != 0) return fail("blocks did not merge back");
  }
  std::printf("ok\n");
  return 0;
}
