// Randomized check of the context arena allocator against a byte-map model:
// blocks never overlap, are granule-aligned, stay inside the range, and
// freeing everything restores one block of the full capacity.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

int main() {
  using grasp::Arena;
  const size_t cap = 1 << 20;
  std::vector<char> owner(cap, 0);
  static char base_storage[1 << 20];
  char* base = base_storage;
  Arena a;
  a.reset(base, cap + 100);  // a ragged size is cut to whole granules
  if (a.capacity() != cap) { std::printf("capacity %zu\n", a.capacity()); return 1; }
  std::mt19937 rng(7);
  struct Blk { char* p; size_t n; };
  std::vector<Blk> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t n = 1 + rng() % 20000;
      char* p = static_cast<char*>(a.alloc(n));
      if (!p) continue;
      const size_t off = p - base;
      if (off % grasp::kGranule || off + n > cap) { std::printf("bad block\n"); return 2; }
      for (size_t i = off; i < off + n; ++i) {
        if (owner[i]) { std::printf("overlap at %zu\n", i); return 3; }
        owner[i] = 1;
      }
      live.push_back({p, n});
    } else {
      const size_t k = rng() % live.size();
      const size_t off = live[k].p - base;
      for (size_t i = off; i < off + live[k].n; ++i) owner[i] = 0;
      a.free(live[k].p);
      live[k] = live.back();
      live.pop_back();
    }
  }
  a.free(nullptr);
  for (auto& b : live) a.free(b.p);
  if (a.used() != 0 || a.largest_free() != cap) { std::printf("leak: used %zu\n", a.used()); return 4; }
  if (!a.alloc(cap) || a.alloc(1)) { std::printf("full-size block\n"); return 5; }
  std::printf("arena ok\n");
  return 0;
}
