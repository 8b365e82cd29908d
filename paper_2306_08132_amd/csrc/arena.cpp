// First-fit sub-allocator of the context arena (see arena.h).
#include "arena.h"

#include <algorithm>

namespace grasp {

namespace {
size_t round_up_granule(size_t x) { return (x + kGranule - 1) / kGranule * kGranule; }
}  // namespace

void Arena::reset(char* base, size_t bytes) {
  base_ = base;
  bytes_ = bytes / kGranule * kGranule;
  free_.clear();
  used_.clear();
  if (bytes_) free_[0] = bytes_;
}

void* Arena::alloc(size_t bytes) {
  const size_t need = round_up_granule(std::max<size_t>(bytes, 1));
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, sz = it->second;
    free_.erase(it);
    if (sz > need) free_[off + need] = sz - need;
    used_[off] = need;
    return base_ + off;
  }
  return nullptr;
}

void Arena::free(void* p) {
  if (!p) return;
  const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, sz = u->second;
  used_.erase(u);
  auto nx = free_.lower_bound(start);
  if (nx != free_.end() && nx->first == start + sz) {
    sz += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(start);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == start) {
      start = pv->first;
      sz += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = sz;
}

size_t Arena::used() const {
  size_t s = 0;
  for (auto& kv : used_) s += kv.second;
  return s;
}

size_t Arena::largest_free() const {
  size_t s = 0;
  for (auto& kv : free_) s = std::max(s, kv.second);
  return s;
}

}  // namespace grasp
