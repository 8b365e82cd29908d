// First-fit sub-allocator over one device address range. Pure host code
// (no HIP): it only does arithmetic on addresses, so it is tested on the CPU.
#pragma once

#include <cstddef>
#include <map>

namespace grasp {

constexpr size_t kGranule = 256;  // allocation granule and alignment (bytes)

// First-fit allocator with coalescing free blocks; 256-byte granules.
class Arena {
 public:
  void reset(char* base, size_t bytes);
  void* alloc(size_t bytes);   // nullptr when no block fits
  void free(void* p);
  size_t capacity() const { return bytes_; }
  size_t used() const;
  size_t largest_free() const;

 private:
  char* base_ = nullptr;
  size_t bytes_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> used_;   // offset -> size
};

}  // namespace grasp
