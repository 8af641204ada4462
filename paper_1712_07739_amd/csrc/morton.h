// 3D Morton keys of cells (10 bits per axis) and binary search in a level's
// ascending keys, shared by the tree builders.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dfmm {

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000FF;
  v = (v | (v << 8)) & 0x0300F00F;
  v = (v | (v << 4)) & 0x030C30C3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249;
  v = (v | (v >> 2)) & 0x030C30C3;
  v = (v | (v >> 4)) & 0x0300F00F;
  v = (v | (v >> 8)) & 0x030000FF;
  v = (v | (v >> 16)) & 0x3ff;
  return v;
}
// key bit 3b+2 = x_b, 3b+1 = y_b, 3b = z_b
__device__ __forceinline__ uint32_t morton(int x, int y, int z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
__device__ __forceinline__ void demorton(uint32_t k, int& x, int& y, int& z) {
  x = compact3(k >> 2);
  y = compact3(k >> 1);
  z = compact3(k);
}
__device__ __forceinline__ int bsearch_key(const uint32_t* keys, int n, uint32_t k) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    uint32_t v = keys[mid];
    if (v == k) return mid;
    if (v < k) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

}  // namespace dfmm
