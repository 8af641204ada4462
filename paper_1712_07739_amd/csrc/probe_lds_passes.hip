// Measurement behind pass_target (internal.h): which lanes of a wave share a
// pass of a 16-byte LDS read (ds_read_b128) on gfx950, and how many bank
// groups there are.  Not part of libdfmm; built and run on its own under
// rocprofv3 with SQ_LDS_BANK_CONFLICT counted per dispatch.
//
// One wave per dispatch; lane l reads 16-byte unit pat[l] of a 1024-unit LDS
// array `kIters` times (every unit index is checked to lie in [0, 1024)).
//   dispatches 0..3: unit = s * l for s = 1, 2, 8, 16 (bank groups)
//   dispatches 4..: every lane reads unit 1 (one address: a broadcast), the
//     reference lane r reads unit 0 and lane b unit 16 (both in bank group 0
//     if there are 16 groups): a conflict iff r and b share a pass; for r in
//     {0, 4, 32, 36}, b = 0..63 (b = r: no moved lane).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

constexpr int kIters = 1000;

__global__ void __launch_bounds__(64) probe(const int* __restrict__ pat, int iters, unsigned* out) {
  __shared__ uint4 lds[1024];
  for (int i = threadIdx.x; i < 1024; i += 64) lds[i] = make_uint4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  int u = pat[threadIdx.x];
  unsigned acc = 0;
  for (int it = 0; it < iters; ++it) {
    asm volatile("" : "+v"(u));  // one read per iteration
    const uint4 v = lds[u];
    acc += v.x ^ v.y ^ v.z ^ v.w;
  }
  out[threadIdx.x] = acc;
}

#define CHECK(x)                                                  \
  do {                                                            \
    hipError_t e_ = (x);                                          \
    if (e_ != hipSuccess) {                                       \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main() {
  std::vector<std::vector<int>> pats;
  std::vector<int> p(64);
  for (int s : {1, 2, 8, 16}) {
    for (int l = 0; l < 64; ++l) p[l] = s * l;
    pats.push_back(p);
  }
  for (int r : {0, 4, 32, 36})
    for (int b = 0; b < 64; ++b) {
      for (int l = 0; l < 64; ++l) p[l] = 1;
      p[r] = 0;
      if (b != r) p[b] = 16;
      pats.push_back(p);
    }
  int* dp = nullptr;
  unsigned* dout = nullptr;
  CHECK(hipMalloc(&dp, 64 * sizeof(int)));
  CHECK(hipMalloc(&dout, 64 * sizeof(unsigned)));
  for (size_t k = 0; k < pats.size(); ++k) {
    for (int l = 0; l < 64; ++l)
      if (pats[k][l] < 0 || pats[k][l] >= 1024) {
        std::printf("pattern %zu out of range\n", k);
        return 1;
      }
    CHECK(hipMemcpy(dp, pats[k].data(), 64 * sizeof(int), hipMemcpyHostToDevice));
    probe<<<1, 64>>>(dp, kIters, dout);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
  }
  std::printf("%zu probe dispatches\n", pats.size());
  return 0;
}
