// Measurement behind the VALU rooflines: the issue rate of the three
// multiply-add forms the M2L products use (v_fmac_f32, v_dot2_f32_f16,
// v_fma_f64), from eight independent register-only chains per thread at
// eight waves per SIMD (2048 blocks of 256 threads).  Not part of libdfmm;
// built and run on its own.  Prints, per form, the time of five launches,
// the multiply-add rate in TFLOP/s and wave64 instructions per SIMD per ns.
#include <hip/hip_runtime.h>

#include <cstdio>
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
constexpr int K = 8;
__global__ void __launch_bounds__(256) f32fma(const float* in, int iters, float* out) {
  float a[K];
  const float b = in[0], c = in[1];
  for (int k = 0; k < K; ++k) a[k] = in[2 + k] + threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = fmaf(a[k], b, c);
  }
  float s = 0; for (int k = 0; k < K; ++k) s += a[k];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) f16dot(const float* in, int iters, float* out) {
  float a[K];
  h2 x; x[0] = (_Float16)in[0]; x[1] = (_Float16)in[1];
  h2 y; y[0] = (_Float16)in[2]; y[1] = (_Float16)in[3];
  for (int k = 0; k < K; ++k) a[k] = in[2 + k] + threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = __builtin_amdgcn_fdot2(x, y, a[k], false);
  }
  float s = 0; for (int k = 0; k < K; ++k) s += a[k];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) f64fma(const float* in, int iters, float* out) {
  double a[K];
  const double b = in[0], c = in[1];
  for (int k = 0; k < K; ++k) a[k] = in[2 + k] + threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = fma(a[k], b, c);
  }
  double s = 0; for (int k = 0; k < K; ++k) s += a[k];
  out[blockIdx.x * 256 + threadIdx.x] = (float)s;
}
int main() {
  const int blocks = 2048, iters = 16384;
  float *in, *out;
  if (hipMalloc(&in, 64 * sizeof(float)) != hipSuccess) return 1;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
  float h[64];
  for (int i = 0; i < 64; ++i) h[i] = 0.999f - 0.001f * i;
  if (hipMemcpy(in, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const char* names[3] = {"f32 fma", "f16 dot2 (2 fma)", "f64 fma"};
  for (int v = 0; v < 3; ++v) {
    for (int rep = 0; rep < 2; ++rep) {
      if (hipEventRecord(e0) != hipSuccess) return 1;
      for (int r = 0; r < 5; ++r) {
        if (v == 0) f32fma<<<blocks, 256>>>(in, iters, out);
        if (v == 1) f16dot<<<blocks, 256>>>(in, iters, out);
        if (v == 2) f64fma<<<blocks, 256>>>(in, iters, out);
      }
      if (hipEventRecord(e1) != hipSuccess) return 1;
      if (hipEventSynchronize(e1) != hipSuccess) return 1;
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
      const double insts = 5.0 * blocks * 4.0 * iters * K;  // wave64 instructions (4 waves per block)
      const double lanes_ops = insts * 64.0;
      const double flop = lanes_ops * (v == 1 ? 4.0 : 2.0);
      printf("%-18s %8.3f ms  %7.1f TFLOP/s  wave-instr per SIMD per ns %.3f\n", names[v], ms, flop / (ms * 1e-3) / 1e12,
             insts / 1024.0 / (ms * 1e6));
    }
  }
  return 0;
}
