// Device-side evaluation of the anisotropic-kernel surrogate network on the
// matrix cores, and its use in place of the unit-circle quadrature (see
// mlp.hip for training and the residual gate).
//
// Network: 6 inputs (unit direction T, normalised c11, c12, c44) -> four
// hidden layers of 128 (SiLU) -> 18 outputs.  Inference runs one wave at a
// time on 32 rows per pass with v_mfma_f32_32x32x16_f16: f16 weights and
// activations, f32 accumulation, bias and SiLU in f32.  The product is
// formed transposed, H_out^T = W H_in^T, so the batch rows are the MFMA's
// N dimension: lane l then holds, for row l % 32, the output features
// m = 32 t + 8 (r / 4) + 4 (l / 32) + r % 4 of tile t in accumulator r.
// Those registers, rounded to f16, are directly the next layer's B operand
// when the next layer's weights list their input features in that order
// (sur_in_feature below), so activations never leave registers.
// Weights are stored in fragment order: for layer L, out tile t, K step c
// and lane l, the eight f16 values lane l feeds the MFMA, so a wave reads
// 1 KB contiguous per MFMA (no LDS bank conflicts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernel_eval.h"

namespace dfmm {

constexpr int kSurLayers = 5;   // 4 hidden layers + output layer
constexpr int kSurHidden = 128;
constexpr int kSurOut = 18;
// distinct (v, p) pairs of the symmetric index pair of d_q G_vp
__device__ __host__ constexpr int sur_pair_v(int k) { return k < 3 ? k : (k == 3 ? 1 : 0); }
__device__ __host__ constexpr int sur_pair_p(int k) { return k < 3 ? k : (k == 5 ? 1 : 2); }

// f32 master parameters: layer l is W [dout][din] row-major, then b [dout].
struct SurLayout {
  int din[kSurLayers], dout[kSurLayers];
  int64_t off[kSurLayers];
  int64_t total;
};

struct SurFeat {
  float f[3];
};

// Inference layout (f16 fragments).  Layer 0: 4 out tiles x 1 K step (the 6
// inputs padded to 16); layers 1..3: 4 x 8; output: 1 x 8 (18 outputs padded
// to 32).  Each (tile, step) holds 64 lanes x 8 halves.
constexpr int kSurFrag = 64 * 8;
__host__ __device__ constexpr int sur_frag_base(int L) {
  return L == 0 ? 0 : (L < 4 ? 4 * kSurFrag + (L - 1) * 32 * kSurFrag : 4 * kSurFrag + 3 * 32 * kSurFrag);
}
constexpr int kSurInfHalves = sur_frag_base(4) + 8 * kSurFrag;  // 55296
constexpr int kSurInfBias = 4 * kSurHidden + 32;                // f32 biases, output padded to 32
constexpr size_t kSurInfLds = sizeof(uint16_t) * kSurInfHalves + sizeof(float) * kSurInfBias;

// Input feature of layer L >= 1 fed by lane half h, element e of K step c:
// the previous layer's output feature held in accumulator r = 8 (c % 2) + e
// of out tile c / 2.
__host__ __device__ constexpr int sur_in_feature(int c, int h, int e) {
  return 32 * (c >> 1) + ((((c & 1) << 3) + e) >> 2) * 8 + 4 * h + (e & 3);
}
// Output feature in accumulator r of out tile t for lane half h.
__host__ __device__ constexpr int sur_out_feature(int t, int r, int h) {
  return 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
}

// What the kernels need to use a trained network.
struct SurDev {
  const uint16_t* wi;         // inference weights (f16 bits), kSurInfHalves
  const float* bi;            // inference biases, kSurInfBias
  SurFeat ft;
  const unsigned char* mask;  // [6][bins][bins], 1 = network within tolerance
  int bins;
  float yscale;
  int on;
};

typedef _Float16 sur_h8 __attribute__((ext_vector_type(8)));
typedef float sur_f16v __attribute__((ext_vector_type(16)));

// Copy the inference weights and biases into LDS (whole block).
__device__ __forceinline__ void sur_stage(const SurDev& s, unsigned char* lds) {
  const uint4* src = reinterpret_cast<const uint4*>(s.wi);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  for (int i = threadIdx.x; i < kSurInfHalves / 8; i += blockDim.x) dst[i] = src[i];
  float* bd = reinterpret_cast<float*>(lds + sizeof(uint16_t) * kSurInfHalves);
  for (int i = threadIdx.x; i < kSurInfBias; i += blockDim.x) bd[i] = s.bi[i];
}

__device__ __forceinline__ float sur_silu(float z) { return z * __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// Bias + SiLU on the four out tiles of a hidden layer, rounded to f16 as the
// next layer's B operand (K step c = 2 t + r / 8, element r % 8).
__device__ __forceinline__ void sur_act(const sur_f16v* acc, const float* bias, int h, sur_h8* B) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) B[2 * t + (r >> 3)][r & 7] = (_Float16)sur_silu(acc[t][r] + bias[sur_out_feature(t, r, h)]);
}

// The network for the 64 rows of a wave, one row per lane: x[6] is this
// lane's row, y[18] receives its outputs.  All 64 lanes must call it
// together (matrix-core instructions and lane shuffles).  lds: the staged
// weights and biases.
__device__ __forceinline__ void sur_wave_eval(const unsigned char* lds, const float* x, float* y) {
  const sur_h8* W = reinterpret_cast<const sur_h8*>(lds);
  const float* bias = reinterpret_cast<const float*>(lds + sizeof(uint16_t) * kSurInfHalves);
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const sur_f16v zero = {};
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    // rows of this pass: the lanes 32 pass .. 32 pass + 31; row n enters
    // through lane n (half 0, elements 0..5)
    float xr[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) xr[i] = __shfl(x[i], (lane & 31) + 32 * pass, 64);
    sur_h8 b0 = {};
    if (h == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) b0[i] = (_Float16)xr[i];
    }
    sur_f16v acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(W[(sur_frag_base(0) / 8) + t * 64 + lane], b0, zero, 0, 0, 0);
    sur_h8 B[8];
    sur_act(acc, bias, h, B);
#pragma unroll 1
    for (int L = 1; L < 4; ++L) {
      const sur_h8* WL = W + sur_frag_base(L) / 8;
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = zero;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(WL[(t * 8 + c) * 64 + lane], B[c], acc[t], 0, 0, 0);
        // keep each step's weight loads next to its products (hoisting them
        // all would need 128 more registers)
        __builtin_amdgcn_sched_barrier(0);
      }
      sur_act(acc, bias + kSurHidden * L, h, B);
    }
    sur_f16v o = zero;
    const sur_h8* WO = W + sur_frag_base(4) / 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) o = __builtin_amdgcn_mfma_f32_32x32x16_f16(WO[c * 64 + lane], B[c], o, 0, 0, 0);
    // outputs 0..17 of row lane % 32: half 0 holds 0-3, 8-11, 16-17 in
    // accumulators 0..9, half 1 holds 4-7, 12-15 in accumulators 0..7
    float v[10], pv[10];
#pragma unroll
    for (int r = 0; r < 10; ++r) v[r] = o[r] + bias[4 * kSurHidden + sur_out_feature(0, r, h)];
#pragma unroll
    for (int r = 0; r < 10; ++r) pv[r] = __shfl_xor(v[r], 32, 64);
    if (h == pass) {
      const float* v0 = h == 0 ? v : pv;
      const float* v1 = h == 0 ? pv : v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        y[r] = v0[r];
        y[8 + r] = v0[4 + r];
        y[4 + r] = v1[r];
        y[12 + r] = v1[4 + r];
      }
      y[16] = v0[8];
      y[17] = v0[9];
    }
  }
}

// Cube-map bin of a unit direction: face = 2*axis + (negative), (u, v) the
// other two coordinates over |T_axis|.
__device__ __forceinline__ int sur_bin(const float* t, int bins) {
  float a0 = fabsf(t[0]), a1 = fabsf(t[1]), a2 = fabsf(t[2]);
  int ax = (a0 >= a1 && a0 >= a2) ? 0 : (a1 >= a2 ? 1 : 2);
  float am = fabsf(t[ax]);
  int face = 2 * ax + (t[ax] < 0.f ? 1 : 0);
  float u = t[(ax + 1) % 3] / am, v = t[(ax + 2) % 3] / am;
  int bi = min(bins - 1, max(0, (int)floorf((u + 1.f) * 0.5f * bins)));
  int bj = min(bins - 1, max(0, (int)floorf((v + 1.f) * 0.5f * bins)));
  return (face * bins + bi) * bins + bj;
}

// D += f * y expanded to the 27 entries (symmetric in v, p), with
// f = scale * yscale / (c44 r^2): the anisotropic part of dG predicted by
// the network (y = its 18 outputs).
template <typename T>
__device__ __forceinline__ void sur_aniso_add(const float* y, T f, T* D) {
#pragma unroll
  for (int c = 0; c < 18; ++c) {
    const int pr = c / 3, q = c % 3;
    const int v = sur_pair_v(pr), p = sur_pair_p(pr);
    D[(v * 3 + p) * 3 + q] += f * (T)y[c];
    if (v != p) D[(p * 3 + v) * 3 + q] += f * (T)y[c];
  }
}

}  // namespace dfmm
