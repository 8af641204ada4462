// Device-side evaluation of the anisotropic-kernel surrogate network and its
// use in place of the unit-circle quadrature (see mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernel_eval.h"

namespace dfmm {

constexpr int kSurLayers = 5;   // 4 hidden layers + output layer
constexpr int kSurHidden = 128;
// distinct (v, p) pairs of the symmetric index pair of d_q G_vp
__device__ __host__ constexpr int sur_pair_v(int k) { return k < 3 ? k : (k == 3 ? 1 : 0); }
__device__ __host__ constexpr int sur_pair_p(int k) { return k < 3 ? k : (k == 5 ? 1 : 2); }

struct SurLayout {
  int din[kSurLayers], dout[kSurLayers];
  int64_t off[kSurLayers];  // start of layer l: W [dout][din] row-major, then b [dout]
  int64_t total;
};

struct SurFeat {
  float f[3];
};

// y[18] = net(x[6]); h: scratch of 2*128 floats, element i at h[i*STRIDE].
template <int STRIDE>
__device__ __forceinline__ void mlp_eval(const float* __restrict__ w, const SurLayout& L, const float* x, float* y,
                                         float* h) {
  // layer 0
  {
    const float* W = w + L.off[0];
    const float* b = W + kSurHidden * 6;
    for (int j = 0; j < kSurHidden; ++j) {
      float z = b[j];
#pragma unroll
      for (int i = 0; i < 6; ++i) z += W[j * 6 + i] * x[i];
      h[j * STRIDE] = z / (1.f + __expf(-z));
    }
  }
  int cur = 0;
  for (int l = 1; l < kSurLayers - 1; ++l) {
    const float* W = w + L.off[l];
    const float* b = W + kSurHidden * kSurHidden;
    float* hin = h + cur * kSurHidden * STRIDE;
    float* hout = h + (1 - cur) * kSurHidden * STRIDE;
    for (int j = 0; j < kSurHidden; ++j) {
      float z = b[j];
      const float* Wr = W + j * kSurHidden;
      for (int i = 0; i < kSurHidden; ++i) z += Wr[i] * hin[i * STRIDE];
      hout[j * STRIDE] = z / (1.f + __expf(-z));
    }
    cur = 1 - cur;
  }
  {
    const float* W = w + L.off[kSurLayers - 1];
    const float* b = W + 18 * kSurHidden;
    const float* hin = h + cur * kSurHidden * STRIDE;
    for (int j = 0; j < 18; ++j) {
      float z = b[j];
      const float* Wr = W + j * kSurHidden;
      for (int i = 0; i < kSurHidden; ++i) z += Wr[i] * hin[i * STRIDE];
      y[j] = z;
    }
  }
}

// What the kernels need to use a trained network.
struct SurDev {
  const float* w;
  SurLayout L;
  SurFeat ft;
  const unsigned char* mask;  // [6][bins][bins], 1 = network within tolerance
  int bins;
  float yscale;
  int on;
};

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

// D += scale * c44^-1 r^-2 * yscale * net(T) expanded to the 27 entries
// (symmetric in v, p), i.e. the anisotropic part of dG predicted by the net.
template <int STRIDE>
__device__ __forceinline__ void sur_aniso_acc(const SurDev& s, float c44, float x0, float x1, float x2, float scale,
                                              float* D, float* h) {
  float r2 = x0 * x0 + x1 * x1 + x2 * x2;
  float ir = rsqrtf(r2);
  float in[6] = {x0 * ir, x1 * ir, x2 * ir, s.ft.f[0], s.ft.f[1], s.ft.f[2]};
  float y[18];
  mlp_eval<STRIDE>(s.w, s.L, in, y, h);
  float f = scale * s.yscale / (c44 * r2);
#pragma unroll
  for (int c = 0; c < 18; ++c) {
    int pr = c / 3, q = c % 3;
    int v = sur_pair_v(pr), p = sur_pair_p(pr);
    D[(v * 3 + p) * 3 + q] += f * y[c];
    if (v != p) D[(p * 3 + v) * 3 + q] += f * y[c];
  }
}

}  // namespace dfmm
