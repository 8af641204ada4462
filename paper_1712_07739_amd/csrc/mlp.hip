// Learned surrogate for the anisotropic part of the Green's-function
// derivative (the costly kernel evaluation of Sec. 2), trained on the GPU.
//
// The singular anisotropic derivative is r^-2 Phi(T) with T = x/r.  The
// network predicts the scaled residual
//     y(T) = c44 (Phi_circle(T) - Phi_iso[Voigt](T)) / yscale
// for the 18 distinct components (v <= p) x q of Phi_vpq, from the features
// (T, normalised c11, c12, c44): 6 -> 4 x 128 (SiLU) -> 18.  Training
// samples are directions drawn by a counter-based generator with targets from
// the FP64 circle quadrature of kernel_eval.h.  Every product of the forward
// and backward passes runs on the matrix cores (f16 operands, f32
// accumulation, f32 master weights and Adam moments); inference uses the
// wave-level network of mlp_eval.h with the weights packed into its f16
// fragment layout after every change.  A cube-map table of direction bins
// records, per bin, the largest error of the network (as inference computes
// it) against the exact quadrature on a grid of validation directions,
// relative to the largest component of Phi there; bins above the tolerance
// keep the exact quadrature.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>

#include "internal.h"
#include "mlp_eval.h"

namespace dfmm {

static inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// SplitMix64 (Steele, Lea, Flood 2014): counter -> 64 random bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t bits) { return (bits >> 11) * (1.0 / 9007199254740992.0); }

// Exact target y(T) (unscaled) in double for a unit direction.
__device__ void exact_residual(const double* T, const Med<double>& m, double* y18, double* phimax) {
  double Dc[27], Di[27];
  for (int i = 0; i < 27; ++i) Dc[i] = Di[i] = 0.0;
  dg_circle_acc<double>(T[0], T[1], T[2], m, 1.0, Dc);
  dg_iso_acc<double>(T[0], T[1], T[2], m.mu, m.nu, 0.0, 1.0, Di);
  double mx = 0.0;
  for (int c = 0; c < 18; ++c) {
    int pr = c / 3, q = c % 3;
    int v = sur_pair_v(pr), p = sur_pair_p(pr);
    int idx = (v * 3 + p) * 3 + q;
    y18[c] = m.c44 * (Dc[idx] - Di[idx]);
    mx = fmax(mx, fabs(m.c44 * Dc[idx]));
  }
  *phimax = mx;
}

__global__ void k_gen_samples(uint64_t seed, int64_t n, Med<double> m, SurFeat ft, float* X, float* Y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t r1 = splitmix64(seed ^ (2 * (uint64_t)i)), r2 = splitmix64(seed ^ (2 * (uint64_t)i + 1));
  double z = 2.0 * u01(r1) - 1.0, ph = 2.0 * 3.14159265358979323846 * u01(r2);
  double s = sqrt(fmax(0.0, 1.0 - z * z));
  double T[3] = {s * cos(ph), s * sin(ph), z};
  double y[18], pm;
  exact_residual(T, m, y, &pm);
  float* x = X + i * 6;
  x[0] = (float)T[0];
  x[1] = (float)T[1];
  x[2] = (float)T[2];
  x[3] = ft.f[0];
  x[4] = ft.f[1];
  x[5] = ft.f[2];
  for (int c = 0; c < 18; ++c) Y[i * 18 + c] = (float)y[c];
}

__global__ void k_scale(float* Y, int64_t n, float s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Y[i] *= s;
}

__global__ void k_sumsq(const float* Y, int64_t n, double* part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += (double)Y[i] * Y[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// C[M x N] (ldc) = alpha op(A) op(B), row-major, f32 in memory;
// op(A)[m][k] = TA ? A[k*lda+m] : A[m*lda+k], op(B)[k][n] = TB ? B[n*ldb+k] :
// B[k*ldb+n].  On the matrix cores: tiles of 64 x 64 per block of four waves
// (each wave a 32 x 32 quarter, v_mfma_f32_32x32x16_f16), K in chunks of 32
// staged in LDS as f16, f32 accumulation.  blockIdx.z selects a K range of
// length kchunk (split-K); its result goes to C + z * (M * ldc).
constexpr int kGemmKC = 32;
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                                              float* C, int ldc, float alpha, int kchunk) {
  __shared__ _Float16 As[64][kGemmKC + 8];  // [m][k] (rows padded against bank conflicts)
  __shared__ _Float16 Bs[64][kGemmKC + 8];  // [n][k]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  C += (int64_t)blockIdx.z * M * ldc;
  sur_f16v acc = {};
  for (int k0 = kb; k0 < ke; k0 += kGemmKC) {
    // reads run along the contiguous index of each operand
    for (int e = threadIdx.x; e < 64 * kGemmKC; e += 256) {
      const int i = TA ? e % 64 : e / kGemmKC, k = TA ? e / 64 : e % kGemmKC;
      const int gm = m0 + i, gk = k0 + k;
      As[i][k] = (_Float16)((gm < M && gk < ke) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.f);
    }
    for (int e = threadIdx.x; e < 64 * kGemmKC; e += 256) {
      const int j = TB ? e / kGemmKC : e % 64, k = TB ? e % kGemmKC : e / 64;
      const int gn = n0 + j, gk = k0 + k;
      Bs[j][k] = (_Float16)((gn < N && gk < ke) ? (TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn]) : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmKC; kk += 16) {
      sur_h8 av, bv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        av[e] = As[wm + (lane & 31)][kk + 8 * (lane >> 5) + e];
        bv[e] = Bs[wn + (lane & 31)][kk + 8 * (lane >> 5) + e];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gm = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), gn = n0 + wn + (lane & 31);
    if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = alpha * acc[r];
  }
}

// Z += b (per column); A = SiLU(Z) when act, else A = Z.
__global__ void k_bias_act(float* Z, const float* b, int64_t rows, int cols, float* A, int act) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  float z = Z[i] + b[i % cols];
  Z[i] = z;
  A[i] = act ? z / (1.f + expf(-z)) : z;
}

// dY = 2 (Yp - Y) (the 1 / (rows*cols) of the mean is applied to the
// gradients at the end, so the backward operands stay in f16's normal
// range); per-block partial sums of the squared error.
__global__ void k_mse(const float* Yp, const float* Y, int64_t n, float* dY, double* part) {
  __shared__ double sh[256];
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    float d = Yp[i] - Y[i];
    dY[i] = 2.f * d;
    e = (double)d * d;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dZ = dA * SiLU'(Z)
__global__ void k_silu_back(const float* dA, const float* Z, int64_t n, float* dZ) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float z = Z[i], s = 1.f / (1.f + expf(-z));
  dZ[i] = dA[i] * s * (1.f + z * (1.f - s));
}

// db[j] = alpha sum_i dZ[i][j]: one block per column, fixed-order tree reduction
__global__ void k_colsum(const float* dZ, int rows, int cols, float alpha, float* db) {
  __shared__ float sh[256];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < rows; i += 256) s += dZ[(int64_t)i * cols + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = alpha * sh[0];
}

// C[i] = sum over the S split-K partials (fixed order)
__global__ void k_sum_parts(const float* part, int64_t n, int S, float* C) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[(int64_t)k * n + i];
  C[i] = s;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_init_params(float* w, SurLayout L, uint64_t seed) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.total) return;
  int l = 0;
  while (l + 1 < kSurLayers && i >= L.off[l + 1]) ++l;
  int64_t local = i - L.off[l];
  int64_t nw = (int64_t)L.dout[l] * L.din[l];
  if (local >= nw) {
    w[i] = 0.f;  // bias
    return;
  }
  double u = u01(splitmix64(seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(i + 1))));
  double lim = sqrt(6.0 / (L.din[l] + L.dout[l]));  // Glorot uniform
  w[i] = (float)((2.0 * u - 1.0) * lim);
}

// f32 master parameters -> the f16 fragment layout of the wave-level
// inference (mlp_eval.h) and its f32 biases.  One thread per f16 value.
__global__ void k_pack_inference(const float* w, SurLayout L, uint16_t* wi, float* bi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kSurInfBias) {
    const int layer = i < 4 * kSurHidden ? i / kSurHidden : 4, m = i < 4 * kSurHidden ? i % kSurHidden : i - 4 * kSurHidden;
    bi[i] = m < L.dout[layer] ? w[L.off[layer] + (int64_t)L.dout[layer] * L.din[layer] + m] : 0.f;
  }
  if (i >= kSurInfHalves) return;
  int layer = 4;
  for (int l = 1; l <= 4; ++l)
    if (i < sur_frag_base(l)) {
      layer = l - 1;
      break;
    }
  const int steps = layer == 0 ? 1 : 8;
  const int local = i - sur_frag_base(layer);
  const int e = local % 8, lane = (local / 8) % 64, ts = local / kSurFrag;
  const int t = ts / steps, c = ts % steps, h = lane >> 5;
  const int m = 32 * t + (lane & 31);
  const int k = layer == 0 ? 8 * h + e : sur_in_feature(c, h, e);
  float v = 0.f;
  if (m < L.dout[layer] && k < L.din[layer]) v = w[L.off[layer] + (int64_t)m * L.din[layer] + k];
  const _Float16 hv = (_Float16)v;
  wi[i] = __builtin_bit_cast(uint16_t, hv);
}

// Network outputs Y[n][18] for rows X[n][6] by the wave-level inference,
// weights staged in LDS once per block; each wave takes 64 rows at a time.
__global__ void __launch_bounds__(512) k_sur_infer(SurDev sd, const float* X, int64_t n, float* Y) {
  extern __shared__ __align__(16) unsigned char lds[];
  sur_stage(sd, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t nw = blockDim.x / 64;
  const int64_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  for (int64_t base = ((int64_t)blockIdx.x * nw + wave) * 64; base < n; base += (int64_t)gridDim.x * nw * 64) {
    const int64_t i = base + lane;
    float x[6] = {1.f, 0.f, 0.f, 0.f, 0.f, 0.f}, y[18];
    if (i < n)
#pragma unroll
      for (int k = 0; k < 6; ++k) x[k] = X[i * 6 + k];
    sur_wave_eval(lds, x, y);
    if (i < n)
#pragma unroll
      for (int k = 0; k < 18; ++k) Y[i * 18 + k] = y[k];
  }
}

// Validation directions of the cube map: bin b = (face, i, j), nsub x nsub
// directions per bin.  Writes the network's input rows and the exact target.
__global__ void k_gate_dirs(SurFeat ft, int bins, int nsub, Med<double> m, float* X, double* Yex, double* pmax) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nbins = 6LL * bins * bins;
  if (idx >= nbins * nsub * nsub) return;
  int64_t b = idx / (nsub * nsub);
  int s = (int)(idx % (nsub * nsub));
  int face = (int)(b / (bins * bins)), bi = (int)((b / bins) % bins), bj = (int)(b % bins);
  double u = -1.0 + 2.0 * (bi + (s / nsub + 0.5) / nsub) / bins;
  double v = -1.0 + 2.0 * (bj + (s % nsub + 0.5) / nsub) / bins;
  double T[3];
  int ax = face >> 1;
  double sg = (face & 1) ? -1.0 : 1.0;
  T[ax] = sg;
  T[(ax + 1) % 3] = u;
  T[(ax + 2) % 3] = v;
  double nn = 1.0 / sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2]);
  for (int d = 0; d < 3; ++d) T[d] *= nn;
  exact_residual(T, m, Yex + idx * 18, pmax + idx);
  float* x = X + idx * 6;
  for (int d = 0; d < 3; ++d) x[d] = (float)T[d];
  x[3] = ft.f[0];
  x[4] = ft.f[1];
  x[5] = ft.f[2];
}

// err[b] = max over a bin's directions of |y_net - y_exact|_inf / |c44 Phi|_inf;
// mask[b] = err[b] <= tol.
__global__ void k_gate_reduce(const float* Yn, const double* Yex, const double* pmax, float yscale, int64_t nbins,
                              int nsub2, float tol, unsigned char* mask, float* binerr) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double e = 0.0;
  for (int s = 0; s < nsub2; ++s) {
    const int64_t r = b * nsub2 + s;
    double es = 0.0;
    for (int c = 0; c < 18; ++c) es = fmax(es, fabs((double)Yn[r * 18 + c] * yscale - Yex[r * 18 + c]));
    e = fmax(e, es / pmax[r]);
  }
  binerr[b] = (float)e;
  mask[b] = e <= tol ? 1 : 0;
}

SurLayout sur_layout(int hidden) {
  SurLayout L;
  int dims[kSurLayers + 1] = {6, hidden, hidden, hidden, hidden, 18};
  int64_t o = 0;
  for (int l = 0; l < kSurLayers; ++l) {
    L.din[l] = dims[l];
    L.dout[l] = dims[l + 1];
    L.off[l] = o;
    o += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
  }
  L.total = o;
  return L;
}

// Split-K scratch of the weight-gradient products (the plan's own buffer).
static int gemm(Surrogate& S, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                int ldb, float* C, int ldc, float alpha, hipStream_t st) {
  int Sp = 1;
  const int tiles = (int)(nb(N, 64) * nb(M, 64));
  if (tiles < 64 && K >= 1024) Sp = std::min(32, K / 256);
  const int kchunk = ((K + Sp - 1) / Sp + kGemmKC - 1) / kGemmKC * kGemmKC;
  Sp = (K + kchunk - 1) / kchunk;
  float* out = C;
  if (Sp > 1) {
    size_t need = (size_t)Sp * M * ldc;
    if (need > S.split_n) {
      hipFree(S.split);
      S.split = nullptr;
      S.split_n = 0;
      DFMM_HIP(hipMalloc(&S.split, sizeof(float) * need));
      S.split_n = need;
    }
    out = S.split;
  }
  dim3 g(nb(N, 64), nb(M, 64), Sp);
  if (!ta && !tb) k_gemm<false, false><<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, out, ldc, alpha, kchunk);
  else if (!ta && tb) k_gemm<false, true><<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, out, ldc, alpha, kchunk);
  else if (ta && !tb) k_gemm<true, false><<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, out, ldc, alpha, kchunk);
  else k_gemm<true, true><<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, out, ldc, alpha, kchunk);
  DFMM_LAUNCH_CHECK();
  if (Sp > 1) {
    k_sum_parts<<<nb((int64_t)M * ldc, 256), 256, 0, st>>>(S.split, (int64_t)M * ldc, Sp, C);
    DFMM_LAUNCH_CHECK();
  }
  return DFMM_OK;
}

// Workspace for one mini-batch of B rows.
struct MlpWork {
  float* Z[kSurLayers] = {};
  float* A[kSurLayers + 1] = {};  // A[0] = input rows (not owned)
  float* dZ = nullptr;
  float* dA = nullptr;
  double* part = nullptr;
  int B = 0;
};

static int work_alloc(MlpWork& w, const SurLayout& L, int B) {
  w.B = B;
  for (int l = 0; l < kSurLayers; ++l) {
    DFMM_HIP(hipMalloc(&w.Z[l], sizeof(float) * (size_t)B * L.dout[l]));
    DFMM_HIP(hipMalloc(&w.A[l + 1], sizeof(float) * (size_t)B * L.dout[l]));
  }
  DFMM_HIP(hipMalloc(&w.dZ, sizeof(float) * (size_t)B * kSurHidden));
  DFMM_HIP(hipMalloc(&w.dA, sizeof(float) * (size_t)B * kSurHidden));
  DFMM_HIP(hipMalloc(&w.part, sizeof(double) * (nb((int64_t)B * 18, 256) + 1)));
  return DFMM_OK;
}
static void work_free(MlpWork& w) {
  for (int l = 0; l < kSurLayers; ++l) {
    hipFree(w.Z[l]);
    hipFree(w.A[l + 1]);
  }
  hipFree(w.dZ);
  hipFree(w.dA);
  hipFree(w.part);
}

// Training forward of n rows of X (A[0] = X), output in w.A[kSurLayers].
static int forward(Surrogate& S, const float* prm, MlpWork& w, const float* X, int n, hipStream_t st) {
  const SurLayout& L = S.L;
  w.A[0] = const_cast<float*>(X);
  for (int l = 0; l < kSurLayers; ++l) {
    const float* W = prm + L.off[l];
    const float* b = W + (int64_t)L.dout[l] * L.din[l];
    int rc = gemm(S, false, true, n, L.dout[l], L.din[l], w.A[l], L.din[l], W, L.din[l], w.Z[l], L.dout[l], 1.f, st);
    if (rc) return rc;
    k_bias_act<<<nb((int64_t)n * L.dout[l], 256), 256, 0, st>>>(w.Z[l], b, n, L.dout[l], w.A[l + 1],
                                                                 l + 1 < kSurLayers);
    DFMM_LAUNCH_CHECK();
  }
  return DFMM_OK;
}

// Loss (host, mean squared error over rows x 18) and gradient into grad.
static int loss_grad(Surrogate& S, const float* prm, float* grad, MlpWork& w, const float* X, const float* Y, int n,
                     hipStream_t st, double* loss) {
  const SurLayout& L = S.L;
  int rc = forward(S, prm, w, X, n, st);
  if (rc) return rc;
  const int64_t no = (int64_t)n * 18;
  const unsigned nbk = nb(no, 256);
  const float inv = 1.f / (float)no;
  float* dY = w.dZ;  // [n][18], carries 2 (Yp - Y); the 1/no is applied to the gradients
  k_mse<<<nbk, 256, 0, st>>>(w.A[kSurLayers], Y, no, dY, w.part);
  DFMM_LAUNCH_CHECK();
  for (int l = kSurLayers - 1; l >= 0; --l) {
    float* gW = grad + L.off[l];
    float* gb = gW + (int64_t)L.dout[l] * L.din[l];
    const float* W = prm + L.off[l];
    // dW = dZ^T A_l ; db = colsum(dZ)
    if ((rc = gemm(S, true, false, L.dout[l], L.din[l], n, w.dZ, L.dout[l], w.A[l], L.din[l], gW, L.din[l], inv, st)))
      return rc;
    k_colsum<<<L.dout[l], 256, 0, st>>>(w.dZ, n, L.dout[l], inv, gb);
    DFMM_LAUNCH_CHECK();
    if (l > 0) {
      // dA_l = dZ W ; dZ_{l-1} = dA_l * SiLU'(Z_{l-1})
      if ((rc = gemm(S, false, false, n, L.din[l], L.dout[l], w.dZ, L.dout[l], W, L.din[l], w.dA, L.din[l], 1.f, st)))
        return rc;
      k_silu_back<<<nb((int64_t)n * L.din[l], 256), 256, 0, st>>>(w.dA, w.Z[l - 1], (int64_t)n * L.din[l], w.dZ);
      DFMM_LAUNCH_CHECK();
    }
  }
  if (loss) {
    std::vector<double> h(nbk);
    DFMM_D2H(h.data(), w.part, sizeof(double) * nbk, st);
    double s = 0.0;
    for (double x : h) s += x;
    *loss = s / (double)no;
  }
  return DFMM_OK;
}

// The inference copy of the current master weights.
int surrogate_pack(dfmm_plan* pl, hipStream_t st) {
  Surrogate& S = pl->sur;
  if (!S.wi) {
    DFMM_HIP(hipMalloc(&S.wi, sizeof(uint16_t) * kSurInfHalves));
    DFMM_HIP(hipMalloc(&S.bi, sizeof(float) * kSurInfBias));
  }
  k_pack_inference<<<nb(kSurInfHalves, 256), 256, 0, st>>>(S.w, S.L, S.wi, S.bi);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

// Blocks of the persistent inference kernels: one per CU (the weights take
// 110 KB of its LDS).
int sur_grid(int device) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0) ncu = 256;
  return ncu;
}

int surrogate_infer(const dfmm_plan* pl, const float* X, int64_t n, float* Y, hipStream_t st) {
  static std::once_flag once;
  std::call_once(once, [] {
    hipFuncSetAttribute((const void*)k_sur_infer, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSurInfLds);
  });
  SurDev sd = sur_dev(pl);
  const int64_t waves = (n + 63) / 64;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(sur_grid(pl->device), (waves + 7) / 8));
  k_sur_infer<<<grid, 512, kSurInfLds, st>>>(sd, X, n, Y);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

int surrogate_alloc(dfmm_plan* pl, uint64_t seed, hipStream_t st) {
  Surrogate& S = pl->sur;
  S.L = sur_layout(kSurHidden);
  double c = pl->prm.c11 + pl->prm.c12 + pl->prm.c44;
  S.ft.f[0] = (float)(pl->prm.c11 / c);
  S.ft.f[1] = (float)(pl->prm.c12 / c);
  S.ft.f[2] = (float)(pl->prm.c44 / c);
  const int64_t P = S.L.total;
  if (!S.w) {
    DFMM_HIP(hipMalloc(&S.w, sizeof(float) * P));
    DFMM_HIP(hipMalloc(&S.g, sizeof(float) * P));
    DFMM_HIP(hipMalloc(&S.m, sizeof(float) * P));
    DFMM_HIP(hipMalloc(&S.v, sizeof(float) * P));
  }
  k_init_params<<<nb(P, 256), 256, 0, st>>>(S.w, S.L, seed);
  DFMM_LAUNCH_CHECK();
  DFMM_HIP(hipMemsetAsync(S.m, 0, sizeof(float) * P, st));
  DFMM_HIP(hipMemsetAsync(S.v, 0, sizeof(float) * P, st));
  int rc = surrogate_pack(pl, st);
  if (rc) return rc;
  DFMM_HIP(hipStreamSynchronize(st));
  return DFMM_OK;
}

// Residual gate of the current weights: bins of bins x bins per cube face,
// nsub x nsub validation directions per bin.
int surrogate_gate(dfmm_plan* pl, int bins, double tol, hipStream_t st) {
  Surrogate& S = pl->sur;
  const int64_t nbins = 6LL * bins * bins;
  const int nsub = 3;
  const int64_t nd = nbins * nsub * nsub;
  float *X = nullptr, *Yn = nullptr, *binerr = nullptr;
  double *Yex = nullptr, *pmax = nullptr;
  int rc = DFMM_OK;
  if (hipMalloc(&X, sizeof(float) * 6 * nd) != hipSuccess || hipMalloc(&Yn, sizeof(float) * 18 * nd) != hipSuccess ||
      hipMalloc(&Yex, sizeof(double) * 18 * nd) != hipSuccess || hipMalloc(&pmax, sizeof(double) * nd) != hipSuccess ||
      hipMalloc(&binerr, sizeof(float) * nbins) != hipSuccess) {
    set_error("surrogate: cannot allocate the gate's scratch");
    rc = DFMM_E_NOMEM;
  }
  if (rc == DFMM_OK) {
    hipFree(S.mask);
    S.mask = nullptr;
    if (hipMalloc(&S.mask, nbins) != hipSuccess) {
      set_error("surrogate: cannot allocate the gate");
      rc = DFMM_E_NOMEM;
    }
  }
  std::vector<float> hb(nbins);
  if (rc == DFMM_OK) {
    S.bins = bins;
    S.tol = tol;
    k_gate_dirs<<<nb(nd, 64), 64, 0, st>>>(S.ft, bins, nsub, pl->med<double>(), X, Yex, pmax);
    rc = hipGetLastError() == hipSuccess ? DFMM_OK : DFMM_E_HIP;
    if (rc == DFMM_OK) rc = surrogate_infer(pl, X, nd, Yn, st);
    if (rc == DFMM_OK) {
      k_gate_reduce<<<nb(nbins, 256), 256, 0, st>>>(Yn, Yex, pmax, S.yscale, nbins, nsub * nsub, (float)tol, S.mask,
                                                    binerr);
      rc = hipGetLastError() == hipSuccess ? DFMM_OK : DFMM_E_HIP;
    }
    if (rc == DFMM_OK && (hipMemcpyAsync(hb.data(), binerr, sizeof(float) * nbins, hipMemcpyDeviceToHost, st) != hipSuccess ||
                          hipStreamSynchronize(st) != hipSuccess))
      rc = DFMM_E_HIP;
    if (rc == DFMM_E_HIP) set_error("surrogate: gate kernels failed");
  }
  hipFree(X);
  hipFree(Yn);
  hipFree(Yex);
  hipFree(pmax);
  hipFree(binerr);
  if (rc) return rc;
  int64_t pass = 0;
  for (float e : hb) pass += e <= tol;
  std::vector<float> sorted(hb);
  std::sort(sorted.begin(), sorted.end());
  S.pass_frac = (double)pass / nbins;
  S.max_err = sorted.back();
  S.med_err = sorted[nbins / 2];
  return DFMM_OK;
}

int surrogate_train(dfmm_plan* pl, const dfmm_surrogate_cfg& cfg, hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  Surrogate& S = pl->sur;
  if (cfg.hidden != kSurHidden) {
    set_error("surrogate: hidden width must be 128");
    return DFMM_E_ARG;
  }
  if (cfg.n_samples < 1024 || cfg.batch < 64 || cfg.batch > cfg.n_samples || cfg.epochs < 1 || !(cfg.lr > 0) ||
      cfg.bins < 1 || cfg.bins > 256 || !(cfg.tol >= 0)) {
    set_error("surrogate: invalid training configuration");
    return DFMM_E_ARG;
  }
  int rc0 = surrogate_alloc(pl, cfg.seed, st);
  if (rc0) return rc0;
  S.trained = 0;
  const int64_t P = S.L.total;
  // samples
  const int64_t n = cfg.n_samples;
  float *X = nullptr, *Y = nullptr;
  DFMM_HIP(hipMalloc(&X, sizeof(float) * 6 * n));
  DFMM_HIP(hipMalloc(&Y, sizeof(float) * 18 * n));
  Med<double> m = pl->med<double>();
  k_gen_samples<<<nb(n, 128), 128, 0, st>>>(cfg.seed ^ 0xA5A5A5A5ull, n, m, S.ft, X, Y);
  DFMM_LAUNCH_CHECK();
  {
    double* part = nullptr;
    DFMM_HIP(hipMalloc(&part, sizeof(double) * 1024));
    k_sumsq<<<1024, 256, 0, st>>>(Y, 18 * n, part);
    std::vector<double> h(1024);
    DFMM_D2H(h.data(), part, sizeof(double) * 1024, st);
    hipFree(part);
    double ss = 0;
    for (double x : h) ss += x;
    double rms = std::sqrt(ss / (18.0 * n));
    S.yscale = (float)(rms > 0 ? rms : 1.0);
    k_scale<<<nb(18 * n, 256), 256, 0, st>>>(Y, 18 * n, 1.f / S.yscale);
    DFMM_LAUNCH_CHECK();
  }
  MlpWork w;
  int rc = work_alloc(w, S.L, cfg.batch);
  if (rc) return rc;
  const int64_t steps_per_epoch = n / cfg.batch;
  const int64_t total = steps_per_epoch * cfg.epochs;
  S.loss_hist.clear();
  int64_t step = 0;
  for (int ep = 0; ep < cfg.epochs && rc == DFMM_OK; ++ep) {
    double ep_loss = 0;
    for (int64_t k = 0; k < steps_per_epoch && rc == DFMM_OK; ++k, ++step) {
      int64_t row = ((k + (int64_t)ep * 7919) % steps_per_epoch) * cfg.batch;
      bool want = (k == steps_per_epoch - 1);
      double l = 0;
      rc = loss_grad(S, S.w, S.g, w, X + row * 6, Y + row * 18, cfg.batch, st, want ? &l : nullptr);
      if (rc) break;
      double frac = (double)step / (double)std::max<int64_t>(1, total - 1);
      float lr = (float)(cfg.lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * frac))));
      float c1 = 1.f - std::pow(0.9f, (float)(step + 1)), c2 = 1.f - std::pow(0.999f, (float)(step + 1));
      k_adam<<<nb(P, 256), 256, 0, st>>>(S.w, S.g, S.m, S.v, P, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
      if (hipGetLastError() != hipSuccess) { rc = DFMM_E_HIP; break; }
      if (want) ep_loss = l;
    }
    S.loss_hist.push_back(ep_loss);
  }
  work_free(w);
  hipFree(X);
  hipFree(Y);
  if (rc) return rc;
  if ((rc = surrogate_pack(pl, st))) return rc;
  if ((rc = surrogate_gate(pl, cfg.bins, cfg.tol, st))) return rc;
  S.n_samples = n;
  S.epochs = cfg.epochs;
  S.trained = 1;
  S.train_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return DFMM_OK;
}

// Test hooks: loss and gradient of the current weights on rows (X, Y) given
// on the device (the training path), and the network outputs for rows X
// (the inference path the kernels use).
int surrogate_loss_grad(dfmm_plan* pl, const float* X, const float* Y, int64_t n, float* grad, double* loss,
                        hipStream_t st) {
  Surrogate& S = pl->sur;
  MlpWork w;
  int rc = work_alloc(w, S.L, (int)n);
  if (rc == DFMM_OK) rc = loss_grad(S, S.w, grad, w, X, Y, (int)n, st, loss);
  hipStreamSynchronize(st);
  work_free(w);
  return rc;
}

int surrogate_forward(const dfmm_plan* pl, const float* X, int64_t n, float* Yout, hipStream_t st) {
  int rc = surrogate_infer(pl, X, n, Yout, st);
  if (rc) return rc;
  DFMM_HIP(hipStreamSynchronize(st));
  return DFMM_OK;
}

}  // namespace dfmm
