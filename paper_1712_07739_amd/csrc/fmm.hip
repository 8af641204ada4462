// Lagrange FMM evaluation (Sec. 4.3, Alg. lagrange) and the direct sum
// (Eq. stress3) on gfx950.
//
// Stages of dfmm_fmm_forces, all on the caller's stream:
//   points   quadrature points and strengths in Morton order (Eq. stress_discrete)
//   P2M      anterpolation of the leaf points onto the p^3 leaf nodes
//   M2M      anterpolation of children onto the parent nodes (separable)
//   M2L      per level: DFT of the multipole weights, Hadamard product with
//            the offset spectra summed over the interaction list (Theorem 1),
//            inverse DFT to the p^3 local nodes
//   L2L      interpolation of the parent's local values at the child nodes
//   leaf     L2P at every point + the direct near field over the 27
//            neighbour leaves
//   forces   Gauss quadrature of (sigma.b) x dS with shape functions (1-s, s)
#include <algorithm>
#include <cmath>

#include <mutex>
#include <utility>

#include "internal.h"

namespace dfmm {

template <typename T>
struct cplx {
  T re, im;
};

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename T>
__device__ __forceinline__ T lagr(int p, int i, T t) {
  // ell_i(t) for nodes k/(p-1), k = 0..p-1: the numerator's product, then
  // one division by the integer product of (i - k) (exact in int, at most
  // 7! in magnitude), not one division per factor
  T v = T(1);
  int den = 1;
  T tp = t * T(p - 1);
  for (int k = 0; k < p; ++k)
    if (k != i) {
      v *= tp - T(k);
      den *= i - k;
    }
  return v / T(den);
}

// ---------------------------------------------------------------- points
__global__ void k_gather(const double* seg, const double* burg, const uint32_t* perm, Quad qd, int64_t N,
                         double* pts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t j = perm[i];
  int64_t s = j / qd.n;
  int k = (int)(j - s * qd.n);
  double x[3], t[3];
  quad_point(seg, s, k, qd, x, t);
  for (int d = 0; d < 3; ++d) {
    pts[d * N + i] = x[d];
    pts[(3 + d) * N + i] = burg[3 * s + d];
    pts[(6 + d) * N + i] = t[d];
  }
}

__device__ __forceinline__ void cell_lo(uint32_t key, double lo0, double lo1, double lo2, double sz,
                                        double* lo) {
  uint32_t v[3] = {key >> 2, key >> 1, key};
  for (int d = 0; d < 3; ++d) {
    uint32_t x = v[d] & 0x09249249;
    x = (x | (x >> 2)) & 0x030C30C3;
    x = (x | (x >> 4)) & 0x0300F00F;
    x = (x | (x >> 8)) & 0x030000FF;
    x = (x | (x >> 16)) & 0x3ff;
    lo[d] = (d == 0 ? lo0 : d == 1 ? lo1 : lo2) + x * sz;
  }
}

// The largest |v| over a block's threads folded into *wmax (the bits of a
// non-negative float, whose order as unsigned integers is the float order);
// every thread of the block calls it.  The running value is read first and
// the atomic issued only above it: it only grows, so a stale read costs at
// most a needless atomic, and the blocks of a level do not all queue on one
// address.
__device__ __forceinline__ void block_absmax(float m, unsigned* wmax) {
  __shared__ float red[16];
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = red[0];
    for (int w = 1; w < (int)((blockDim.x + 63) >> 6); ++w) r = fmaxf(r, red[w]);
    const unsigned u = __float_as_uint(r);
    if (u > __hip_atomic_load(wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(wmax, u);
  }
}

// ------------------------------------------------------------------- P2M
// One block per leaf; thread = node m.  Points are staged in LDS in chunks of
// 64 with their 1D basis values and 9-component strengths b (x) t.  wmax
// (f16 path, or null): the level's largest |W| is folded in.
template <typename T>
__global__ void k_p2m(const double* pts, int64_t N, const int* first, const int* count, const uint32_t* key,
                      double lo0, double lo1, double lo2, double sD, int p, T* W, const int* cell,
                      unsigned* wmax) {
  extern __shared__ unsigned char shraw[];
  T* Lb = (T*)shraw;          // [64][3][p]
  T* qs = Lb + 64 * 3 * p;    // [64][9]
  // leaf blockIdx.x of the launch; its cell (the row of key and W) is the
  // same index, or cell[blockIdx.x] (the leaves of one level of an adaptive tree)
  const int li = blockIdx.x, leaf = cell ? cell[li] : li, p3 = p * p * p;
  const int f0 = first[li], cnt = count[li];
  double lo[3];
  cell_lo(key[leaf], lo0, lo1, lo2, sD, lo);
  const int tid = threadIdx.x;
  const int m1 = tid / (p * p), m2 = (tid / p) % p, m3 = tid % p;
  T acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = T(0);
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    int nc = min(64, cnt - c0);
    for (int e = tid; e < nc * 3; e += blockDim.x) {
      int pt = e / 3, d = e % 3;
      T t = (T)((pts[d * N + f0 + c0 + pt] - lo[d]) / sD);
      for (int i = 0; i < p; ++i) Lb[(pt * 3 + d) * p + i] = lagr<T>(p, i, t);
    }
    for (int e = tid; e < nc * 9; e += blockDim.x) {
      int pt = e / 9, c = e % 9;
      int64_t j = f0 + c0 + pt;
      qs[pt * 9 + c] = (T)(pts[(3 + c / 3) * N + j] * pts[(6 + c % 3) * N + j]);
    }
    __syncthreads();
    if (tid < p3) {
      for (int pt = 0; pt < nc; ++pt) {
        T w = Lb[(pt * 3 + 0) * p + m1] * Lb[(pt * 3 + 1) * p + m2] * Lb[(pt * 3 + 2) * p + m3];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] += w * qs[pt * 9 + c];
      }
    }
    __syncthreads();
  }
  float am = 0.f;
  if (tid < p3) {
    T* out = W + (int64_t)leaf * 9 * p3;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      out[c * p3 + tid] = acc[c];
      am = fmaxf(am, fabsf((float)acc[c]));
    }
  }
  if (wmax) block_absmax(am, wmax);
}

// ------------------------------------------------------- separable passes
// out[g][a][b][i] = sum_m M(i, m) in[g][a][b][m] along one axis, for the
// three axes in turn; M(i, m) = S[bit][i][m] (anterpolation, M2M) or
// S[bit][m][i] (interpolation, L2L).  A thread takes one line along the axis:
// its P values in registers, all P outputs.  The bit is the same for the
// whole block, so the matrix entries are uniform loads (scalar registers).
// ACC adds the result to out.
template <typename T, bool INTERP, bool ACC, int P, int AXIS>
__device__ __forceinline__ void pass_axis(const T* in, T* out, const T* __restrict__ S, int bit, int ncomp) {
  constexpr int p3 = P * P * P;
  constexpr int stride = AXIS == 2 ? 1 : AXIS == 1 ? P : P * P;
  const T* Sb = S + bit * P * P;
  for (int L = threadIdx.x; L < ncomp * P * P; L += blockDim.x) {
    const int g = L / (P * P), q = L % (P * P);
    const int base = g * p3 + (AXIS == 2 ? q * P : AXIS == 1 ? (q / P) * P * P + q % P : q);
    T x[P];
#pragma unroll
    for (int m = 0; m < P; ++m) x[m] = in[base + m * stride];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      T v = T(0);
#pragma unroll
      for (int m = 0; m < P; ++m) v = fma(INTERP ? Sb[m * P + i] : Sb[i * P + m], x[m], v);
      if (ACC)
        out[base + i * stride] += v;
      else
        out[base + i * stride] = v;
    }
  }
}

// M2M: one block per parent cell; the children's W (next finer level) are
// anterpolated onto the parent's nodes one child at a time.  wmax (f16 path,
// or null): the parent level's largest |W| is folded in.
constexpr int kM2mThreads = 512;  // 9 P^2 lines a pass: one round up to P = 7
template <typename T, int P>
__global__ void __launch_bounds__(kM2mThreads) k_m2m(const int* first, const int* count, const uint32_t* ckey, const T* Wc, T* Wp,
                      const T* __restrict__ Sg, unsigned* wmax) {
  extern __shared__ unsigned char shraw[];
  constexpr int p3 = P * P * P;
  T* A = (T*)shraw;
  T* B = A + 9 * p3;
  T* C = B + 9 * p3;
  for (int e = threadIdx.x; e < 9 * p3; e += blockDim.x) C[e] = T(0);
  const int par = blockIdx.x;
  const int c0 = first[par], nc = count[par];
  // a thread's share of a child's 9 P^3 values, the next child's loaded while
  // the current one is transformed
  constexpr int kM2mVals = (9 * p3 + kM2mThreads - 1) / kM2mThreads;
  T nx[kM2mVals];
  auto load = [&](int c) {
    const T* src = Wc + (int64_t)c * 9 * p3;
#pragma unroll
    for (int k = 0; k < kM2mVals; ++k) {
      const int e = threadIdx.x + k * kM2mThreads;
      if (e < 9 * p3) nx[k] = src[e];
    }
  };
  if (nc > 0) load(c0);
  for (int c = c0; c < c0 + nc; ++c) {
    const uint32_t bits = ckey[c] & 7;
#pragma unroll
    for (int k = 0; k < kM2mVals; ++k) {
      const int e = threadIdx.x + k * kM2mThreads;
      if (e < 9 * p3) A[e] = nx[k];
    }
    if (c + 1 < c0 + nc) load(c + 1);
    __syncthreads();
    pass_axis<T, false, false, P, 2>(A, B, Sg, bits & 1, 9);
    __syncthreads();
    pass_axis<T, false, false, P, 1>(B, A, Sg, (bits >> 1) & 1, 9);
    __syncthreads();
    pass_axis<T, false, true, P, 0>(A, C, Sg, (bits >> 2) & 1, 9);
    __syncthreads();
  }
  T* dst = Wp + (int64_t)par * 9 * p3;
  float am = 0.f;
  for (int e = threadIdx.x; e < 9 * p3; e += blockDim.x) {
    dst[e] = C[e];
    am = fmaxf(am, fabsf((float)C[e]));
  }
  if (wmax) block_absmax(am, wmax);
}

// L2L: one block per child cell; adds the parent's interpolated local values.
template <typename T, int P>
__global__ void k_l2l(const int* parent, const uint32_t* key, const T* sp, T* sc, const T* __restrict__ Sg) {
  extern __shared__ unsigned char shraw[];
  constexpr int p3 = P * P * P;
  T* A = (T*)shraw;
  T* B = A + 6 * p3;
  const int c = blockIdx.x;
  const uint32_t bits = key[c] & 7;
  const T* src = sp + (int64_t)parent[c] * 6 * p3;
  for (int e = threadIdx.x; e < 6 * p3; e += blockDim.x) A[e] = src[e];
  __syncthreads();
  pass_axis<T, true, false, P, 2>(A, B, Sg, bits & 1, 6);
  __syncthreads();
  pass_axis<T, true, false, P, 1>(B, A, Sg, (bits >> 1) & 1, 6);
  __syncthreads();
  T* dst = sc + (int64_t)c * 6 * p3;
  pass_axis<T, true, true, P, 0>(A, dst, Sg, (bits >> 2) & 1, 6);
}

// Stabilised interpolation (Sec. 4.3): the least-squares projector Pm of the
// node values (symmetric, p x p) along the three axes of every cell of a
// level, in place, ncomp components per cell.  Applied to the multipole
// weights that enter the M2L and to the local values before they go to the
// children or the points.  One block per cell.
template <typename T, int P>
__global__ void k_project(T* data, int ncomp, const T* __restrict__ Pm) {
  extern __shared__ unsigned char shraw[];
  constexpr int p3 = P * P * P;
  T* A = (T*)shraw;
  T* B = A + ncomp * p3;
  T* src = data + (int64_t)blockIdx.x * ncomp * p3;
  for (int e = threadIdx.x; e < ncomp * p3; e += blockDim.x) A[e] = src[e];
  __syncthreads();
  pass_axis<T, false, false, P, 2>(A, B, Pm, 0, ncomp);
  __syncthreads();
  pass_axis<T, false, false, P, 1>(B, A, Pm, 0, ncomp);
  __syncthreads();
  pass_axis<T, false, false, P, 0>(A, src, Pm, 0, ncomp);
}

// Blocks are dispatched round-robin over the 8 XCDs; this bijection of
// [0, n) gives XCD x the contiguous range of items [x q + min(x, r), ...)
// (n = 8 q + r), so that items next to each other in memory meet in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t L, int64_t n) {
  const int64_t q = n / 8, r = n % 8, x = L % 8, k = L / 8;
  return x * q + (x < r ? x : r) + k;
}

// ------------------------------------------------- f16 scale of a level
// DFMM_MIXED_F16: the source spectra of a level are stored as f16 scaled by
// a power of two s_W, from the level's largest multipole weight m:
// |What| <= p^3 m (the forward DFT has unit-modulus twiddles), so s_W puts
// p^3 m in [2^13, 2^14), clear of f16's overflow; f16's relative precision
// does not depend on the scale.
__device__ __forceinline__ float h16_wscale(const unsigned* wmax, int p3) {
  const float m = __uint_as_float(*wmax) * (float)p3;
  if (!(m > 0.f) || !(m < 3.0e38f)) return 1.f;
  int e;
  frexpf(m, &e);
  return ldexpf(1.f, 14 - e);
}

// Largest |x| over the n floats of one level's weights into *out (float
// bits; non-negative floats order as unsigned integers): 16-byte loads over
// the aligned body (a level's weights start on a 4-byte boundary; the first
// block takes the unaligned head and the tail), one atomic per block.
__global__ void __launch_bounds__(256) k_wmax(const float* x, int64_t n, unsigned* out) {
  __shared__ float sh[256];
  int64_t head = (int64_t)(((16u - ((uintptr_t)x & 15u)) & 15u) / 4u);
  if (head > n) head = n;
  const int64_t nb4 = (n - head) / 4, tail0 = head + 4 * nb4;
  float m = 0.f;
  if (blockIdx.x == 0 && threadIdx.x < head) m = fabsf(x[threadIdx.x]);
  if (blockIdx.x == 0 && threadIdx.x < n - tail0) m = fmaxf(m, fabsf(x[tail0 + threadIdx.x]));
  const float4* x4 = reinterpret_cast<const float4*>(x + head);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nb4; i += (int64_t)gridDim.x * 256) {
    const float4 v = x4[i];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(sh[0]));
}

__global__ void k_fill_uint(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ uint32_t pack_h2(float re, float im) {
  const _Float16 a = (_Float16)re, b = (_Float16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// ------------------------------------------------------------ forward DFT
constexpr int kDftThreads = 512;  // threads per cell of a DFT block (at most 1024 a block)
// One block per cell of a level (or per CPB consecutive cells, below):
// W[cell][9][P^3] (real, zero-padded to n^3,
// n = 2P - 1) -> What[f][cell][9], f = (f1 n + f2) P + f3, the half spectrum
// in the last axis (the input is real).  Three passes of length-P to
// length-n (or P) DFTs, G components at a time.  A thread takes one input
// line of a pass, holds its P values in registers and produces all of the
// line's outputs, so each value is read once; the twiddles
// exp(-2 pi i k / n), k < n, are read once into (scalar) registers, and the
// fully unrolled loops index them with constants.  The first pass reads W
// straight from memory; the intermediate lines go through LDS.  Rows of
// neighbouring cells share cache lines, so cells are spread over the XCDs in
// contiguous ranges (xcd_block).
// One line of a complex pass, P inputs -> all n = 2P - 1 outputs.  Outputs f
// and n - f use conjugate twiddles, so with A = sum re(x) c, B = sum im(x) s,
// C = sum re(x) s and D = sum im(x) c, X[f] = (A - B, C + D) and
// X[n - f] = (A + B, D - C): four multiply-adds per input for two outputs.
// Output 0 is the plain sum.  put(f, value) stores output f.
template <typename T, int P, typename Put>
__device__ __forceinline__ void dft_line_pairs(const cplx<T>* x, const T* c, const T* s, Put put) {
  constexpr int n = 2 * P - 1;
  {
    T re = x[0].re, im = x[0].im;
#pragma unroll
    for (int m = 1; m < P; ++m) {
      re += x[m].re;
      im += x[m].im;
    }
    put(0, cplx<T>{re, im});
  }
#pragma unroll
  for (int f = 1; f < P; ++f) {
    T A = x[0].re, B = 0, C = 0, D = x[0].im;
#pragma unroll
    for (int m = 1; m < P; ++m) {
      const T cc = c[(f * m) % n], ss = s[(f * m) % n];
      A = fma(x[m].re, cc, A);
      B = fma(x[m].im, ss, B);
      C = fma(x[m].re, ss, C);
      D = fma(x[m].im, cc, D);
    }
    put(f, cplx<T>{A - B, C + D});
    put(n - f, cplx<T>{A + B, D - C});
  }
}

// Only the frequencies with first index f1 in [fa, fb) are stored, at f - fa n P
// (the spectrum in chunks along the first axis, for large trees).  A block
// takes CPB consecutive cells (512 threads per cell): the rows of one frequency
// of neighbouring cells are neighbours in What, so the last pass writes CPB
// rows in one piece.
template <typename T, int P, bool H16, int CPB>
__global__ void __launch_bounds__(kDftThreads * CPB) k_fdft(const T* __restrict__ W, int64_t ncell, int G,
                                                    const T* __restrict__ twg, cplx<T>* __restrict__ What,
                                                    const unsigned* __restrict__ wmax, int fa, int fb) {
  constexpr int n = 2 * P - 1, p3 = P * P * P;
  extern __shared__ __align__(16) unsigned char shraw[];
  cplx<T>* X1 = (cplx<T>*)shraw;       // [CPB][G][P][P][P]  (q, g, m1, m2, f3)
  cplx<T>* X2 = X1 + CPB * G * p3;     // [CPB][G][P][n][P]  (q, g, m1, f2, f3)
  T c[n], s[n];
#pragma unroll
  for (int k = 0; k < n; ++k) {
    c[k] = twg[2 * k];
    s[k] = twg[2 * k + 1];
  }
  const int64_t cell0 = CPB * xcd_block(blockIdx.x, (ncell + CPB - 1) / CPB);
  const int nq = (int)min<int64_t>(CPB, ncell - cell0);  // cells of this block
  const int L1 = G * P * P, L3 = G * n * P;           // lines per cell of passes 1-2 and 3
  for (int c0 = 0; c0 < 9; c0 += G) {
    // along the last axis: P real values -> P half-spectrum values
    for (int it = threadIdx.x; it < nq * L1; it += blockDim.x) {
      const int q = it / L1, l = it % L1;
      const T* src = W + ((cell0 + q) * 9 + c0) * p3 + l * P;
      T x[P];
#pragma unroll
      for (int m = 0; m < P; ++m) x[m] = src[m];
#pragma unroll
      for (int f = 0; f < P; ++f) {
        T re = 0, im = 0;
#pragma unroll
        for (int m = 0; m < P; ++m) {
          re = fma(x[m], c[(f * m) % n], re);
          im = fma(x[m], s[(f * m) % n], im);
        }
        X1[it * P + f] = cplx<T>{re, im};
      }
    }
    __syncthreads();
    // along the middle axis: P -> n
    for (int it = threadIdx.x; it < nq * L1; it += blockDim.x) {
      const int f3 = it % P, gm = it / P;  // gm = (q G + g) P + m1
      cplx<T> x[P];
#pragma unroll
      for (int m = 0; m < P; ++m) x[m] = X1[(gm * P + m) * P + f3];
      dft_line_pairs<T, P>(x, c, s, [&](int f, cplx<T> v) { X2[(gm * n + f) * P + f3] = v; });
    }
    __syncthreads();
    // along the first axis: P -> n, into What (the G components of a
    // frequency, then the cells, are neighbours in memory, so they are
    // neighbouring lanes)
    for (int it = threadIdx.x; it < nq * L3; it += blockDim.x) {
      const int g = it % G, q = (it / G) % nq, r = it / (G * nq);  // r = f2 P + f3
      const cplx<T>* x2 = X2 + (q * G + g) * P * n * P + r;
      const int64_t cell = cell0 + q;
      cplx<T> x[P];
#pragma unroll
      for (int m = 0; m < P; ++m) x[m] = x2[m * n * P];
      if constexpr (H16) {
        const float sw = h16_wscale(wmax, p3);
        uint32_t* W16 = reinterpret_cast<uint32_t*>(What);
        dft_line_pairs<T, P>(x, c, s, [&](int f, cplx<T> v) {
          if (f >= fa && f < fb)
            W16[((int64_t)((f - fa) * n * P + r) * ncell + cell) * 9 + c0 + g] =
                pack_h2((float)v.re * sw, (float)v.im * sw);
        });
      } else {
        dft_line_pairs<T, P>(x, c, s, [&](int f, cplx<T> v) {
          if (f >= fa && f < fb) What[((int64_t)((f - fa) * n * P + r) * ncell + cell) * 9 + c0 + g] = v;
        });
      }
    }
    __syncthreads();
  }
}

template <int P>
constexpr size_t lds_fdft_t(int G, size_t es) {
  return 2 * es * (size_t)G * (P * P * P + P * (2 * P - 1) * P);
}
// cells per block of the forward DFT: two where their LDS fits (G = 9)
template <typename T, int P>
constexpr int fdft_cpb() {
  return 2 * lds_fdft_t<P>(9, sizeof(T)) <= 160 * 1024 ? 2 : 1;
}

// ------------------------------------------------------ Hadamard product
// One block per (window of kM2LWindowF Morton-consecutive targets, frequency
// f).  The spectra of the 158 canonical offsets at frequency f sit in LDS;
// the spectrum of a mirrored offset -o is -conj of that of o, so its
// contribution -conj(K) w = -conj(K conj(w)) is folded into the same loop
// with a sign.  Two lanes share a target and walk its interaction list:
//   Shat[f][T][r] = sum_{(J, o) in I(T)} sum_k Khat_o(f)[r][k] What[f][J][k].
// The load of the source's nine values is one of the kernel's limits (with
// the LDS reads of the spectra and the multiply-adds), so the two lanes of a
// target split it: lane h loads components 4h..4h+3 and component 8 and
// multiplies only those (the split by component described with f_unit_of),
// and the two lanes exchange partial sums once per target.  The spectra are
// stored in the lanes' reading order, so the block's copy of them into LDS
// is a straight copy.  With many windows, blocks are remapped so that
// each of the 8 XCDs (blocks are dispatched round-robin over them) works
// through a contiguous range of windows at one frequency at a time:
// neighbouring windows share sources in that XCD's L2.
// The spectra take 73.3 KB of LDS per block, so two blocks (384 targets,
// twelve waves each) share a CU: six waves per SIMD.  (Splitting by component
// rather than by stress row, which removed the per-step exchange of four
// source values: 137 -> 127 VALU operations per lane and step, 202.5 ->
// 198.5 ms on 1M segments.)
// Symmetry-reduced store: one level's spectra of the 158 canonical offsets,
// expanded from the 16 class spectra Kc [nf][16][54] into the layout the
// Hadamard kernels read (the lanes' reading order: f_unit_of, d_unit_of,
// h16_word_of), in a workspace of the tree, before the level's product.
// With o = R o_c,
//   Khat_o(f)[a b w r] = det(R) s_a s_b s_w s_r Khat_{o_c}(R^T f)[pi(a) pi(b) pi(w) pi(r)],
// where (R^T f)_{pi(i)} = s_i f_i (mod n) and the half spectrum supplies g
// with g_3 >= p as the conjugate of -g.  One thread per (f, id, source
// entry), so a wave's loads run along the class spectrum's rows.
__device__ __constant__ const int kVoigtA[6] = {0, 1, 2, 1, 0, 0};
__device__ __constant__ const int kVoigtB[6] = {0, 1, 2, 2, 2, 1};
__device__ __constant__ const int kVoigtOf[9] = {0, 5, 4, 5, 1, 3, 4, 3, 2};
template <typename T, bool H16>
__global__ void k_sym_expand(const cplx<T>* __restrict__ Kc, const SymEntry* __restrict__ symtab, int nf, int n,
                             int p, float scale, cplx<T>* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nf * kNumCanon * 54) return;
  const int f = (int)(e / (kNumCanon * 54));
  const int rem = (int)(e - (int64_t)f * kNumCanon * 54), id = rem / 54, src = rem - 54 * id;
  const int fv[3] = {f / (n * p), (f / p) % n, f % p};
  const SymEntry se = symtab[id];
  int g[3], pinv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = se.sg[i] * fv[i];
    g[se.pi[i]] = t < 0 ? t + n : t;
    pinv[se.pi[i]] = i;
  }
  const bool cj = g[2] >= p;
  if (cj)
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = g[i] == 0 ? 0 : n - g[i];
  const int abs_ = src / 9, wrs = src - 9 * abs_;
  const int a = pinv[kVoigtA[abs_]], b = pinv[kVoigtB[abs_]], w = pinv[wrs / 3], r = pinv[wrs % 3];
  const int sgn = se.det * se.sg[a] * se.sg[b] * se.sg[w] * se.sg[r];
  const cplx<T> x = Kc[((int64_t)((g[0] * n + g[1]) * p + g[2]) * kNumSymClass + se.cls) * 54 + src];
  const cplx<T> v{sgn > 0 ? x.re : -x.re, (sgn > 0) != cj ? x.im : -x.im};
  const int ab = kVoigtOf[3 * a + b], wr = w * 3 + r;
  if (H16) {
    // all 316 offsets: slot 2 id holds o, slot 2 id + 1 holds -o (-conj)
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out);
    const int64_t e0 = ((int64_t)f * kNumOffsets + 2 * id) * kKOffsetH + h16_word_of(ab, wr);
    o32[e0] = pack_h2((float)v.re * scale, (float)v.im * scale);
    o32[e0 + kKOffsetH] = pack_h2(-(float)v.re * scale, (float)v.im * scale);
  } else if (sizeof(T) == 4)
    out[((int64_t)f * kNumCanon + id) * kKOffsetF + f_unit_of(ab, wr)] = v;
  else
    out[((int64_t)f * kNumCanon + id) * kKOffsetD + d_unit_of(ab, wr)] = v;
}

constexpr int kHadThreads = 2 * kM2LWindowF;
static_assert(kM2LWindowF % kWaveTargets == 0 && 2 * kWaveTargets == 64,
              "a wave holds kWaveTargets targets, two lanes each");
// Dynamic LDS of the M2L kernels: one frequency's spectra (f32: 158 offsets,
// f16: 316, double: 158).
constexpr int kHadLdsF = (int)sizeof(cplx<float>) * kNumCanon * kKOffsetF;
constexpr int kHadLdsH = (int)sizeof(uint32_t) * kNumOffsets * kKOffsetH;
constexpr int kHadLdsD = (int)sizeof(cplx<double>) * kNumCanon * kKOffsetD;
static_assert(2 * kHadLdsF <= 160 * 1024 && 2 * kHadLdsH <= 160 * 1024 && kHadLdsD <= 160 * 1024, "blocks per CU");

__global__ void __launch_bounds__(kHadThreads) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_hadamard(const cplx<float>* What, const cplx<float>* Khat, const int* lenq, const int* wbase, const uint32_t* ilw,
           const uint32_t* order, int64_t ncell, int nf, int nwin, int remap, cplx<float>* Shat) {
  extern __shared__ __align__(16) unsigned char shraw[];
  float4* Ks4 = (float4*)shraw;  // [158][2][kKHalfF] complex
  int win, f;
  if (remap) {
    const int64_t L = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int wx = (nwin + 7) / 8;
    const int xcd = (int)(L % 8);
    const int64_t k = L / 8;
    f = (int)(k / wx);
    win = xcd * wx + (int)(k % wx);
    if (win >= nwin || f >= nf) return;
  } else {
    win = blockIdx.x;
    f = blockIdx.y;
  }
  const float4* kf = reinterpret_cast<const float4*>(Khat + (int64_t)f * kNumCanon * kKOffsetF);
  for (int e = threadIdx.x; e < kNumCanon * kKOffsetF / 2; e += blockDim.x) Ks4[e] = kf[e];
  __syncthreads();
  // lane pair -> target: the 8 targets of an LDS pass are consecutive
  const int64_t tt = (int64_t)win * kM2LWindowF + (threadIdx.x >> 6) * kWaveTargets + pass_target((threadIdx.x & 63) >> 1);
  if (tt >= ncell) return;  // both lanes of a target leave together
  const int h = threadIdx.x & 1;
  const int64_t t = order[tt];
  const int len = lenq[tt];
  // accumulator a holds stress row (3h + a) mod 6
  float ar[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ai[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // A list entry is one 32-bit word: the source cell in bits 0..22, the
  // canonical offset in bits 23..30 and the mirror flag in bit 31 (the host
  // checks that a level's cells and its slice of the source spectra fit).  The
  // wave's 32 targets have their entries of one step side by side (one cache
  // line per load); halving the entries from 8 bytes was 1.6% faster, for one
  // more operation per step.  Loads take a uniform base and one offset
  // register.
  const char* wfb = reinterpret_cast<const char*>(What + (int64_t)f * ncell * 9);
  const char* ilb = reinterpret_cast<const char*>(ilw);
  constexpr uint32_t kStep = kWaveTargets * sizeof(uint32_t);  // bytes per step of a wave's block
  const char* kb = reinterpret_cast<const char*>(shraw) + h * (kKHalfF * 8);
  const uint32_t hoff = 32u * (uint32_t)h;
  auto entry = [&](uint32_t eb) { return *reinterpret_cast<const uint32_t*>(ilb + eb); };
  typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));
  auto load_src = [&](uint32_t j, cplx<float>* v) {
    const uint32_t o = (j & 0x7FFFFFu) * 72u;
    const f4a8 x = *reinterpret_cast<const f4a8*>(wfb + (o + hoff));
    const f4a8 y = *reinterpret_cast<const f4a8*>(wfb + (o + hoff) + 16);
    const float2 z = *reinterpret_cast<const float2*>(wfb + o + 64);
    v[0] = {x.x, x.y};
    v[1] = {x.z, x.w};
    v[2] = {y.x, y.y};
    v[3] = {y.z, y.w};
    v[4] = {z.x, z.y};
  };
  auto pair = [&](uint32_t j, const cplx<float>* v) {
    // a mirrored offset's spectrum is -conj(K) of the canonical K, and
    // -conj(K) w = Kr (-wr) - Ki wi + i (Ki wr + Kr (-wi)): the real parts of
    // K meet sign-flipped source values, with no fix-up per row
    const uint32_t sgb = j & 0x80000000u;
    float nr[5], ni[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      nr[c] = __uint_as_float(__float_as_uint(v[c].re) ^ sgb);
      ni[c] = __uint_as_float(__float_as_uint(v[c].im) ^ sgb);
    }
    // the lane's 27 complex spectrum entries: 13 float4 and one float2
    const float4* K4 = reinterpret_cast<const float4*>(kb + ((j >> 23) & 0xFFu) * (uint32_t)(kKOffsetF * 8));
    float kk[54];
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      const float4 q = K4[i];
      kk[4 * i] = q.x;
      kk[4 * i + 1] = q.y;
      kk[4 * i + 2] = q.z;
      kk[4 * i + 3] = q.w;
    }
    {
      const float2 q = reinterpret_cast<const float2*>(K4)[26];
      kk[52] = q.x;
      kk[53] = q.y;
    }
    // v[c]: component 4h + c (c < 4), component 8 (c = 4)
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
      for (int a = 0; a < (c < 4 ? 6 : 3); ++a) {
        const int e = c < 4 ? 4 * a + c : 24 + a;
        const float kr = kk[2 * e], ki = kk[2 * e + 1];
        ar[a] = fma(kr, nr[c], ar[a]);
        ar[a] = fma(-ki, v[c].im, ar[a]);
        ai[a] = fma(ki, v[c].re, ai[a]);
        ai[a] = fma(kr, ni[c], ai[a]);
      }
  };
  // The next list entry is loaded one step ahead (carried through an empty
  // asm statement, which keeps the compiler from turning it back into a load
  // at the top of the loop), so a step's source loads do not wait on its
  // index; the entry after a list's end is the zero padding of the wave's
  // block.  This needs few registers (76), which leaves room for six waves
  // per SIMD; prefetching the source values as well (two buffers, 105
  // registers, four waves per SIMD) was 4% slower.  The two lanes of a target
  // run the same iterations.
  if (len > 0) {
    uint32_t eb = kStep * (uint32_t)wbase[tt / kWaveTargets] + sizeof(uint32_t) * (uint32_t)(tt % kWaveTargets);
    uint32_t jo = entry(eb);
    for (int e = 0; e < len; ++e, eb += kStep) {
      const uint32_t jn = entry(eb + kStep);
      cplx<float> v[5];
      load_src(jo, v);
      pair(jo, v);
      jo = jn;
      asm volatile("" : "+v"(jo));
    }
  }
  // rows 3h..3h+2: accumulators 0..2 here, 3..5 in the partner lane (quad
  // permutation 1, 0, 3, 2)
  cplx<float>* out = Shat + ((int64_t)f * ncell + t) * 6 + 3 * h;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float pr = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(ar[3 + r]), 0xB1, 0xF, 0xF, false));
    const float pi = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(ai[3 + r]), 0xB1, 0xF, 0xF, false));
    out[r] = cplx<float>{ar[r] + pr, ai[r] + pi};
  }
}

// The Hadamard product on f16 operands (DFMM_MIXED_F16): the same blocks,
// list walk and source loads as k_hadamard, with every complex value a pair
// of f16 (real in the low half) and the products done by v_dot2_f32_f16, two
// multiply-adds with f32 accumulation per instruction:
//   K w:  re = (kr, ki).(wr, -wi),  im = (kr, ki).(wi, wr),
// the sign of the real part's product taken by the instruction's neg_hi
// modifier and the imaginary part's operand half-swapped once per pair.  A
// lane multiplies only the five source components it loads (h16_word_of):
// the two lanes of a target exchange their partial sums once, after the
// list, instead of source values at every step.
// LDS holds the spectra of all 316 offsets (the mirrored offset -o as -conj
// of o), so there is no per-pair mirror handling; a list entry's bits 23..31
// are the offset's slot 2 id + mirror.  The spectra take 74 KB of LDS per
// frequency (two blocks per CU, as for the f32 product) and a source row 36
// bytes.  Operator and source spectra carry power-of-two scales that the
// inverse DFT removes.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(kHadThreads) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_hadamard16(const uint32_t* What, const uint32_t* Khat, const int* lenq, const int* wbase, const uint32_t* ilw,
             const uint32_t* order, int64_t ncell, int nf, int nwin, int remap, cplx<float>* Shat) {
  extern __shared__ __align__(16) unsigned char shraw[];
  uint4* Ks4 = (uint4*)shraw;  // [316][15] 16-byte units
  int win, f;
  if (remap) {
    const int64_t L = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int wx = (nwin + 7) / 8;
    const int xcd = (int)(L % 8);
    const int64_t k = L / 8;
    f = (int)(k / wx);
    win = xcd * wx + (int)(k % wx);
    if (win >= nwin || f >= nf) return;
  } else {
    win = blockIdx.x;
    f = blockIdx.y;
  }
  const uint4* kf = reinterpret_cast<const uint4*>(Khat + (int64_t)f * kNumOffsets * kKOffsetH);
  for (int e = threadIdx.x; e < kNumOffsets * kKOffsetH / 4; e += blockDim.x) Ks4[e] = kf[e];
  __syncthreads();
  // lane pair -> target: the 8 targets of an LDS pass are consecutive
  const int64_t tt = (int64_t)win * kM2LWindowF + (threadIdx.x >> 6) * kWaveTargets + pass_target((threadIdx.x & 63) >> 1);
  if (tt >= ncell) return;  // both lanes of a target leave together
  const int h = threadIdx.x & 1;
  const int64_t t = order[tt];
  const int len = lenq[tt];
  // accumulator a holds stress row (3h + a) mod 6
  float ar[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ai[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const char* wfb = reinterpret_cast<const char*>(What + (int64_t)f * ncell * 9);
  const char* ilb = reinterpret_cast<const char*>(ilw);
  constexpr uint32_t kStep = kWaveTargets * sizeof(uint32_t);
  const char* kb = reinterpret_cast<const char*>(shraw) + h * (kKHalfH * 4);
  const uint32_t hoff = 16u * (uint32_t)h;
  auto entry = [&](uint32_t eb) { return *reinterpret_cast<const uint32_t*>(ilb + eb); };
  typedef unsigned u4a4 __attribute__((ext_vector_type(4), aligned(4)));
  // lane h: components 4h..4h+3 and 8 of the 36-byte source row
  auto load_src = [&](uint32_t j, uint32_t* v) {
    const uint32_t o = (j & 0x7FFFFFu) * 36u;
    const u4a4 x = *reinterpret_cast<const u4a4*>(wfb + (o + hoff));
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
    v[4] = *reinterpret_cast<const uint32_t*>(wfb + o + 32);
  };
  auto pair = [&](uint32_t j, const uint32_t* v) {
    const uint4* K4 = reinterpret_cast<const uint4*>(kb + (j >> 23) * (uint32_t)(kKOffsetH * 4));
    uint32_t kk[28];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const uint4 x = K4[i];
      kk[4 * i] = x.x;
      kk[4 * i + 1] = x.y;
      kk[4 * i + 2] = x.z;
      kk[4 * i + 3] = x.w;
    }
    // v[c]: component 4h + c (c < 4), component 8 (c = 4)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const half2v q = __builtin_bit_cast(half2v, __builtin_amdgcn_alignbit(v[c], v[c], 16));  // (wi, wr)
#pragma unroll
      for (int a = 0; a < (c < 4 ? 6 : 3); ++a) {
        const uint32_t kv = c < 4 ? kk[4 * a + c] : kk[24 + a];
        // re: (kr, ki).(wr, -wi), the sign taken by the instruction's neg_hi
        // modifier on the source operand
        asm("v_dot2_f32_f16 %0, %1, %2, %0 neg_hi:[0,1,0]" : "+v"(ar[a]) : "v"(kv), "v"(v[c]));
        ai[a] = __builtin_amdgcn_fdot2(__builtin_bit_cast(half2v, kv), q, ai[a], false);
      }
    }
  };
  // A step's source values are loaded one step ahead and its list entry two
  // steps ahead (the entries after a list's end are the zero padding of the
  // wave's block, kIlwPad steps), so neither load waits at its use; two steps
  // per iteration alternate between two source buffers.
  if (len > 0) {
    uint32_t eb = kStep * (uint32_t)wbase[tt / kWaveTargets] + sizeof(uint32_t) * (uint32_t)(tt % kWaveTargets);
    uint32_t jo = entry(eb), jn = entry(eb + kStep);
    uint32_t va[5], vb[5];
    load_src(jo, va);
    int e = 0;
    for (; e + 1 < len; e += 2, eb += 2 * kStep) {
      const uint32_t j2 = entry(eb + 2 * kStep);
      load_src(jn, vb);
      pair(jo, va);
      const uint32_t j3 = entry(eb + 3 * kStep);
      load_src(j2, va);
      pair(jn, vb);
      jo = j2;
      jn = j3;
      asm volatile("" : "+v"(jn));
    }
    if (e < len) pair(jo, va);
  }
  // rows 3h..3h+2: accumulators 0..2 here, 3..5 in the partner lane (quad
  // permutation 1, 0, 3, 2)
  cplx<float>* out = Shat + ((int64_t)f * ncell + t) * 6 + 3 * h;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float pr = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(ar[3 + r]), 0xB1, 0xF, 0xF, false));
    const float pi = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(ai[3 + r]), 0xB1, 0xF, 0xF, false));
    out[r] = cplx<float>{ar[r] + pr, ai[r] + pi};
  }
}

// The double-precision Hadamard product: the blocks, list walk and source
// loads of k_hadamard, with one 16-byte complex per LDS unit, and the 6x9
// product split between a target's two lanes by source component as in
// k_hadamard16 (d_unit_of): no source value crosses lanes, and the partial
// sums of the rows a lane writes are exchanged once per target.  The spectra
// of a frequency are stored in the lanes' reading order (lane h's 27 values of
// offset c at unit 55 c + 27 h), and a block copies them into LDS as they
// are: 139 KB, so one block of 1024 threads (four waves per SIMD) runs per
// CU.  Per step a lane reads 27 complex spectrum values (432 B of LDS) for
// 108 double multiply-adds.  (Reading one of the three rows from memory
// instead, to share the load between LDS and L2, made the kernel 2.5 times
// slower: the rows are 144-byte reads at random offsets.)  The LDS allows
// four waves per SIMD, and the kernel says so (amdgpu_waves_per_eu): left to
// target eight, the compiler fits it into 64 registers by issuing its 27
// spectrum reads one at a time, each waited for before its multiply-adds
// (455 -> 375 ms on 1M segments).
constexpr int kHadThreadsD = 2 * kM2LWindowD;
static_assert(kM2LWindowD % kWaveTargets == 0, "whole waves per window");
__global__ void __launch_bounds__(kHadThreadsD) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_hadamard64(const cplx<double>* What, const cplx<double>* Khat, const int* lenq, const int* wbase, const uint32_t* ilw,
             const uint32_t* order, int64_t ncell, int nf, int nwin, int remap, cplx<double>* Shat) {
  extern __shared__ __align__(16) unsigned char shraw[];
  cplx<double>* Ks = (cplx<double>*)shraw;  // [158][kKOffsetD]
  int win, f;
  if (remap) {
    const int64_t L = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int wx = (nwin + 7) / 8;
    const int xcd = (int)(L % 8);
    const int64_t k = L / 8;
    f = (int)(k / wx);
    win = xcd * wx + (int)(k % wx);
    if (win >= nwin || f >= nf) return;
  } else {
    win = blockIdx.x;
    f = blockIdx.y;
  }
  const double2* kf = reinterpret_cast<const double2*>(Khat + (int64_t)f * kNumCanon * kKOffsetD);
  double2* Ks2 = reinterpret_cast<double2*>(Ks);
  for (int e = threadIdx.x; e < kNumCanon * kKOffsetD; e += blockDim.x) Ks2[e] = kf[e];
  __syncthreads();
  // lane pair -> target: the 8 targets of an LDS pass are consecutive
  const int64_t tt = (int64_t)win * kM2LWindowD + (threadIdx.x >> 6) * kWaveTargets + pass_target((threadIdx.x & 63) >> 1);
  if (tt >= ncell) return;  // both lanes of a target leave together
  const int h = threadIdx.x & 1;
  const int64_t t = order[tt];
  const int len = lenq[tt];
  // accumulator a holds stress row (3h + a) mod 6
  double ar[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, ai[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // list entries as in k_hadamard: source cell in bits 0..22, canonical
  // offset in bits 23..30, mirror flag in bit 31
  const char* wfb = reinterpret_cast<const char*>(What + (int64_t)f * ncell * 9);
  const char* ilb = reinterpret_cast<const char*>(ilw);
  constexpr uint32_t kStep = kWaveTargets * sizeof(uint32_t);
  const cplx<double>* kb = Ks + h * kKHalfD;
  const uint32_t hoff = 64u * (uint32_t)h;
  auto entry = [&](uint32_t eb) { return *reinterpret_cast<const uint32_t*>(ilb + eb); };
  auto load_src = [&](uint32_t j, double2* v) {
    // components 4h..4h+3 and 8 of the source row (144 bytes)
    const uint32_t o = (j & 0x7FFFFFu) * 144u;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const double2*>(wfb + (o + hoff) + 16 * k);
    v[4] = *reinterpret_cast<const double2*>(wfb + o + 128);
  };
  auto pair = [&](uint32_t j, const double2* v) {
    // a mirrored offset's spectrum is -conj(K) of the canonical K, and
    // -conj(K) w = Kr (-wr) - Ki wi + i (Ki wr + Kr (-wi)): the real parts of
    // K meet sign-flipped source values, with no fix-up per row
    const int sgb = (int)(j & 0x80000000u);
    double nr[5], ni[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      nr[c] = __hiloint2double(__double2hiint(v[c].x) ^ sgb, __double2loint(v[c].x));
      ni[c] = __hiloint2double(__double2hiint(v[c].y) ^ sgb, __double2loint(v[c].y));
    }
    const cplx<double>* K = kb + ((j >> 23) & 0xFFu) * (uint32_t)kKOffsetD;
    // v[c]: component 4h + c (c < 4), component 8 (c = 4)
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
      for (int a = 0; a < (c < 4 ? 6 : 3); ++a) {
        const double2 q = *reinterpret_cast<const double2*>(K + (c < 4 ? 4 * a + c : 24 + a));
        ar[a] = fma(q.x, nr[c], ar[a]);
        ar[a] = fma(-q.y, v[c].y, ar[a]);
        ai[a] = fma(q.y, v[c].x, ai[a]);
        ai[a] = fma(q.x, ni[c], ai[a]);
      }
  };
  // next entry one step ahead, as in k_hadamard (prefetching the source
  // values too, as k_hadamard16 does, was 2% slower here: this kernel is
  // bound by its LDS reads); the two lanes of a target run the same
  // iterations
  if (len > 0) {
    uint32_t eb = kStep * (uint32_t)wbase[tt / kWaveTargets] + sizeof(uint32_t) * (uint32_t)(tt % kWaveTargets);
    uint32_t jo = entry(eb);
    for (int e = 0; e < len; ++e, eb += kStep) {
      const uint32_t jn = entry(eb + kStep);
      double2 v[5];
      load_src(jo, v);
      pair(jo, v);
      jo = jn;
      asm volatile("" : "+v"(jo));
    }
  }
  // rows 3h..3h+2: accumulators 0..2 here, 3..5 in the partner lane (quad
  // permutation 1, 0, 3, 2)
  auto partner = [](double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
  };
  cplx<double>* out = Shat + ((int64_t)f * ncell + t) * 6 + 3 * h;
#pragma unroll
  for (int r = 0; r < 3; ++r) out[r] = cplx<double>{ar[r] + partner(ar[3 + r]), ai[r] + partner(ai[3 + r])};
}

// ------------------------------------------------------------ inverse DFT
// One line of an inverse complex pass, n = 2P - 1 inputs -> the first P
// outputs, with twiddles c + i sn = exp(+2 pi i k / n).  Inputs f and n - f
// have conjugate twiddles, so they enter as u = x[f] + x[n - f] (times c) and
// v = x[f] - x[n - f] (times i sn): four multiply-adds per input pair and
// output.  put(l, value) stores output l.
template <typename T, int P, typename Put>
__device__ __forceinline__ void idft_line_pairs(const cplx<T>* x, const T* c, const T* sn, Put put) {
  constexpr int n = 2 * P - 1;
  cplx<T> u[P], v[P];
#pragma unroll
  for (int f = 1; f < P; ++f) {
    u[f] = cplx<T>{x[f].re + x[n - f].re, x[f].im + x[n - f].im};
    v[f] = cplx<T>{x[f].re - x[n - f].re, x[f].im - x[n - f].im};
  }
#pragma unroll
  for (int l = 0; l < P; ++l) {
    T re = x[0].re, im = x[0].im;
#pragma unroll
    for (int f = 1; f < P; ++f) {
      const T cc = c[(f * l) % n], ss = sn[(f * l) % n];
      re = fma(u[f].re, cc, fma(-v[f].im, ss, re));
      im = fma(u[f].im, cc, fma(v[f].re, ss, im));
    }
    put(l, cplx<T>{re, im});
  }
}

// One block per CPB consecutive cells (1024 threads when CPB > 1), whose
// rows of one frequency the first pass reads in one piece:
// Shat[f][cell][6] -> s[cell][6][P^3] (overwrites): the
// inverse transform of the half spectrum of a real circular convolution, of
// which only the outputs l < P are needed (the rest is the wrap-around of the
// embedding).  As in the forward transform, a thread takes one line of a
// pass in registers and produces all of its P outputs, with the twiddles
// exp(+2 pi i k / n) in scalar registers.  The first pass reads the spectrum
// straight from memory, each value once: a cell's 48-byte row at each
// frequency, with cells spread over the XCDs in contiguous ranges so that
// neighbouring cells' rows meet in one L2 (the frequency-major layout makes
// the Hadamard product's stores land together, which gains more than these
// reads cost).  The last pass uses the Hermitian symmetry of the last axis
// (f3 = 0 once, f3 > 0 twice, real part).
template <typename T, int P, int CPB>
__global__ void __launch_bounds__(CPB > 1 ? 1024 : kDftThreads) k_idft(const cplx<T>* __restrict__ Shat, int64_t ncell,
                                                    const T* __restrict__ twg, T* __restrict__ s,
                                                    const unsigned* __restrict__ wmax, float kscale, int fa, int fb,
                                                    int acc_out) {
  constexpr int n = 2 * P - 1, p3 = P * P * P, nf = n * n * P;
  extern __shared__ __align__(16) unsigned char shraw[];
  cplx<T>* Y1 = (cplx<T>*)shraw;           // [CPB][6][n(f2)][P(f3)][P(l1)]
  cplx<T>* Y2 = Y1 + CPB * 6 * n * P * P;  // [CPB][6][P(f3)][P(l1)][P(l2)]
  T c[n], sn[n];  // exp(+2 pi i k / n) = c[k] + i sn[k]
#pragma unroll
  for (int k = 0; k < n; ++k) {
    c[k] = twg[2 * k];
    sn[k] = -twg[2 * k + 1];
  }
  const int64_t cell0 = CPB * xcd_block(blockIdx.x, (ncell + CPB - 1) / CPB);
  const int nq = (int)min<int64_t>(CPB, ncell - cell0);  // cells of this block
  // the f16 product's spectra carry the operator and source scales
  const T scale = wmax ? T(1) / (T(n * n * n) * (T)kscale * (T)h16_wscale(wmax, p3)) : T(1) / T(n * n * n);
  const cplx<T>* src = Shat + cell0 * 6;
  // along the first axis: n -> P (lanes over component, then cell, then
  // line: the rows of one frequency of neighbouring cells are neighbours)
  for (int it = threadIdx.x; it < nq * 6 * n * P; it += blockDim.x) {
    const int g = it % 6, q = (it / 6) % nq, r = it / (6 * nq);  // r = f2 P + f3
    cplx<T> x[n];
#pragma unroll
    for (int f = 0; f < n; ++f)
      x[f] = (f >= fa && f < fb) ? src[(int64_t)((f - fa) * n * P + r) * ncell * 6 + 6 * q + g]
                                 : cplx<T>{T(0), T(0)};
    idft_line_pairs<T, P>(x, c, sn, [&](int l, cplx<T> v) { Y1[((q * 6 + g) * n * P + r) * P + l] = v; });
  }
  __syncthreads();
  // along the middle axis: n -> P
  for (int it = threadIdx.x; it < nq * 6 * P * P; it += blockDim.x) {
    const int l1 = it % P, f3 = (it / P) % P, g = it / (P * P);  // g = q 6 + component
    cplx<T> x[n];
#pragma unroll
    for (int f = 0; f < n; ++f) x[f] = Y1[((g * n + f) * P + f3) * P + l1];
    idft_line_pairs<T, P>(x, c, sn, [&](int l, cplx<T> v) { Y2[((g * P + f3) * P + l1) * P + l] = v; });
  }
  __syncthreads();
  // along the last axis: half spectrum (P) -> P real outputs
  for (int it = threadIdx.x; it < nq * 6 * P * P; it += blockDim.x) {
    const int l2 = it % P, l1 = (it / P) % P, g = it / (P * P);  // g = q 6 + component
    cplx<T> x[P];
#pragma unroll
    for (int f = 0; f < P; ++f) x[f] = Y2[((g * P + f) * P + l1) * P + l2];
    T* out = s + (cell0 * 6 + g) * p3 + (l1 * P + l2) * P;
#pragma unroll
    for (int l = 0; l < P; ++l) {
      T acc = 0;
#pragma unroll
      for (int f = 1; f < P; ++f) acc = fma(x[f].re, c[(f * l) % n], fma(-x[f].im, sn[(f * l) % n], acc));
      const T v = (x[0].re + T(2) * acc) * scale;
      out[l] = acc_out ? out[l] + v : v;
    }
  }
}

template <int P>
constexpr size_t lds_idft_t(size_t es) {
  return 2 * es * ((size_t)6 * (2 * P - 1) * P * P + (size_t)6 * P * P * P);
}
// cells per block of the inverse DFT (1024 threads for more than one): three
// at the larger orders where their LDS fits, else two where that fits
template <typename T, int P>
constexpr int idft_cpb() {
  return P >= 6 && 3 * lds_idft_t<P>(sizeof(T)) <= 160 * 1024 ? 3 : 2 * lds_idft_t<P>(sizeof(T)) <= 160 * 1024 ? 2 : 1;
}

// ------------------------------------------------ near field + L2P (leaf)
// Near field.  One wave per leaf.  With nt <= 64 targets, S = 64/nt (rounded down to a
// power of two) lanes share a target and split its sources; partial sums are
// combined with xor shuffles.  In MIXED precision pairs are evaluated in float
// (displacements formed in double) with compensated float accumulation, and
// pairs closer than 2a are left to k_close_eval (double precision, run after this
// kernel), which keeps double-precision code and its registers out of here.
__device__ __forceinline__ void kadd_f(float& s, float& c, float x) {
  const float y = x - c;
  const float z = s + y;
  c = (z - s) - y;
  s = z;
}

// Single precision: ask for 3 waves per SIMD (the register budget that the
// pair evaluation fits without spilling); double precision: no constraint.
template <typename T>
constexpr int leaf_min_waves() {
  return std::is_same<T, float>::value ? 3 : 1;
}

template <typename T, bool MIXED, bool ISO>
__global__ void __launch_bounds__(64, leaf_min_waves<T>())
    k_leaf(const double* pts, int64_t N, const int* first, const int* count, const int* nbr, Med<T> m,
           Med<double> m64, double* sig) {
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int t0 = first[leaf], nt = count[leaf];
  __shared__ int nb_first[27], nb_cnt[27];
  if (lane < 27) {
    int j = nbr[(int64_t)leaf * 27 + lane];
    nb_first[lane] = j >= 0 ? first[j] : 0;
    nb_cnt[lane] = j >= 0 ? count[j] : 0;
  }
  __syncthreads();
  const double a2x4 = 4.0 * m64.a * m64.a;
  // Passes over the leaf's targets: 64 at a time with one lane each, then the
  // remainder in power-of-two chunks c with S = 64/c lanes per target, so
  // every pass keeps all 64 lanes busy.
  for (int c0 = 0, per = 64; c0 < nt; c0 += per) {
    const int rem = nt - c0;
    per = 64;
    while (per > rem) per >>= 1;
    const int S = 64 / per;
    const int ti = c0 + lane / S, slice = lane % S;
    const bool act = ti < nt;
    const int64_t i = t0 + (act ? ti : 0);
    const double xt0 = pts[i], xt1 = pts[N + i], xt2 = pts[2 * N + i];
    T acc[6], cmp[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = cmp[c] = T(0);
    int base = 0;
    for (int q = 0; q < 27; ++q) {
      const int fj = nb_first[q], cj = nb_cnt[q];
      if (act) {
        int jj = (slice - (base % S) + S) % S;
        for (; jj < cj; jj += S) {
          const int64_t j = fj + jj;
          double d0 = xt0 - pts[j], d1 = xt1 - pts[N + j], d2 = xt2 - pts[2 * N + j];
          if (MIXED && d0 * d0 + d1 * d1 + d2 * d2 < a2x4) {
            // nearly coincident pair: evaluated by k_close_eval
          } else {
            T D[27], b[3], tt[3];
            for (int c = 0; c < 3; ++c) b[c] = (T)pts[(3 + c) * N + j], tt[c] = (T)pts[(6 + c) * N + j];
            dg_medium_t<T, ISO>((T)d0, (T)d1, (T)d2, m, D);
            if (MIXED) {
              T ds[6] = {0, 0, 0, 0, 0, 0};
              contract_b_t<T>(D, m.c12, m.c44, m.hh, b, tt, ds);
#pragma unroll
              for (int c = 0; c < 6; ++c) {  // Kahan-compensated accumulation
                T y = ds[c] - cmp[c];
                T z = acc[c] + y;
                cmp[c] = (z - acc[c]) - y;
                acc[c] = z;
              }
            } else {
              contract_b_t<T>(D, m.c12, m.c44, m.hh, b, tt, acc);
            }
          }
        }
      }
      base += cj;
    }
    double tot[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tot[c] = (double)acc[c] - (double)cmp[c];
    for (int o = S / 2; o >= 1; o >>= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) tot[c] += __shfl_xor(tot[c], o, 64);
    if (act && slice == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sig[i * 6 + c] = tot[c];
    }
  }
}

// Near field with the learned surrogate (cubic medium, single precision):
// the one-sided pair loop of k_leaf, with the anisotropic part of dG taken
// from the network wherever the pair's direction bin passed the residual
// gate.  The network runs on the matrix cores for all 64 pairs of a wave at
// once (mlp_eval.h), so the loops are arranged to be uniform across the wave:
// one wave per leaf (persistent blocks of eight waves, leaves strided over
// the grid), each lane walking its target's sources in the order k_leaf
// uses, one source per lane and step.  A step evaluates the network when any
// lane's pair is gated in; lanes whose pair is not keep the exact quadrature.
// The weights sit in LDS (110 KB), one block per CU.
constexpr int kSurLeafThreads = 512;
__global__ void __launch_bounds__(kSurLeafThreads) k_leaf_sur(const double* pts, int64_t N, const int* first,
                                                              const int* count, const int* nbr, int64_t nleaf,
                                                              Med<float> m, Med<double> m64, SurDev sd, double* sig) {
  extern __shared__ __align__(16) unsigned char lds[];
  sur_stage(sd, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t nw = kSurLeafThreads / 64;
  const int64_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const double a2x4 = 4.0 * m64.a * m64.a;
  const float fscale = sd.yscale / m.c44;
  for (int64_t leaf = (int64_t)blockIdx.x * nw + wave; leaf < nleaf; leaf += (int64_t)gridDim.x * nw) {
    const int t0 = first[leaf], nt = count[leaf];
    for (int c0 = 0, per = 64; c0 < nt; c0 += per) {
      const int rem = nt - c0;
      per = 64;
      while (per > rem) per >>= 1;
      const int S = 64 / per;
      const int ti = c0 + lane / S, slice = lane % S;
      const bool act = ti < nt;
      const int64_t i = t0 + (act ? ti : 0);
      const double xt0 = pts[i], xt1 = pts[N + i], xt2 = pts[2 * N + i];
      float acc[6], cmp[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] = cmp[c] = 0.f;
      int base = 0;
      for (int q = 0; q < 27; ++q) {
        const int jl = nbr[leaf * 27 + q];
        const int fj = jl >= 0 ? first[jl] : 0, cj = jl >= 0 ? count[jl] : 0;
        const int start = (slice - (base % S) + S) % S;
        const int nsteps = (cj + S - 1) / S;  // the same on every lane
        for (int it = 0; it < nsteps; ++it) {
          const int jj = start + it * S;
          bool use = act && jj < cj;
          double d0 = 0, d1 = 0, d2 = 0;
          int64_t j = 0;
          if (use) {
            j = fj + jj;
            d0 = xt0 - pts[j];
            d1 = xt1 - pts[N + j];
            d2 = xt2 - pts[2 * N + j];
            if (d0 * d0 + d1 * d1 + d2 * d2 < a2x4) use = false;  // near-coincident: k_close_eval
          }
          const float f0 = (float)d0, f1 = (float)d1, f2 = (float)d2;
          const float rr = f0 * f0 + f1 * f1 + f2 * f2;
          float x6[6] = {1.f, 0.f, 0.f, sd.ft.f[0], sd.ft.f[1], sd.ft.f[2]};
          bool gated = false;
          if (use && rr > 0.f) {
            const float ir = rsqrtf(rr);
            x6[0] = f0 * ir;
            x6[1] = f1 * ir;
            x6[2] = f2 * ir;
            gated = sd.mask[sur_bin(x6, sd.bins)] != 0;
          }
          float D[27];
          if (__ballot(gated)) {
            float y[18];
            sur_wave_eval(lds, x6, y);
            // the network's part first, so that its outputs die before the
            // exact quadrature of the other lanes
            if (gated) {
#pragma unroll
              for (int c = 0; c < 27; ++c) D[c] = 0.f;
              dg_iso_acc<float>(f0, f1, f2, m.mu, m.nu, m.a, 1.f, D);
              const float qd = rr / (rr + m.a * m.a);
              sur_aniso_add<float>(y, qd * sqrtf(qd) * fscale / rr, D);
            }
          }
          if (use) {
            float b[3], tt[3];
            if (!gated) dg_medium_t<float, false>(f0, f1, f2, m, D);
            for (int c = 0; c < 3; ++c) b[c] = (float)pts[(3 + c) * N + j], tt[c] = (float)pts[(6 + c) * N + j];
            float ds[6] = {0, 0, 0, 0, 0, 0};
            contract_b_t<float>(D, m.c12, m.c44, m.hh, b, tt, ds);
#pragma unroll
            for (int c = 0; c < 6; ++c) kadd_f(acc[c], cmp[c], ds[c]);
          }
        }
        base += cj;
      }
      double tot[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) tot[c] = (double)acc[c] - (double)cmp[c];
      for (int o = S / 2; o >= 1; o >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) tot[c] += __shfl_xor(tot[c], o, 64);
      if (act && slice == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) sig[i * 6 + c] = tot[c];
      }
    }
  }
}

// Symmetric near field (cubic medium; single precision, and double precision
// in the FP64 path, where no pair is left out).  The kernel's
// derivative is odd, dG(-x) = -dG(x), so one evaluation per unordered pair of
// points serves both directions: sigma_i += K(x_i - x_j) q_j and
// sigma_j += K(x_j - x_i) q_i = -(the contraction of the same dG with q_i).
// One block per unordered pair of neighbouring leaves {A, B}: B = A + o with
// o the neighbour offsets q = 13..26 (q = 13: the leaf with itself, pairs
// i < j).  Thread = point pair (i in A, j in B), one wave per block, or four
// for leaves of more than 64 points in single precision; in single precision,
// pairs closer than 2a are left to k_close_eval.  Each round of pairs is
// reduced in LDS in a fixed order (a target of A sums its consecutive pairs,
// a target of B its pairs in order of i) into compensated sums, and the block writes one partial
// per (target, neighbour slot): slot q for the targets of A, slot 26 - q (the
// offset of A seen from B) for those of B.  k_near_sum then adds a target's
// 27 slots in slot order, so every sum has a fixed order.
template <typename T>
__device__ __forceinline__ void kadd(T& s, T& c, T x) {
  const T y = x - c;
  const T z = s + y;
  c = (z - s) - y;
  s = z;
}

// BIG = false takes the leaf pairs with at most 64 points on each side (LDS
// for 64 accumulators per side, so LDS does not limit occupancy); BIG = true
// takes the others, with accumulators for the largest leaf (lmax).
// Threads of a block: leaf pairs with more than 64 points on a side take
// rounds of 256 point pairs (four waves share one set of LDS sums, which
// would otherwise limit a CU to two waves per SIMD in single precision, and
// to about one wave per CU in FP64), 64 else.  Single-precision sums are
// compensated; FP64 ones are plain (no compensation arrays: 12 FP64 values
// of LDS per point where 24 left large leaves one block per CU).
template <typename T, bool BIG>
constexpr int sym_threads() {
  return BIG ? 256 : 64;
}

template <typename T>
constexpr int sym_min_waves() {
  return 3;
}

template <typename T, bool MIXED, bool BIG>
__global__ void __launch_bounds__((sym_threads<T, BIG>()), sym_min_waves<T>())
    k_leaf_sym(const double* pts, int64_t N, const int* first, const int* count, const int* nbr, Med<T> m,
               double a2x4, int lmax, T* part, const int* bigp) {
  constexpr int NT = sym_threads<T, BIG>();  // threads = point pairs per round
  extern __shared__ __align__(16) unsigned char symraw[];
  T* symsh = reinterpret_cast<T*>(symraw);
  // small leaves: grid (leaves, 14); large: one block per listed pair
  const int A = BIG ? bigp[blockIdx.x] / 14 : (int)blockIdx.x;
  const int q = 13 + (BIG ? bigp[blockIdx.x] % 14 : (int)blockIdx.y), lane = threadIdx.x;
  const int B = nbr[(int64_t)A * 27 + q];
  if (B < 0) return;
  const bool self = q == 13;
  const int fa = first[A], na = count[A], fb = first[B], nb = count[B];
  if ((na > 64 || nb > 64) != BIG) return;
  if (!BIG) lmax = 64;
  constexpr bool KC = sizeof(T) == 4;  // compensated sums
  T* accA = symsh;                      // [lmax][6]
  T* cmpA = accA + (KC ? lmax * 6 : 0);  // [lmax][6] (single precision)
  T* accB = cmpA + lmax * 6;
  T* cmpB = accB + (KC ? lmax * 6 : 0);
  T* vij = cmpB + lmax * 6;             // [NT][6] contributions to A's targets
  T* vji = vij + NT * 6;                // [NT][6] contributions to B's targets
  auto cmp_of = [&](const T* c, int w) -> double {
    if constexpr (KC) return (double)c[w];
    else return 0.0;
  };
  auto add = [&](T& s, T& c, T x) {
    if constexpr (KC) kadd(s, c, x);
    else s += x;
  };
  for (int e = lane; e < lmax * 6; e += NT) {
    accA[e] = accB[e] = T(0);
    if constexpr (KC) cmpA[e] = cmpB[e] = T(0);
  }
  __syncthreads();
  // With the leaf itself only the pairs i < j are enumerated, row by row:
  // row i holds (i, i+1 .. na-1) and starts at pair row0(i).
  const int npair = self ? na * (na - 1) / 2 : na * nb;
  auto row0 = [&](int i) { return i * na - i * (i + 1) / 2; };
  int ic = 0, rlo = 0, rhi = 0;  // this lane's row; rows of the round's first and last pair
  for (int p0 = 0; p0 < npair; p0 += NT) {
    const int p = p0 + lane;
    int i, j;
    if (self) {
      while (ic + 1 < na && row0(ic + 1) <= p) ++ic;
      while (rlo + 1 < na && row0(rlo + 1) <= p0) ++rlo;
      const int plast = min(p0 + NT - 1, npair - 1);
      while (rhi + 1 < na && row0(rhi + 1) <= plast) ++rhi;
      i = ic;
      j = i + 1 + (p - row0(i));
    } else {
      i = p / nb;
      j = p - i * nb;
    }
    T fi[6] = {0, 0, 0, 0, 0, 0}, fj[6] = {0, 0, 0, 0, 0, 0};
    if (p < npair) {
      const int64_t gi = fa + i, gj = fb + j;
      const double d0 = pts[gi] - pts[gj], d1 = pts[N + gi] - pts[N + gj], d2 = pts[2 * N + gi] - pts[2 * N + gj];
      if (!MIXED || d0 * d0 + d1 * d1 + d2 * d2 >= a2x4) {
        T D[27], bj[3], tj[3], bi[3], ti[3];
        for (int c = 0; c < 3; ++c) {
          bj[c] = (T)pts[(3 + c) * N + gj], tj[c] = (T)pts[(6 + c) * N + gj];
          bi[c] = (T)pts[(3 + c) * N + gi], ti[c] = (T)pts[(6 + c) * N + gi];
        }
        dg_medium_t<T, false>((T)d0, (T)d1, (T)d2, m, D);
        contract_b_t<T>(D, m.c12, m.c44, m.hh, bj, tj, fi);
        contract_b_t<T>(D, m.c12, m.c44, m.hh, bi, ti, fj);
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      vij[lane * 6 + c] = fi[c];
      vji[lane * 6 + c] = -fj[c];  // dG(x_j - x_i) = -dG(x_i - x_j)
    }
    __syncthreads();
    const int pend = min(p0 + NT, npair);
    // one lane per (target, component); the running sum goes through
    // registers (one LDS read and write per round, not one per term)
    for (int w = lane; w < na * 6; w += NT) {  // A's target ii: one run of consecutive pairs
      const int ii = w / 6, c = w - ii * 6;
      const int s0 = self ? row0(ii) : ii * nb, len = self ? na - 1 - ii : nb;
      const int lo = max(s0, p0), hi = min(s0 + len, pend);
      if (lo >= hi) continue;
      T sa = accA[w], ca = (T)cmp_of(cmpA, w);
      for (int r = lo; r < hi; ++r) add(sa, ca, vij[(r - p0) * 6 + c]);
      accA[w] = sa;
      if constexpr (KC) cmpA[w] = ca;
    }
    for (int w = lane; self && w < nb * 6; w += NT) {  // B's target jj: pairs (i, jj), i < jj, in order of i
      const int jj = w / 6, c = w - jj * 6;
      const int iend = min(rhi, jj - 1);
      if (rlo > iend) continue;
      T sb = accB[w], cb = (T)cmp_of(cmpB, w);
      for (int i = rlo; i <= iend; ++i) {
        const int r = row0(i) + jj - i - 1;
        if (r >= p0 && r < pend) add(sb, cb, vji[(r - p0) * 6 + c]);
      }
      accB[w] = sb;
      if constexpr (KC) cmpB[w] = cb;
    }
    for (int w = lane; !self && w < nb * 6; w += NT) {  // B's target jj: lanes with p % nb == jj, in order
      const int jj = w / 6, c = w - jj * 6;
      const int r0 = p0 + ((jj - p0 % nb) % nb + nb) % nb;
      if (r0 >= pend) continue;
      T sb = accB[w], cb = (T)cmp_of(cmpB, w);
      for (int r = r0; r < pend; r += nb) add(sb, cb, vji[(r - p0) * 6 + c]);
      accB[w] = sb;
      if constexpr (KC) cmpB[w] = cb;
    }
    __syncthreads();
  }
  for (int ii = lane; ii < na; ii += NT)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = (double)accA[ii * 6 + c] - cmp_of(cmpA, ii * 6 + c);
      if (self) v += (double)accB[ii * 6 + c] - cmp_of(cmpB, ii * 6 + c);
      part[((int64_t)(fa + ii) * 27 + q) * 6 + c] = (T)v;
    }
  if (!self)
    for (int jj = lane; jj < nb; jj += NT)
#pragma unroll
      for (int c = 0; c < 6; ++c)
        part[((int64_t)(fb + jj) * 27 + (26 - q)) * 6 + c] =
            (T)((double)accB[jj * 6 + c] - cmp_of(cmpB, jj * 6 + c));
}

// The same symmetric near field for the leaf pairs with at most 64 points on
// each side, one wave per leaf A over all its pairs {A, A + o} (slots q =
// 13..26) as one run of point pairs: rounds of 64 pairs run across the
// pairs' boundaries, so only the run's last round is partly empty (one wave
// per leaf pair left most rounds partly empty: the 66 self pairs of a
// 12-point leaf took two rounds of 64).  Every target sums the same terms in
// the same order as with one wave per leaf pair, and a leaf pair's partials
// are written when its last pair has been summed.
template <typename T, bool MIXED>
__global__ void __launch_bounds__(64, sizeof(T) == 4 ? 4 : 3)
    k_leaf_sym_run(const double* pts, int64_t N, const int* first, const int* count, const int* nbr, Med<T> m,
                   double a2x4, T* part) {
  constexpr int NT = 64;
  // Single-precision sums are compensated; double-precision ones need not
  // be, and without the two compensation arrays (12 KB of LDS a wave) three
  // waves share a SIMD, where 18 KB allowed two.
  constexpr bool KC = sizeof(T) == 4;
  __shared__ T accA[64 * 6], cmpA[KC ? 64 * 6 : 1], accB[64 * 6], cmpB[KC ? 64 * 6 : 1], vij[NT * 6], vji[NT * 6];
  auto cmp_of = [&](const T* c, int w) -> double {
    if constexpr (KC) return (double)c[w];
    else return 0.0;
  };
  auto clear = [&](T* acc, T* c, int w) {
    acc[w] = T(0);
    if constexpr (KC) c[w] = T(0);
  };
  auto add = [&](T& s, T& c, T x) {
    if constexpr (KC) kadd(s, c, x);
    else s += x;
  };
  __shared__ int sB[14], sq[14], sstart[15], snseg;
  const int A = blockIdx.x, lane = threadIdx.x;
  const int fa = first[A], na = count[A];
  if (na > 64) return;  // all of A's pairs go to the large-leaf kernel
  if (lane == 0) {
    int ns = 0, tot = 0;
    for (int q = 13; q < 27; ++q) {
      const int B = nbr[(int64_t)A * 27 + q];
      if (B < 0 || count[B] > 64) continue;
      sB[ns] = B;
      sq[ns] = q;
      sstart[ns] = tot;
      tot += q == 13 ? na * (na - 1) / 2 : na * count[B];
      ++ns;
    }
    sstart[ns] = tot;
    snseg = ns;
  }
  for (int e = lane; e < 64 * 6; e += NT) {
    clear(accA, cmpA, e);
    clear(accB, cmpB, e);
  }
  __syncthreads();
  const int nseg = snseg, total = sstart[nseg];
  // the self pairs (slot 13, when present) come first; row i of them holds
  // (i, i+1 .. na-1) and starts at pair row0(i)
  const bool has_self = nseg > 0 && sq[0] == 13;
  const int nself = has_self ? sstart[1] : 0;
  auto row0 = [&](int i) { return i * na - i * (i + 1) / 2; };
  int ic = 0, rlo = 0, rhi = 0;
  int sflush = 0;  // segments before sflush have been written
  // writes segment s's partials (the lanes own the same items as in the sums)
  // and clears the sums for the next segment
  auto flush = [&](int s) {
    const int q = sq[s], B = sB[s], fb = first[B], nb = count[B];
    const bool self = q == 13;
    for (int w = lane; w < na * 6; w += NT) {
      double v = (double)accA[w] - cmp_of(cmpA, w);
      if (self) v += (double)accB[w] - cmp_of(cmpB, w);
      part[((int64_t)(fa + w / 6) * 27 + q) * 6 + w % 6] = (T)v;
      clear(accA, cmpA, w);
      if (self) clear(accB, cmpB, w);
    }
    if (!self)
      for (int w = lane; w < nb * 6; w += NT) {
        part[((int64_t)(fb + w / 6) * 27 + (26 - q)) * 6 + w % 6] = (T)((double)accB[w] - cmp_of(cmpB, w));
        clear(accB, cmpB, w);
      }
  };
  for (int p0 = 0; p0 < total; p0 += NT) {
    const int p = p0 + lane, pend = min(p0 + NT, total);
    T fi[6] = {0, 0, 0, 0, 0, 0}, fj[6] = {0, 0, 0, 0, 0, 0};
    if (p < total) {
      int s = 0;
      while (s + 1 < nseg && sstart[s + 1] <= p) ++s;
      const int pl = p - sstart[s];
      int i, j, fb;
      if (sq[s] == 13) {
        while (ic + 1 < na && row0(ic + 1) <= pl) ++ic;
        i = ic;
        j = i + 1 + (pl - row0(i));
        fb = fa;
      } else {
        const int nb = count[sB[s]];
        i = pl / nb;
        j = pl - i * nb;
        fb = first[sB[s]];
      }
      const int64_t gi = fa + i, gj = fb + j;
      const double d0 = pts[gi] - pts[gj], d1 = pts[N + gi] - pts[N + gj], d2 = pts[2 * N + gi] - pts[2 * N + gj];
      if (!MIXED || d0 * d0 + d1 * d1 + d2 * d2 >= a2x4) {
        T D[27], bj[3], tj[3], bi[3], ti[3];
        for (int c = 0; c < 3; ++c) {
          bj[c] = (T)pts[(3 + c) * N + gj], tj[c] = (T)pts[(6 + c) * N + gj];
          bi[c] = (T)pts[(3 + c) * N + gi], ti[c] = (T)pts[(6 + c) * N + gi];
        }
        dg_medium_t<T, false>((T)d0, (T)d1, (T)d2, m, D);
        contract_b_t<T>(D, m.c12, m.c44, m.hh, bj, tj, fi);
        contract_b_t<T>(D, m.c12, m.c44, m.hh, bi, ti, fj);
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      vij[lane * 6 + c] = fi[c];
      vji[lane * 6 + c] = -fj[c];  // dG(x_j - x_i) = -dG(x_i - x_j)
    }
    // rows of the round's first and last self pairs
    if (p0 < nself) {
      while (rlo + 1 < na && row0(rlo + 1) <= p0) ++rlo;
      const int plast = min(pend, nself) - 1;
      while (rhi + 1 < na && row0(rhi + 1) <= plast) ++rhi;
    }
    __syncthreads();
    // each segment met by the round: its sums as with one wave per leaf pair
    // (pair indices local to the segment), then its partials once it ends
    for (int s = sflush; s < nseg && sstart[s] < pend; ++s) {
      const int q = sq[s], s0 = sstart[s], s1 = sstart[s + 1];
      const int lo = max(p0, s0) - s0, hi = min(pend, s1) - s0;  // local pairs of this round
      const int off = s0 - p0;                                    // local pair r is vij[(r + off) * 6]
      const bool self = q == 13;
      const int nb = self ? na : count[sB[s]];
      for (int w = lane; w < na * 6; w += NT) {  // A's target ii: one run of consecutive pairs
        const int ii = w / 6, c = w - ii * 6;
        const int r0 = self ? row0(ii) : ii * nb, len = self ? na - 1 - ii : nb;
        const int a = max(r0, lo), b = min(r0 + len, hi);
        if (a >= b) continue;
        T sa = accA[w], ca = (T)cmp_of(cmpA, w);
        for (int r = a; r < b; ++r) add(sa, ca, vij[(r + off) * 6 + c]);
        accA[w] = sa;
        if constexpr (KC) cmpA[w] = ca;
      }
      if (self) {
        for (int w = lane; w < na * 6; w += NT) {  // B's target jj: pairs (i, jj), i < jj, in order of i
          const int jj = w / 6, c = w - jj * 6;
          const int iend = min(rhi, jj - 1);
          if (rlo > iend) continue;
          T sb = accB[w], cb = (T)cmp_of(cmpB, w);
          for (int i = rlo; i <= iend; ++i) {
            const int r = row0(i) + jj - i - 1;
            if (r >= lo && r < hi) add(sb, cb, vji[(r + off) * 6 + c]);
          }
          accB[w] = sb;
          if constexpr (KC) cmpB[w] = cb;
        }
      } else {
        for (int w = lane; w < nb * 6; w += NT) {  // B's target jj: local pairs r with r % nb == jj, in order
          const int jj = w / 6, c = w - jj * 6;
          const int r0 = lo + ((jj - lo % nb) % nb + nb) % nb;
          if (r0 >= hi) continue;
          T sb = accB[w], cb = (T)cmp_of(cmpB, w);
          for (int r = r0; r < hi; r += nb) add(sb, cb, vji[(r + off) * 6 + c]);
          accB[w] = sb;
          if constexpr (KC) cmpB[w] = cb;
        }
      }
      if (s1 <= pend) {
        flush(s);
        sflush = s + 1;
      }
    }
    __syncthreads();
  }
  // segments without pairs (the self pairs of a leaf with one point)
  for (int s = sflush; s < nseg; ++s) flush(s);
}

// Near-field stress of each point: its 27 neighbour-slot partials in slot
// order (slots of absent neighbour leaves are skipped).
template <typename T>
__global__ void k_near_sum(const T* part, int64_t N, const int* pleaf, const int* nbr, double* sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int leaf = pleaf[i];
  double tot[6] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < 27; ++q)
    if (nbr[(int64_t)leaf * 27 + q] >= 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) tot[c] += (double)part[(i * 27 + q) * 6 + c];
#pragma unroll
  for (int c = 0; c < 6; ++c) sig[i * 6 + c] = tot[c];
}

template <typename T, bool BIG>
inline size_t sym_lds(int lmax) {
  return sizeof(T) * ((sizeof(T) == 4 ? 24 : 12) * (size_t)lmax + 2 * (size_t)sym_threads<T, BIG>() * 6);
}
static_assert(sizeof(float) * (24 * kSymMaxLeaf + 2 * 256 * 6) <= 160 * 1024 &&
                  sizeof(double) * (12 * kSymMaxLeaf + 2 * 256 * 6) <= 160 * 1024,
              "the large-leaf near field's LDS at the largest symmetric leaf");

// The near-coincident pairs (closer than 2a) that the single-precision near
// field skips, in double precision.  The tree holds them per target point, in
// the order the near field visits its sources, and as unordered pairs with
// their two list entries.  One thread per unordered pair evaluates the
// kernel derivative once (it is odd: dG(x_j - x_i) = -dG(x_i - x_j)) and
// writes the stress of both list entries; then one thread per target adds
// its entries in list order (a fixed summation order) to the near field.
template <bool ISO>
__global__ void __launch_bounds__(64) k_close_eval(const double* pts, int64_t N, const int2* cpair,
                                                   const int2* cuni, int64_t nuni, Med<double> m64, double* cval) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nuni) return;
  const int2 ks = cuni[u];
  const int2 pr = cpair[ks.x];
  const int64_t it = pr.x, j = pr.y;
  const double d0 = pts[it] - pts[j], d1 = pts[N + it] - pts[N + j], d2 = pts[2 * N + it] - pts[2 * N + j];
  double D[27], bb[3], tt[3], v[6] = {0, 0, 0, 0, 0, 0}, w[6] = {0, 0, 0, 0, 0, 0};
  dg_medium_t<double, ISO>(d0, d1, d2, m64, D);
  for (int c = 0; c < 3; ++c) bb[c] = pts[(3 + c) * N + j], tt[c] = pts[(6 + c) * N + j];
  contract_b_t<double>(D, m64.c12, m64.c44, m64.hh, bb, tt, v);
#pragma unroll
  for (int c = 0; c < 6; ++c) cval[(int64_t)ks.x * 6 + c] = v[c];
  if (ks.y >= 0) {
    for (int c = 0; c < 3; ++c) bb[c] = pts[(3 + c) * N + it], tt[c] = pts[(6 + c) * N + it];
    contract_b_t<double>(D, m64.c12, m64.c44, m64.hh, bb, tt, w);
#pragma unroll
    for (int c = 0; c < 6; ++c) cval[(int64_t)ks.y * 6 + c] = -w[c];
  }
}

__global__ void k_close_sum(const int* cstart, int64_t N, const double* cval, double* sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int k = cstart[i]; k < cstart[i + 1]; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += cval[(int64_t)k * 6 + c];
  if (cstart[i + 1] > cstart[i])
#pragma unroll
    for (int c = 0; c < 6; ++c) sig[i * 6 + c] += acc[c];
}

// L2P: far-field stress at each point by interpolation of its leaf's local
// values (Lagrange basis on the leaf's equispaced nodes), added to the near
// field already in sig.  One thread per point.
template <typename T, int P>
__global__ void k_l2p(const double* pts, int64_t N, const int* pleaf, const uint32_t* key, const T* s, double lo0,
                      double lo1, double lo2, double sD, double* sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int leaf = pleaf[i];
  double lo[3];
  cell_lo(key[leaf], lo0, lo1, lo2, sD, lo);
  constexpr int p3 = P * P * P;
  const T* sl = s + (int64_t)leaf * 6 * p3;
  const T t[3] = {(T)((pts[i] - lo[0]) / sD), (T)((pts[N + i] - lo[1]) / sD), (T)((pts[2 * N + i] - lo[2]) / sD)};
  T L1[P], L2[P];  // the first axis' basis value is formed inside its (rolled) loop
#pragma unroll
  for (int k = 0; k < P; ++k) {
    L1[k] = lagr<T>(P, k, t[1]);
    L2[k] = lagr<T>(P, k, t[2]);
  }
  T far[6] = {0, 0, 0, 0, 0, 0};
  for (int l1 = 0; l1 < P; ++l1) {
    const T L0 = lagr<T>(P, l1, t[0]);
#pragma unroll
    for (int l2 = 0; l2 < P; ++l2) {
      const T w12 = L0 * L1[l2];
#pragma unroll
      for (int l3 = 0; l3 < P; ++l3) {
        const T w = w12 * L2[l3];
        const int node = (l1 * P + l2) * P + l3;
#pragma unroll
        for (int c = 0; c < 6; ++c) far[c] = fma(w, sl[c * p3 + node], far[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) sig[i * 6 + c] += (double)far[c];
}

template <typename T>
static void l2p_launch(int p, int64_t N, const double* pts, const int* pleaf, const uint32_t* key, const T* s,
                       const double* lo, double sD, double* sig, hipStream_t st) {
  const unsigned blocks = (unsigned)((N + 255) / 256);
#define L2P(P_) k_l2p<T, P_><<<blocks, 256, 0, st>>>(pts, N, pleaf, key, s, lo[0], lo[1], lo[2], sD, sig)
  switch (p) {
    case 2: L2P(2); break;
    case 3: L2P(3); break;
    case 4: L2P(4); break;
    case 5: L2P(5); break;
    case 6: L2P(6); break;
    case 7: L2P(7); break;
    default: L2P(8); break;
  }
#undef L2P
}

// ---------------------------------------------------------------- forces
__device__ __forceinline__ void pk_force(const double* sg, const double* b, const double* dS, double* fx) {
  double sb0 = sg[0] * b[0] + sg[5] * b[1] + sg[4] * b[2];
  double sb1 = sg[5] * b[0] + sg[1] * b[1] + sg[3] * b[2];
  double sb2 = sg[4] * b[0] + sg[3] * b[1] + sg[2] * b[2];
  fx[0] = sb1 * dS[2] - sb2 * dS[1];
  fx[1] = sb2 * dS[0] - sb0 * dS[2];
  fx[2] = sb0 * dS[1] - sb1 * dS[0];
}

// forces[t] for segments seg_idx(t) (= t, or targets[t]); stress of point k of
// target t at sig[row(t, k)] with row = inv[s*nq + k] (FMM) or t*nq + k (direct).
__global__ void k_forces(const double* seg, const double* burg, const int64_t* targets, const uint32_t* inv,
                         const double* sig, Quad qd, int64_t nt, double* forces) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int64_t s = targets ? targets[t] : t;
  const double* x = seg + 6 * s;
  double dS[3] = {x[3] - x[0], x[4] - x[1], x[5] - x[2]};
  double b[3] = {burg[3 * s], burg[3 * s + 1], burg[3 * s + 2]};
  double f1[3] = {0, 0, 0}, f2[3] = {0, 0, 0};
  for (int k = 0; k < qd.n; ++k) {
    int64_t row = inv ? (int64_t)inv[s * qd.n + k] : t * qd.n + k;
    double fx[3];
    pk_force(sig + row * 6, b, dS, fx);
    double sk = 0.5 * (1.0 + qd.u[k]), hw = 0.5 * qd.w[k];
    for (int c = 0; c < 3; ++c) {
      f1[c] += hw * (1.0 - sk) * fx[c];
      f2[c] += hw * sk * fx[c];
    }
  }
  for (int c = 0; c < 3; ++c) {
    forces[6 * t + c] = f1[c];
    forces[6 * t + 3 + c] = f2[c];
  }
}

// ---------------------------------------------------------------- direct
__global__ void k_points_plain(const double* seg, const double* burg, Quad qd, int64_t N, double* pts) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  int64_t s = j / qd.n;
  int k = (int)(j - s * qd.n);
  const double* x = seg + 6 * s;
  double dS[3] = {x[3] - x[0], x[4] - x[1], x[5] - x[2]};
  double c = 0.5 * (1.0 + qd.u[k]), hw = 0.5 * qd.w[k];
  for (int d = 0; d < 3; ++d) {
    pts[d * N + j] = x[d] + c * dS[d];
    pts[(3 + d) * N + j] = burg[3 * s + d];
    pts[(6 + d) * N + j] = hw * dS[d];
  }
}

// Block = 256 target points x one chunk of sources (staged in LDS in tiles).
// part[chunk][tp][6] holds the chunk's partial stress in double.
template <bool FP32, bool ISO>
__global__ void __launch_bounds__(256) k_direct(const double* pts, int64_t N, const int64_t* targets, int nq,
                                                int64_t ntp, int64_t chunk, Med<double> m64, Med<float> m32,
                                                double* part) {
  __shared__ double sp[9][256];
  const int64_t tp = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool act = tp < ntp;
  int64_t src_pt = 0;
  if (act) {
    int64_t t = tp / nq;
    int k = (int)(tp - t * nq);
    src_pt = (targets ? targets[t] : t) * nq + k;
  }
  const double x0 = act ? pts[src_pt] : 0, x1 = act ? pts[N + src_pt] : 0, x2 = act ? pts[2 * N + src_pt] : 0;
  const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(N, j0 + chunk);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  float af[6] = {0, 0, 0, 0, 0, 0}, cf[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t jt = j0; jt < j1; jt += 256) {
    const int nt = (int)min((int64_t)256, j1 - jt);
    __syncthreads();
    if (threadIdx.x < nt)
      for (int c = 0; c < 9; ++c) sp[c][threadIdx.x] = pts[c * N + jt + threadIdx.x];
    __syncthreads();
    if (!act) continue;
    for (int j = 0; j < nt; ++j) {
      double d0 = x0 - sp[0][j], d1 = x1 - sp[1][j], d2 = x2 - sp[2][j];
      if (FP32) {
        float D[27], b[3] = {(float)sp[3][j], (float)sp[4][j], (float)sp[5][j]},
                     t[3] = {(float)sp[6][j], (float)sp[7][j], (float)sp[8][j]};
        dg_medium_t<float, ISO>((float)d0, (float)d1, (float)d2, m32, D);
        float ds[6] = {0, 0, 0, 0, 0, 0};
        contract_b_t<float>(D, m32.c12, m32.c44, m32.hh, b, t, ds);
        for (int c = 0; c < 6; ++c) {
          float y = ds[c] - cf[c];
          float z = af[c] + y;
          cf[c] = (z - af[c]) - y;
          af[c] = z;
        }
      } else {
        double D[27], b[3] = {sp[3][j], sp[4][j], sp[5][j]}, t[3] = {sp[6][j], sp[7][j], sp[8][j]};
        dg_medium_t<double, ISO>(d0, d1, d2, m64, D);
        contract_b_t<double>(D, m64.c12, m64.c44, m64.hh, b, t, acc);
      }
    }
  }
  if (act) {
    double* o = part + ((int64_t)blockIdx.y * ntp + tp) * 6;
    for (int c = 0; c < 6; ++c) o[c] = FP32 ? ((double)af[c] - (double)cf[c]) : acc[c];
  }
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_check_targets(const int64_t* targets, int64_t nt, int64_t nseg, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nt && (targets[i] < 0 || targets[i] >= nseg)) atomicOr(bad, 1);
}

__global__ void k_direct_reduce(const double* part, int64_t ntp, int nchunk, double* sig) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntp * 6) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * ntp * 6 + i];
  sig[i] = s;
}

// ------------------------------------------------------------ host side
// DFT launches, specialised on the interpolation order.  Forward: as many
// components per round as fit the LDS; inverse: all six in one round.
template <typename T, int P>
static int dft_groups(bool fwd) {
  const size_t es = sizeof(T);
  for (int G : {9, 3, 1})
    if (lds_fdft_t<P>(G, es) <= 160 * 1024) return G;
  (void)fwd;
  return 1;
}

// wmax: non-null for DFMM_MIXED_F16 (f16 source spectra, scaled; the inverse
// transform removes the operator scale kscale and the source scale).
template <typename T, int P>
static void dft_launch(bool fwd, unsigned blocks, const void* in, int64_t ncell, const T* tw, void* out,
                       const unsigned* wmax, float kscale, int fa, int fb, int acc, hipStream_t st) {
  const int G = dft_groups<T, P>(fwd);
  constexpr int C = fdft_cpb<T, P>();
  const unsigned fblocks = (unsigned)((blocks + C - 1) / C);
  if (fwd && wmax)
    k_fdft<T, P, true, C><<<fblocks, kDftThreads * C, C * lds_fdft_t<P>(G, sizeof(T)), st>>>(
        (const T*)in, ncell, G, tw, (cplx<T>*)out, wmax, fa, fb);
  else if (fwd)
    k_fdft<T, P, false, C><<<fblocks, kDftThreads * C, C * lds_fdft_t<P>(G, sizeof(T)), st>>>(
        (const T*)in, ncell, G, tw, (cplx<T>*)out, nullptr, fa, fb);
  else
  {
    constexpr int C = idft_cpb<T, P>();
    k_idft<T, P, C><<<(unsigned)((blocks + C - 1) / C), C > 1 ? 1024 : kDftThreads, C * lds_idft_t<P>(sizeof(T)), st>>>(
        (const cplx<T>*)in, ncell, tw, (T*)out, wmax, kscale, fa, fb, acc);
  }
}

// fa, fb: the chunk of first frequency indices (0, n for the whole
// spectrum); acc: the inverse transform adds to its output.
template <typename T>
static void dft(int p, bool fwd, unsigned blocks, const void* in, int64_t ncell, const T* tw, void* out,
                const unsigned* wmax, float kscale, int fa, int fb, int acc, hipStream_t st) {
  switch (p) {
    case 2: dft_launch<T, 2>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    case 3: dft_launch<T, 3>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    case 4: dft_launch<T, 4>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    case 5: dft_launch<T, 5>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    case 6: dft_launch<T, 6>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    case 7: dft_launch<T, 7>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
    default: dft_launch<T, 8>(fwd, blocks, in, ncell, tw, out, wmax, kscale, fa, fb, acc, st); break;
  }
}

// M2M (up) or L2L (down) launch, specialised on the order.  For M2M, a / b
// are the parents' first child and child count; for L2L, a is the parent
// index of each child (b unused).
template <typename T, int P>
static void tree_pass_p(bool up, unsigned blocks, size_t shm, const int* a, const int* b, const uint32_t* key,
                        const T* in, T* out, const T* S, unsigned* wmax, hipStream_t st) {
  if (up)
    k_m2m<T, P><<<blocks, kM2mThreads, shm, st>>>(a, b, key, in, out, S, wmax);
  else
    k_l2l<T, P><<<blocks, 256, shm, st>>>(a, key, in, out, S);
}

template <typename T>
static void tree_pass(int p, bool up, unsigned blocks, size_t shm, const int* a, const int* b, const uint32_t* key,
                      const T* in, T* out, const T* S, unsigned* wmax, hipStream_t st) {
  switch (p) {
    case 2: tree_pass_p<T, 2>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    case 3: tree_pass_p<T, 3>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    case 4: tree_pass_p<T, 4>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    case 5: tree_pass_p<T, 5>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    case 6: tree_pass_p<T, 6>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    case 7: tree_pass_p<T, 7>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
    default: tree_pass_p<T, 8>(up, blocks, shm, a, b, key, in, out, S, wmax, st); break;
  }
}

template <typename T>
static void project(int p, unsigned blocks, T* data, int ncomp, const T* Pm, hipStream_t st) {
  const size_t shm = sizeof(T) * 2 * ncomp * (size_t)p * p * p;
#define PROJ(P_) k_project<T, P_><<<blocks, 256, shm, st>>>(data, ncomp, Pm)
  switch (p) {
    case 2: PROJ(2); break;
    case 3: PROJ(3); break;
    case 4: PROJ(4); break;
    case 5: PROJ(5); break;
    case 6: PROJ(6); break;
    case 7: PROJ(7); break;
    default: PROJ(8); break;
  }
#undef PROJ
}

template <typename T, int... Ps>
static void dft_lds_attrs(std::integer_sequence<int, Ps...>) {
  const int mx = 160 * 1024;
  ((void)hipFuncSetAttribute((const void*)k_fdft<T, Ps + 2, false, fdft_cpb<T, Ps + 2>()>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, mx), ...);
  ((void)hipFuncSetAttribute((const void*)k_fdft<T, Ps + 2, true, fdft_cpb<T, Ps + 2>()>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, mx), ...);
  ((void)hipFuncSetAttribute((const void*)k_idft<T, Ps + 2, idft_cpb<T, Ps + 2>()>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, mx), ...);
  // k_m2m: its three buffers (it also has a small static array)
  ((void)hipFuncSetAttribute((const void*)k_m2m<T, Ps + 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(T) * 27 * (Ps + 2) * (Ps + 2) * (Ps + 2))), ...);
  ((void)hipFuncSetAttribute((const void*)k_l2l<T, Ps + 2>, hipFuncAttributeMaxDynamicSharedMemorySize, mx), ...);
  ((void)hipFuncSetAttribute((const void*)k_project<T, Ps + 2>, hipFuncAttributeMaxDynamicSharedMemorySize, mx), ...);
}

struct StageTimer {
  dfmm_tree* t;
  hipStream_t st;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  int begin(int stage) {
    if (!t->timing) return DFMM_OK;
    hipEvent_t a, b;
    DFMM_HIP(hipEventCreate(&a));
    DFMM_HIP(hipEventCreate(&b));
    DFMM_HIP(hipEventRecord(a, st));
    ev.push_back({stage, {a, b}});
    return DFMM_OK;
  }
  int end() {
    if (!t->timing) return DFMM_OK;
    DFMM_HIP(hipEventRecord(ev.back().second.second, st));
    return DFMM_OK;
  }
  int finish() {
    if (!t->timing) return DFMM_OK;
    DFMM_HIP(hipEventSynchronize(ev.back().second.second));
    for (auto& e : ev) {
      float ms = 0;
      DFMM_HIP(hipEventElapsedTime(&ms, e.second.first, e.second.second));
      t->stage_ms[e.first] += ms;
      hipEventDestroy(e.second.first);
      hipEventDestroy(e.second.second);
    }
    t->timed_calls++;
    return DFMM_OK;
  }
};

#define STAGE(id, body)             \
  do {                              \
    int rc_ = tm.begin(id);         \
    if (rc_) return rc_;            \
    body;                           \
    DFMM_LAUNCH_CHECK();            \
    rc_ = tm.end();                 \
    if (rc_) return rc_;            \
  } while (0)

template <typename T>
static int run_fmm(const dfmm_plan* pl, dfmm_tree* t, const double* seg, const double* burg, double* forces,
                   hipStream_t st) {
  const int p = pl->p, p3 = p * p * p, n = pl->n, nf = pl->nf, D = t->D;  // the tree's deepest level
  const int64_t N = t->N;
  const size_t es = sizeof(T);
  const Tables<T>& tb = *(const Tables<T>*)(std::is_same<T, double>::value ? (const void*)&pl->t64
                                                                          : (const void*)&pl->t32);
  const double* lo = pl->prm.box_lo;
  const double L = pl->prm.box_size;
  T* W = (T*)t->W;
  T* s = (T*)t->s;
  cplx<T>* What = (cplx<T>*)t->What;
  cplx<T>* Shat = (cplx<T>*)t->Shat;
  StageTimer tm{t, st, {}};
  const auto& LD = t->lv[D];
  const double sD = L / std::ldexp(1.0, D);

  STAGE(0, (k_gather<<<nblk(N, 256), 256, 0, st>>>(seg, burg, t->perm, pl->quad, N, t->pts)));
  // The near field needs only the gathered points: it runs on the tree's
  // second stream beside P2M..L2L, unless stages are being timed one by one
  // or the caller's stream is being captured into a graph (there the near
  // field stays on the capturing stream; a batch overlaps its configurations
  // across its own lanes instead).
  hipStream_t nst = st;
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  DFMM_HIP(hipStreamIsCapturing(st, &capture));
  if (!t->timing && t->side && capture == hipStreamCaptureStatusNone) {
    DFMM_HIP(hipEventRecord(t->fork, st));
    DFMM_HIP(hipStreamWaitEvent(t->side, t->fork, 0));
    nst = t->side;
  }
#define ACALL(call)     \
  do {                  \
    int r_ = (call);    \
    if (r_) return r_;  \
  } while (0)
  {
    Med<T> m = pl->med<T>();
    Med<double> m64 = pl->med<double>();
#define LEAF_ARGS t->pts, N, LD.first, LD.count, t->nbr, m, m64, t->sig
    SurDev sd = sur_dev(pl);
    if constexpr (std::is_same<T, float>::value) {
      if (t->adaptive) {
        STAGE(6, ACALL(adapt_near<T>(pl, t, nst)));
      } else if (!pl->iso && sd.on) {
        const int grid = (int)std::max<int64_t>(
            1, std::min<int64_t>(sur_grid(pl->device), (LD.n + kSurLeafThreads / 64 - 1) / (kSurLeafThreads / 64)));
        STAGE(6, (k_leaf_sur<<<grid, kSurLeafThreads, kSurInfLds, nst>>>(t->pts, N, LD.first, LD.count, t->nbr, LD.n,
                                                                          m, m64, sd, t->sig)));
      } else if (pl->iso)
        STAGE(6, (k_leaf<T, true, true><<<(unsigned)LD.n, 64, 0, nst>>>(LEAF_ARGS)));
      else if (t->part) {
        const double a2x4 = 4.0 * m64.a * m64.a;
        STAGE(6, (k_leaf_sym_run<T, true><<<(unsigned)LD.n, 64, 0, nst>>>(t->pts, N, LD.first, LD.count, t->nbr, m,
                                                                         a2x4, (T*)t->part)));
        if (t->nbig > 0)
          STAGE(6, (k_leaf_sym<T, true, true><<<(unsigned)t->nbig, sym_threads<T, true>(), sym_lds<T, true>(t->max_leaf_pts), nst>>>(
                       t->pts, N, LD.first, LD.count, t->nbr, m, a2x4, t->max_leaf_pts, (T*)t->part, t->bigp)));
      }
      else
        STAGE(6, (k_leaf<T, true, false><<<(unsigned)LD.n, 64, 0, nst>>>(LEAF_ARGS)));
      if (!t->adaptive && !pl->iso && !sd.on && t->part)
        STAGE(6, (k_near_sum<T><<<nblk(N, 256), 256, 0, nst>>>((const T*)t->part, N, t->pleaf, t->nbr, t->sig)));
      if (t->nclose > 0) {
        if (pl->iso)
          STAGE(6, (k_close_eval<true><<<nblk(t->nuni, 64), 64, 0, nst>>>(t->pts, N, t->cpair, t->cuni, t->nuni,
                                                                          m64, t->cval)));
        else
          STAGE(6, (k_close_eval<false><<<nblk(t->nuni, 64), 64, 0, nst>>>(t->pts, N, t->cpair, t->cuni, t->nuni,
                                                                           m64, t->cval)));
        STAGE(6, (k_close_sum<<<nblk(N, 256), 256, 0, nst>>>(t->cstart, N, t->cval, t->sig)));
      }
    } else {
      if (t->adaptive) {
        STAGE(6, ACALL(adapt_near<T>(pl, t, nst)));
      } else if (pl->iso) {
        STAGE(6, (k_leaf<T, false, true><<<(unsigned)LD.n, 64, 0, nst>>>(LEAF_ARGS)));
      } else if (t->part) {
        STAGE(6, (k_leaf_sym_run<T, false><<<(unsigned)LD.n, 64, 0, nst>>>(t->pts, N, LD.first, LD.count, t->nbr, m,
                                                                          0.0, (T*)t->part)));
        if (t->nbig > 0)
          STAGE(6, (k_leaf_sym<T, false, true><<<(unsigned)t->nbig, sym_threads<T, true>(), sym_lds<T, true>(t->max_leaf_pts), nst>>>(
                       t->pts, N, LD.first, LD.count, t->nbr, m, 0.0, t->max_leaf_pts, (T*)t->part, t->bigp)));
        STAGE(6, (k_near_sum<T><<<nblk(N, 256), 256, 0, nst>>>((const T*)t->part, N, t->pleaf, t->nbr, t->sig)));
      } else {
        STAGE(6, (k_leaf<T, false, false><<<(unsigned)LD.n, 64, 0, nst>>>(LEAF_ARGS)));
      }
    }
#undef LEAF_ARGS
  }
  // DFMM_MIXED_F16: each level's largest |W|, for the f16 scale of its
  // spectra, folded in by the kernels that write W (P2M, M2M); when the
  // projection below changes W afterwards, taken by k_wmax once it has
  const bool h16 = std::is_same<T, float>::value && pl->h16;
  const bool wfuse = h16 && pl->lsq == 0;
  if (wfuse) STAGE(0, (k_fill_uint<<<1, 64, 0, st>>>(t->wmax, D + 1, 0u)));
  auto wm_of = [&](int l) { return wfuse ? t->wmax + l : nullptr; };
  const int p2m_bs = std::max(64, ((p3 + 63) / 64) * 64);
  const size_t p2m_shm = es * (64 * 3 * p + 64 * 9);
  // P2M of the leaves of level l of an adaptive tree (after that level's M2M,
  // which leaves zeros in its leaves)
  auto p2m_level = [&](int l) {
    if (t->leaf_n[l] > 0)
      k_p2m<T><<<(unsigned)t->leaf_n[l], p2m_bs, p2m_shm, st>>>(
          t->pts, N, t->gl_pf + t->leaf_off[l], t->gl_pc + t->leaf_off[l], t->gkey, lo[0], lo[1], lo[2],
          L / std::ldexp(1.0, l), p, W, t->gl_cell + t->leaf_off[l], wm_of(l));
  };
  if (t->adaptive)
    STAGE(0, p2m_level(D));
  else
    STAGE(0, (k_p2m<T><<<(unsigned)LD.n, p2m_bs, p2m_shm, st>>>(t->pts, N, LD.first, LD.count, LD.key, lo[0],
                                                                  lo[1], lo[2], sD, p, W + LD.off * 9 * p3,
                                                                  nullptr, wm_of(D))));
  {
    size_t shm = es * 27 * p3;
    for (int l = D - 1; l >= 2; --l) {
      const auto& Lc = t->lv[l + 1];
      const auto& Lp = t->lv[l];
      STAGE(1, tree_pass<T>(p, true, (unsigned)Lp.n, shm, Lp.first, Lp.count, Lc.key, W + Lc.off * 9 * p3,
                               W + Lp.off * 9 * p3, tb.S, wm_of(l), st));
      if (t->adaptive) STAGE(1, p2m_level(l));
    }
  }
  // stabilised interpolation: the M2L takes the projected weights (the
  // upward pass above used the Lagrange ones, whose parent transfer is exact)
  if (pl->lsq > 0)
    for (int l = 2; l <= D; ++l)
      if (t->lv[l].n > 0) STAGE(1, project<T>(p, (unsigned)t->lv[l].n, W + t->lv[l].off * 9 * p3, 9, tb.Pm, st));
  if (h16 && !wfuse) {
    STAGE(2, (k_fill_uint<<<1, 64, 0, st>>>(t->wmax, D + 1, 0u)));
    for (int l = 2; l <= D; ++l) {
      const auto& Lv = t->lv[l];
      const int64_t nw = Lv.n * 9 * p3;
      if (nw > 0)
        STAGE(2, (k_wmax<<<(unsigned)std::min<int64_t>(8192, (nw / 4 + 255) / 256 + 1), 256, 0, st>>>(
                     (const float*)(W + Lv.off * 9 * p3), nw, t->wmax + l)));
    }
  }
  for (int l = 2; l <= D; ++l) {
    const auto& Lv = t->lv[l];
    if (Lv.n == 0) continue;
    const unsigned* wm = h16 ? t->wmax + l : nullptr;
    const int wsz = m2l_window(pl->mixed);
    const int nwin = (int)((Lv.n + wsz - 1) / wsz);
    const int remap = nwin >= 16;
    // symmetry-reduced store: this level's 158 offset spectra, expanded into
    // the tree's workspace
    const cplx<T>* kh = (const cplx<T>*)pl->lev[l].khat;
    const float ksc = pl->lev[l].kscale;
    if (pl->sym) {
      if (h16)
        STAGE(3, (k_sym_expand<T, true><<<nblk((int64_t)nf * kNumCanon * 54, 256), 256, 0, st>>>(
                     kh, pl->symtab, nf, n, p, ksc, (cplx<T>*)t->kexp)));
      else
        STAGE(3, (k_sym_expand<T, false><<<nblk((int64_t)nf * kNumCanon * 54, 256), 256, 0, st>>>(
                     kh, pl->symtab, nf, n, p, 1.f, (cplx<T>*)t->kexp)));
      kh = (const cplx<T>*)t->kexp;
    }
    // the spectrum in chunks of first frequency indices [fa, fb): forward
    // DFT of the chunk, its Hadamard product, inverse DFT added to s
    for (int fa = 0; fa < n; fa += t->fchunk) {
      const int fb = std::min(n, fa + t->fchunk);
      const int nfc = (fb - fa) * n * p;     // frequencies of the chunk
      const int64_t fbase = (int64_t)fa * n * p;
      dim3 g(remap ? 8 * ((nwin + 7) / 8) : nwin, nfc);
      STAGE(2, dft<T>(p, true, (unsigned)Lv.n, W + Lv.off * 9 * p3, Lv.n, tb.tw, What, wm, 1.f, fa, fb, 0, st));
      if (h16)
        STAGE(3, (k_hadamard16<<<g, kHadThreads, kHadLdsH, st>>>(
                     (const uint32_t*)What, (const uint32_t*)kh + fbase * kNumOffsets * kKOffsetH, Lv.lenq,
                     Lv.wbase, Lv.ilw, Lv.order, Lv.n, nfc, nwin, remap, (cplx<float>*)Shat)));
      else if constexpr (std::is_same<T, float>::value)
        STAGE(3, (k_hadamard<<<g, kHadThreads, kHadLdsF, st>>>(
                     What, kh + fbase * kNumCanon * kKOffsetF, Lv.lenq, Lv.wbase, Lv.ilw, Lv.order, Lv.n, nfc,
                     nwin, remap, Shat)));
      else
        STAGE(3, (k_hadamard64<<<g, kHadThreadsD, kHadLdsD, st>>>(
                     What, kh + fbase * kNumCanon * kKOffsetD, Lv.lenq, Lv.wbase, Lv.ilw, Lv.order, Lv.n, nfc, nwin,
                     remap, Shat)));
      STAGE(4, dft<T>(p, false, (unsigned)Lv.n, Shat, Lv.n, tb.tw, s + Lv.off * 6 * p3, wm, ksc, fa, fb, fa > 0, st));
    }
  }
  // adaptive tree: the points of each X leaf onto the nodes of the cells
  // that list it, before the local values go down the tree
  if (t->adaptive) STAGE(4, ACALL(adapt_p2l<T>(pl, t, s, st)));
  {
    // stabilised interpolation: each level's local values are projected
    // before they go to the children (L2L) or the points (L2P)
    if (pl->lsq > 0 && t->lv[2].n > 0)
      STAGE(5, project<T>(p, (unsigned)t->lv[2].n, s + t->lv[2].off * 6 * p3, 6, tb.Pm, st));
    size_t shm = es * 12 * p3;
    for (int l = 3; l <= D; ++l) {
      const auto& Lv = t->lv[l];
      const auto& Lp = t->lv[l - 1];
      STAGE(5, tree_pass<T>(p, false, (unsigned)Lv.n, shm, Lv.parent, nullptr, Lv.key, s + Lp.off * 6 * p3,
                               s + Lv.off * 6 * p3, tb.S, nullptr, st));
      if (pl->lsq > 0 && Lv.n > 0) STAGE(5, project<T>(p, (unsigned)Lv.n, s + Lv.off * 6 * p3, 6, tb.Pm, st));
    }
  }
  if (nst != st) {
    DFMM_HIP(hipEventRecord(t->join, nst));
    DFMM_HIP(hipStreamWaitEvent(st, t->join, 0));
  }
  if (t->adaptive) {
    // W lists (multipole weights at the nodes of finer cells onto a leaf's
    // points), then L2P from each point's leaf, whatever its level
    STAGE(6, ACALL(adapt_m2p<T>(pl, t, W, st)));
    STAGE(6, ACALL(adapt_l2p<T>(pl, t, s, st)));
  } else {
    STAGE(6, l2p_launch<T>(p, N, t->pts, t->pleaf, LD.key, s + LD.off * 6 * p3, lo, sD, t->sig, st));
  }
  STAGE(7, (k_forces<<<nblk(t->nseg, 128), 128, 0, st>>>(seg, burg, nullptr, t->inv, t->sig, pl->quad,
                                                          t->nseg, forces)));
  if (capture == hipStreamCaptureStatusNone && t->done) {
    DFMM_HIP(hipEventRecord(t->done, st));
    t->done_set = true;
  }
  return tm.finish();
}

template <typename T>
static void set_lds_attrs_once() {
  const int mx = 160 * 1024;
  hipFuncSetAttribute((const void*)k_hadamard, hipFuncAttributeMaxDynamicSharedMemorySize, kHadLdsF);
  hipFuncSetAttribute((const void*)k_hadamard16, hipFuncAttributeMaxDynamicSharedMemorySize, kHadLdsH);
  hipFuncSetAttribute((const void*)k_hadamard64, hipFuncAttributeMaxDynamicSharedMemorySize, kHadLdsD);
  hipFuncSetAttribute((const void*)k_leaf_sym<T, sizeof(T) == 4, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      mx);
  dft_lds_attrs<T>(std::make_integer_sequence<int, kMaxOrder - 1>{});
  // k_p2m: 64 points' basis values and strengths at the largest order (it
  // also has a small static array)
  hipFuncSetAttribute((const void*)k_p2m<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)(sizeof(T) * 64 * (3 * kMaxOrder + 9)));
  hipFuncSetAttribute((const void*)k_leaf_sur, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
}

// Kernel attributes are set once per process and precision, from whichever
// thread gets there first.
template <typename T>
static void set_lds_attrs() {
  static std::once_flag once;
  std::call_once(once, set_lds_attrs_once<T>);
}

void fmm_prepare(const dfmm_plan* pl) {
  if (pl->mixed) set_lds_attrs<float>();
  else set_lds_attrs<double>();
}

int fmm_forces_impl(const dfmm_plan* pl, dfmm_tree* t, const double* seg, const double* burg, double* forces,
                    hipStream_t st) {
  if (pl->mixed) {
    set_lds_attrs<float>();
    return run_fmm<float>(pl, t, seg, burg, forces, st);
  }
  set_lds_attrs<double>();
  return run_fmm<double>(pl, t, seg, burg, forces, st);
}

// Direct sum on caller-provided scratch: pts [9][N], part [nchunk][ntp][6],
// sig [ntp][6] (double); bad: one int (zeroed here by a fill kernel, not a
// memset, so that the call may be captured).  With targets, their indices
// are checked first (one host synchronisation).  Asynchronous otherwise.
static int direct_core(const dfmm_plan* pl, const double* seg, const double* burg, int64_t nseg,
                       const int64_t* targets, int64_t ntgt, double* forces, int fp32, hipStream_t st,
                       double* pts, double* part, double* sig, int* bad, int64_t nchunk, int64_t chunk) {
  const int nq = pl->quad.n;
  const int64_t N = nseg * nq, ntp = ntgt * nq;
  const int64_t tb = (ntp + 255) / 256;
  if (targets) {
    // reject target indices outside [0, nseg) before any kernel reads through them
    int hbad = 0;
    k_fill_int<<<1, 64, 0, st>>>(bad, 1, 0);
    DFMM_LAUNCH_CHECK();
    k_check_targets<<<nblk(ntgt, 256), 256, 0, st>>>(targets, ntgt, nseg, bad);
    DFMM_LAUNCH_CHECK();
    DFMM_D2H(&hbad, bad, sizeof(int), st);
    if (hbad) {
      set_error("direct_forces: target index outside [0, n_seg)");
      return DFMM_E_ARG;
    }
  }
  k_points_plain<<<nblk(N, 256), 256, 0, st>>>(seg, burg, pl->quad, N, pts);
  DFMM_LAUNCH_CHECK();
  dim3 g((unsigned)tb, (unsigned)nchunk);
#define DIRECT_ARGS pts, N, targets, nq, ntp, chunk, pl->med<double>(), pl->med<float>(), part
  if (fp32 && pl->iso)
    k_direct<true, true><<<g, 256, 0, st>>>(DIRECT_ARGS);
  else if (fp32)
    k_direct<true, false><<<g, 256, 0, st>>>(DIRECT_ARGS);
  else if (pl->iso)
    k_direct<false, true><<<g, 256, 0, st>>>(DIRECT_ARGS);
  else
    k_direct<false, false><<<g, 256, 0, st>>>(DIRECT_ARGS);
#undef DIRECT_ARGS
  DFMM_LAUNCH_CHECK();
  k_direct_reduce<<<nblk(ntp * 6, 256), 256, 0, st>>>(part, ntp, (int)nchunk, sig);
  DFMM_LAUNCH_CHECK();
  k_forces<<<nblk(ntgt, 128), 128, 0, st>>>(seg, burg, targets, nullptr, sig, pl->quad, ntgt, forces);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

// Source chunks of the direct sum: enough blocks to fill the chip (about
// 4096), each chunk a multiple of the 256-point LDS tile.
static void direct_chunks(int64_t N, int64_t ntp, int64_t* nchunk, int64_t* chunk) {
  const int64_t tb = (ntp + 255) / 256;
  int64_t nc = std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (4096 + tb - 1) / tb));
  *chunk = ((N + nc - 1) / nc + 255) / 256 * 256;
  *nchunk = (N + *chunk - 1) / *chunk;
}

int direct_forces_impl(const dfmm_plan* pl, const double* seg, const double* burg, int64_t nseg,
                       const int64_t* targets, int64_t ntgt, double* forces, int fp32, hipStream_t st) {
  const int nq = pl->quad.n;
  const int64_t N = nseg * nq, ntp = ntgt * nq;
  int64_t nchunk, chunk;
  direct_chunks(N, ntp, &nchunk, &chunk);
  double *pts = nullptr, *part = nullptr, *sig = nullptr;
  if (hipMalloc(&pts, sizeof(double) * 9 * N) != hipSuccess ||
      hipMalloc(&part, sizeof(double) * 6 * ntp * nchunk) != hipSuccess ||
      hipMalloc(&sig, sizeof(double) * 6 * ntp) != hipSuccess) {
    hipFree(pts);
    hipFree(part);
    hipFree(sig);
    set_error("direct_forces: cannot allocate scratch");
    return DFMM_E_NOMEM;
  }
  int rc = direct_core(pl, seg, burg, nseg, targets, ntgt, forces, fp32, st, pts, part, sig, (int*)sig, nchunk,
                       chunk);
  hipError_t e = hipStreamSynchronize(st);
  hipFree(pts);
  hipFree(part);
  hipFree(sig);
  if (rc == DFMM_OK && e != hipSuccess) {
    set_error(std::string("direct_forces: ") + hipGetErrorString(e));
    rc = DFMM_E_HIP;
  }
  return rc;
}

// ------------------------------------------- direct sum without allocation
// For callers that cannot allocate device memory (graph capture, tight
// serving loops): the same direct sum with its scratch in this file-scope
// array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): the device address is looked up once per device with
// hipGetSymbolAddress and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int scratch_ptr(void** out) {
  int dev = 0;
  DFMM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("direct_forces_noalloc: device index beyond the supported range");
    return DFMM_E_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("direct_forces_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return DFMM_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DFMM_OK;
}

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t direct_noalloc_bytes(const dfmm_plan* pl, int64_t nseg, int64_t ntgt) {
  const int nq = pl->quad.n;
  const int64_t N = nseg * nq, ntp = ntgt * nq;
  int64_t nchunk, chunk;
  direct_chunks(N, ntp, &nchunk, &chunk);
  return up256(sizeof(double) * 9 * N) + up256(sizeof(double) * 6 * ntp * nchunk) +
         up256(sizeof(double) * 6 * ntp);
}

int direct_forces_noalloc_impl(const dfmm_plan* pl, const double* seg, const double* burg, int64_t nseg,
                               const int64_t* targets, int64_t ntgt, double* forces, int fp32, hipStream_t st) {
  const size_t need = direct_noalloc_bytes(pl, nseg, ntgt);
  if (need > (size_t)kScratchBytes) {
    set_error("direct_forces_noalloc: needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string((long long)kScratchBytes) + " it has (fewer segments or targets, or the allocating call)");
    return DFMM_E_ARG;
  }
  void* base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  const int nq = pl->quad.n;
  const int64_t N = nseg * nq, ntp = ntgt * nq;
  int64_t nchunk, chunk;
  direct_chunks(N, ntp, &nchunk, &chunk);
  unsigned char* b = (unsigned char*)base;
  double* pts = (double*)b;
  double* part = (double*)(b + up256(sizeof(double) * 9 * N));
  double* sig = (double*)((unsigned char*)part + up256(sizeof(double) * 6 * ntp * nchunk));
  return direct_core(pl, seg, burg, nseg, targets, ntgt, forces, fp32, st, pts, part, sig, (int*)sig, nchunk, chunk);
}

}  // namespace dfmm
