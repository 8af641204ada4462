// Device-side evaluation of the dislocation kernel (Sec. 2).
//
//  * dG_iso: derivative of the isotropic Green's function of Eq. k_iso with
//    R replaced by R_a = sqrt(R^2 + a^2) (non-singular core):
//      G_vp = [delta_vp lap(R_a) - d_v d_p R_a / (2(1-nu))] / (8 pi mu).
//  * dG_circle: singular anisotropic derivative by the trapezoid rule on the
//    unit circle normal to T = x/r (the anisotropic Green's function has no
//    closed form and is evaluated numerically, Sec. 2):
//      d_s G_ij = 1/(8 pi^2 r^2) int_0^{2 pi} (z_s F_ij - T_s M_ij) dphi,
//      M = (zCz)^-1, F = M A M, A_ik = C_ijkl (T_j z_l + z_j T_l).
//    The integrand has period pi, so the nphi-point rule is evaluated on
//    nphi/2 angles in [0, pi) and doubled.
//  * dG_medium: for a cubic medium the non-singular form
//      dG_a = dG_iso_a[Voigt] + (R/R_a)^3 (dG_circle - dG_iso_0[Voigt]);
//    for an isotropic medium the closed form alone.
//  * contract_b_t: stress of one source point with rank-one strength
//    q = b (x) t (t = (omega/2) dS) through K = -eps C C dG (Eq. kernel,
//    negated), using the cubic form of C:
//      C_ijkl = c12 d_ij d_kl + c44 (d_ik d_jl + d_il d_jk) + h d_ijkl,
//      h = c11 - c12 - 2 c44.
#pragma once
#include <hip/hip_runtime.h>

namespace dfmm {

template <typename T>
struct Med {
  T c12, c44, hh;   // cubic constants (hh = c11 - c12 - 2 c44)
  T a;              // core radius
  T mu, nu;         // isotropic moduli (the medium's, or its Voigt average)
  int iso;          // 1: closed form only
  int nhalf;        // circle angles on [0, pi)
  const T* cs;      // cos/sin of 2 pi k / (2 nhalf), k < nhalf, interleaved
};

template <typename T>
__device__ __forceinline__ T fast_rcp(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);  // 1 ulp: ample for the float evaluation
}
// double: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each squares the relative error), within an ulp or
// two of 1/x, not correctly rounded; every argument here is a positive
// normal number (2 (1 - nu), the determinant of a positive definite matrix)
template <>
__device__ __forceinline__ double fast_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <typename T>
__device__ __forceinline__ T fast_rsqrt(T x) {
  return T(1) / sqrt(x);
}
template <>
__device__ __forceinline__ float fast_rsqrt<float>(float x) {
  return __builtin_amdgcn_rsqf(x);  // 1 ulp, as above
}
// a / b: exact in double, a times the 1-ulp reciprocal in float
template <typename T>
__device__ __forceinline__ T fast_div(T a, T b) {
  return a / b;
}
template <>
__device__ __forceinline__ float fast_div<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}

// D[(v*3+p)*3+q] += scale * d_q G_vp (isotropic, core a).
template <typename T>
__device__ __forceinline__ void dg_iso_acc(T x0, T x1, T x2, T mu, T nu, T a, T scale, T* D) {
  T x[3] = {x0, x1, x2};
  T r2 = x0 * x0 + x1 * x1 + x2 * x2;
  T ra2 = r2 + a * a;
  if (ra2 == T(0)) return;
  T ira = fast_rsqrt(ra2);
  T ira2 = ira * ira;
  T ira3 = ira * ira2;
  T ira5 = ira3 * ira2;
  T c = fast_div(scale, T(8) * T(3.14159265358979323846) * mu);
  T h = fast_rcp(T(2) * (T(1) - nu));
  T dl = -(T(2) * ira3 + T(3) * a * a * ira5);  // d_q lap(R_a) = dl * x_q
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        T d3 = T(3) * x[v] * x[p] * x[q] * ira5;
        T lin = T(0);
        if (v == p) lin += x[q];
        if (v == q) lin += x[p];
        if (p == q) lin += x[v];
        d3 -= lin * ira3;
        T val = -h * d3;
        if (v == p) val += dl * x[q];
        D[(v * 3 + p) * 3 + q] += c * val;
      }
}

// D += scale * (singular anisotropic d_q G_vp) by circle quadrature.  Only
// the (i <= j) half of the symmetric index pair is accumulated.
template <typename T>
__device__ __forceinline__ void dg_circle_acc(T x0, T x1, T x2, const Med<T>& m, T scale, T* D) {
  T r2 = x0 * x0 + x1 * x1 + x2 * x2;
  if (r2 == T(0)) return;
  T ir = fast_rsqrt(r2);
  T t[3] = {x0 * ir, x1 * ir, x2 * ir};
  // e1: the axis least aligned with T, made orthogonal to T; e2 = T x e1
  int ax = 0;
  T am = fabs(t[0]);
  if (fabs(t[1]) < am) { ax = 1; am = fabs(t[1]); }
  if (fabs(t[2]) < am) ax = 2;
  T e1[3] = {-t[ax] * t[0], -t[ax] * t[1], -t[ax] * t[2]};
  e1[ax] += T(1);
  T n1 = fast_rsqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  e1[0] *= n1; e1[1] *= n1; e1[2] *= n1;
  T e2[3] = {t[1] * e1[2] - t[2] * e1[1], t[2] * e1[0] - t[0] * e1[2], t[0] * e1[1] - t[1] * e1[0]};
  const T cc = m.c12 + m.c44, c44 = m.c44, ch = cc + m.hh;
  const T ct[3] = {cc * t[0], cc * t[1], cc * t[2]};
  const T dt[3] = {T(2) * ch * t[0], T(2) * ch * t[1], T(2) * ch * t[2]};
  // symmetric pairs (i, j): 00 11 22 01 02 12
  constexpr int PI_[6] = {0, 1, 2, 0, 0, 1}, PJ_[6] = {0, 1, 2, 1, 2, 2};
  // z = cos(phi) e1 + sin(phi) e2 and T are fixed vectors times scalars, so
  // the sums of z_s F_ij and T_s M_ij are formed as sum cos F_ij, sum sin F_ij
  // and sum M_ij (18 accumulations per angle instead of 36), and the vectors
  // are applied once after the loop.
  T acc_c[6], acc_s[6], acc_m[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) acc_c[i] = acc_s[i] = acc_m[i] = T(0);
#pragma unroll 1
  for (int k = 0; k < m.nhalf; ++k) {
    T co = m.cs[2 * k], si = m.cs[2 * k + 1];
    T z[3] = {co * e1[0] + si * e2[0], co * e1[1] + si * e2[1], co * e1[2] + si * e2[2]};
    // N = (c12 + c44) z z^T + diag(c44 + hh z_i^2): diagonal (c12 + c44 + hh) z_i^2 + c44
    T N00 = ch * z[0] * z[0] + c44, N11 = ch * z[1] * z[1] + c44, N22 = ch * z[2] * z[2] + c44;
    T N01 = cc * z[0] * z[1], N02 = cc * z[0] * z[2], N12 = cc * z[1] * z[2];
    T m00 = N11 * N22 - N12 * N12, m01 = N02 * N12 - N01 * N22, m02 = N01 * N12 - N02 * N11;
    T m11 = N00 * N22 - N02 * N02, m12 = N01 * N02 - N00 * N12, m22 = N00 * N11 - N01 * N01;
    T idet = fast_rcp(N00 * m00 + N01 * m01 + N02 * m02);
    T M[9] = {m00 * idet, m01 * idet, m02 * idet, m01 * idet, m11 * idet,
              m12 * idet, m02 * idet, m12 * idet, m22 * idet};
    // A = (c12 + c44)(T z^T + z T^T) + 2 hh diag(T_i z_i)
    T A[9];
    A[0] = dt[0] * z[0];
    A[4] = dt[1] * z[1];
    A[8] = dt[2] * z[2];
    A[1] = A[3] = ct[0] * z[1] + z[0] * ct[1];
    A[2] = A[6] = ct[0] * z[2] + z[0] * ct[2];
    A[5] = A[7] = ct[1] * z[2] + z[1] * ct[2];
    T P[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P[i * 3 + j] = M[i * 3] * A[j] + M[i * 3 + 1] * A[3 + j] + M[i * 3 + 2] * A[6 + j];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int i = PI_[q], j = PJ_[q];
      T F = P[i * 3] * M[j] + P[i * 3 + 1] * M[3 + j] + P[i * 3 + 2] * M[6 + j];
      acc_c[q] = fma(co, F, acc_c[q]);
      acc_s[q] = fma(si, F, acc_s[q]);
      acc_m[q] += M[i * 3 + j];
    }
  }
  T acc[18];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int s = 0; s < 3; ++s) acc[q * 3 + s] = e1[s] * acc_c[q] + e2[s] * acc_s[q] - t[s] * acc_m[q];
  // (2 pi / nphi) * 2 / (8 pi^2 r^2) with nphi = 2 nhalf
  T f = fast_div(scale, T(2) * T(3.14159265358979323846) * T(2 * m.nhalf) * r2);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int i = PI_[q], j = PJ_[q];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      D[(i * 3 + j) * 3 + s] += f * acc[q * 3 + s];
      if (i != j) D[(j * 3 + i) * 3 + s] += f * acc[q * 3 + s];
    }
  }
}

template <typename T>
__device__ __forceinline__ void dg_medium(T x0, T x1, T x2, const Med<T>& m, T* D) {
#pragma unroll
  for (int i = 0; i < 27; ++i) D[i] = T(0);
  // the circle rule first, while D is still zero (keeps D out of the
  // registers live across the angle loop), then the closed-form terms
  T damp = T(0);
  if (!m.iso) {
    T r2 = x0 * x0 + x1 * x1 + x2 * x2;
    if (r2 > T(0)) {
      T q = fast_div(r2, r2 + m.a * m.a);
      damp = q * sqrt(q);
      dg_circle_acc(x0, x1, x2, m, damp, D);
    }
  }
  dg_iso_acc(x0, x1, x2, m.mu, m.nu, m.a, T(1), D);
  if (damp != T(0)) dg_iso_acc(x0, x1, x2, m.mu, m.nu, T(0), -damp, D);
}

// dg_medium with the isotropic/anisotropic branch fixed at compile time.
template <typename T, bool ISO>
__device__ __forceinline__ void dg_medium_t(T x0, T x1, T x2, const Med<T>& m, T* D) {
  if (ISO) {
#pragma unroll
    for (int i = 0; i < 27; ++i) D[i] = T(0);
    dg_iso_acc(x0, x1, x2, m.mu, m.nu, m.a, T(1), D);
  } else {
    dg_medium(x0, x1, x2, m, D);
  }
}

// sig[6] += stress of a source with strength b (x) t seen through dG (D).
template <typename T>
__device__ __forceinline__ void contract_b_t(const T* D, T c12, T c44, T hh, const T* b, const T* t,
                                             T* sig) {
  T F[9];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const T* Dv = D + v * 9;  // Dv[p*3+q] = d_q G_vp
    T tr = Dv[0] + Dv[4] + Dv[8];
    T E[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      T s1 = b[0] * Dv[0 * 3 + n] + b[1] * Dv[1 * 3 + n] + b[2] * Dv[2 * 3 + n];  // sum_p b_p D_vpn
      T s2 = b[0] * Dv[n * 3 + 0] + b[1] * Dv[n * 3 + 1] + b[2] * Dv[n * 3 + 2];  // sum_q b_q D_vnq
      E[n] = c12 * b[n] * tr + c44 * (s1 + s2) + hh * b[n] * Dv[n * 3 + n];
    }
    // F_vg = (t x E_v)_g
    F[v * 3 + 0] = t[1] * E[2] - t[2] * E[1];
    F[v * 3 + 1] = t[2] * E[0] - t[0] * E[2];
    F[v * 3 + 2] = t[0] * E[1] - t[1] * E[0];
  }
  T trF = F[0] + F[4] + F[8];
  sig[0] -= c12 * trF + (T(2) * c44 + hh) * F[0];
  sig[1] -= c12 * trF + (T(2) * c44 + hh) * F[4];
  sig[2] -= c12 * trF + (T(2) * c44 + hh) * F[8];
  sig[3] -= c44 * (F[5] + F[7]);
  sig[4] -= c44 * (F[2] + F[6]);
  sig[5] -= c44 * (F[1] + F[3]);
}

}  // namespace dfmm
