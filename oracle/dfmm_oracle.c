/*
 * dfmm_oracle.c -- plain FP64 CPU oracle for the stress and Peach-Koehler
 * forces of straight dislocation segments (Chen, Aubry, Oppelstrup, Arsenlis,
 * Darve, "Fast algorithms for evaluating the stress field of dislocation lines
 * in anisotropic elastic media").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * Everything is double precision, written for readability rather than speed:
 *   - Gauss-Legendre rule (Sec. 2, Eq. stress_discrete, n-point quadrature)
 *   - stiffness tensor of a cubic (or isotropic) crystal
 *   - isotropic Green's function and its derivative (Eq. k_iso) with the
 *     non-singular replacement R -> R_a = sqrt(R^2 + a^2) (the paper cites the
 *     non-singular theory for this Green's function)
 *   - anisotropic Green's function derivative by trapezoid quadrature over the
 *     unit circle normal to the field direction (the paper evaluates the
 *     anisotropic Green's function numerically, Sec. 2; its spherical-harmonic
 *     coefficient tables are not reproduced here)
 *   - the 54-component kernel K = eps C C dG (Eq. kernel), negated so that the
 *     stress of a straight dislocation has the standard sign
 *   - the direct sum s(x_i) = sum_j K(x_i - y_j) q_j (Eq. stress3) with a
 *     Neumaier-compensated accumulation in fixed source order
 *   - forces at the two segment ends by Gauss quadrature of (sigma.b) x dS
 *     with linear shape functions (Sec. 1 and the Peach-Koehler formula, Sec. 2)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* Voigt order of the symmetric stress index pair (alpha, beta). */
static const int VA[6] = {0, 1, 2, 1, 0, 0};
static const int VB[6] = {0, 1, 2, 2, 2, 1};

static int C4(int i, int j, int k, int l) { return ((i * 3 + j) * 3 + k) * 3 + l; }

static double levi(int i, int j, int k) {
  if (i == j || j == k || i == k) return 0.0;
  /* even permutations of (0,1,2) */
  if ((i == 0 && j == 1 && k == 2) || (i == 1 && j == 2 && k == 0) ||
      (i == 2 && j == 0 && k == 1))
    return 1.0;
  return -1.0;
}

/* ---------------------------------------------------------------------- */
/* Gauss-Legendre nodes u[k] (ascending) and weights w[k] on [-1, 1].      */
/* Newton iteration on the Legendre polynomial P_n from the three-term     */
/* recurrence.                                                             */
void or_gauss_legendre(int n, double* u, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = cos(PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0; }
      /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    u[n - 1 - i] = x;
    w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

/* ---------------------------------------------------------------------- */
/* Stiffness C_ijkl of a cubic crystal in its cube axes:                   */
/* C_iiii = c11, C_iijj = c12 (i != j), C_ijij = C_ijji = c44 (i != j).    */
void or_stiffness(double c11, double c12, double c44, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double v = 0.0;
          if (i == j && k == l && i == k) v = c11;
          else if (i == j && k == l) v = c12;
          else if ((i == k && j == l) || (i == l && j == k)) v = c44;
          C[C4(i, j, k, l)] = v;
        }
}

/* Medium description shared by the routines below:
 * prm[0..2] = c11, c12, c44; prm[3] = core radius a; prm[4] = circle points. */
static int is_isotropic(const double* prm) {
  return fabs(2.0 * prm[2] - (prm[0] - prm[1])) <= 1e-12 * fabs(prm[2]);
}

/* Isotropic moduli (mu, nu) of the medium; for a cubic medium the Voigt
 * averages mu_V = (c11 - c12 + 3 c44)/5, lambda_V = (c11 + 4 c12 - 2 c44)/5. */
void or_voigt(const double* prm, double* mu, double* nu) {
  double c11 = prm[0], c12 = prm[1], c44 = prm[2];
  double m = (c11 - c12 + 3.0 * c44) / 5.0;
  double l = (c11 + 4.0 * c12 - 2.0 * c44) / 5.0;
  *mu = m;
  *nu = l / (2.0 * (l + m));
}

/* ---------------------------------------------------------------------- */
/* Isotropic Green's function, Eq. k_iso, with R replaced by R_a:          */
/* G_vp = [delta_vp lap(R_a) - d_v d_p R_a / (2(1-nu))] / (8 pi mu).       */
void or_G_iso(const double* x, double mu, double nu, double a, double* G) {
  double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double Ra = sqrt(r2 + a * a);
  double Ra3 = Ra * Ra * Ra;
  double lap = 2.0 / Ra + a * a / Ra3; /* sum_i d_i d_i R_a */
  double c = 1.0 / (8.0 * PI * mu);
  double h = 1.0 / (2.0 * (1.0 - nu));
  for (int v = 0; v < 3; ++v)
    for (int p = 0; p < 3; ++p) {
      double d2 = (v == p ? 1.0 / Ra : 0.0) - x[v] * x[p] / Ra3; /* d_v d_p R_a */
      G[v * 3 + p] = c * ((v == p ? lap : 0.0) - h * d2);
    }
}

/* D[(v*3+p)*3+q] = d_q G_vp of the function above. */
void or_dG_iso(const double* x, double mu, double nu, double a, double* D) {
  double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double Ra2 = r2 + a * a;
  if (Ra2 == 0.0) { memset(D, 0, 27 * sizeof(double)); return; }
  double Ra = sqrt(Ra2);
  double Ra3 = Ra * Ra2, Ra5 = Ra3 * Ra2;
  double c = 1.0 / (8.0 * PI * mu);
  double h = 1.0 / (2.0 * (1.0 - nu));
  for (int v = 0; v < 3; ++v)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        /* d_q lap(R_a) */
        double dlap = -2.0 * x[q] / Ra3 - 3.0 * a * a * x[q] / Ra5;
        /* d_v d_p d_q R_a */
        double d3 = -((v == p ? x[q] : 0.0) + (v == q ? x[p] : 0.0) + (p == q ? x[v] : 0.0)) / Ra3 +
                    3.0 * x[v] * x[p] * x[q] / Ra5;
        D[(v * 3 + p) * 3 + q] = c * ((v == p ? dlap : 0.0) - h * d3);
      }
}

/* ---------------------------------------------------------------------- */
/* Unit-circle quadrature for the anisotropic (singular) Green's function. */
/* With T = x/r and z(phi) = cos(phi) e1 + sin(phi) e2 on the unit circle  */
/* normal to T, and N(z)_ik = C_ijkl z_j z_l, M = N^{-1}:                  */
/*   G_ij   = 1/(8 pi^2 r)   int_0^{2pi} M_ij dphi                          */
/*   d_sG_ij = 1/(8 pi^2 r^2) int_0^{2pi} (z_s F_ij - T_s M_ij) dphi        */
/* with F = M A M and A_ik = C_ijkl (T_j z_l + z_j T_l).  The second line  */
/* follows from G = (1/8pi^2) int_{|k|=1} N(k)^{-1} delta(k.x) dk by       */
/* differentiating the delta function.  The trapezoid rule with nphi      */
/* equally spaced angles is used.                                          */
static void circle_basis(const double* T, double* e1, double* e2) {
  int m = 0;
  double am = fabs(T[0]);
  if (fabs(T[1]) < am) { m = 1; am = fabs(T[1]); }
  if (fabs(T[2]) < am) { m = 2; }
  double ax[3] = {0, 0, 0};
  ax[m] = 1.0;
  double d = ax[0] * T[0] + ax[1] * T[1] + ax[2] * T[2];
  for (int i = 0; i < 3; ++i) e1[i] = ax[i] - d * T[i];
  double n = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int i = 0; i < 3; ++i) e1[i] /= n;
  e2[0] = T[1] * e1[2] - T[2] * e1[1];
  e2[1] = T[2] * e1[0] - T[0] * e1[2];
  e2[2] = T[0] * e1[1] - T[1] * e1[0];
}

static void inv3(const double* A, double* B) {
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  double id = 1.0 / det;
  B[0] = c00 * id;
  B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = c01 * id;
  B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = c02 * id;
  B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

void or_G_circle(const double* x, const double* C, int nphi, double* G) {
  double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double T[3] = {x[0] / r, x[1] / r, x[2] / r}, e1[3], e2[3];
  circle_basis(T, e1, e2);
  double acc[9] = {0};
  for (int k = 0; k < nphi; ++k) {
    double ph = 2.0 * PI * k / nphi;
    double z[3];
    for (int i = 0; i < 3; ++i) z[i] = cos(ph) * e1[i] + sin(ph) * e2[i];
    double N[9] = {0}, M[9];
    for (int i = 0; i < 3; ++i)
      for (int kk = 0; kk < 3; ++kk)
        for (int j = 0; j < 3; ++j)
          for (int l = 0; l < 3; ++l) N[i * 3 + kk] += C[C4(i, j, kk, l)] * z[j] * z[l];
    inv3(N, M);
    for (int i = 0; i < 9; ++i) acc[i] += M[i];
  }
  double f = (2.0 * PI / nphi) / (8.0 * PI * PI * r);
  for (int i = 0; i < 9; ++i) G[i] = f * acc[i];
}

void or_dG_circle(const double* x, const double* C, int nphi, double* D) {
  double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  if (r2 == 0.0) { memset(D, 0, 27 * sizeof(double)); return; }
  double r = sqrt(r2);
  double T[3] = {x[0] / r, x[1] / r, x[2] / r}, e1[3], e2[3];
  circle_basis(T, e1, e2);
  double acc[27] = {0};
  for (int k = 0; k < nphi; ++k) {
    double ph = 2.0 * PI * k / nphi;
    double z[3];
    for (int i = 0; i < 3; ++i) z[i] = cos(ph) * e1[i] + sin(ph) * e2[i];
    double N[9] = {0}, M[9], A[9] = {0}, MA[9] = {0}, F[9] = {0};
    for (int i = 0; i < 3; ++i)
      for (int kk = 0; kk < 3; ++kk)
        for (int j = 0; j < 3; ++j)
          for (int l = 0; l < 3; ++l) {
            double c = C[C4(i, j, kk, l)];
            N[i * 3 + kk] += c * z[j] * z[l];
            A[i * 3 + kk] += c * (T[j] * z[l] + z[j] * T[l]);
          }
    inv3(N, M);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) MA[i * 3 + j] += M[i * 3 + l] * A[l * 3 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) F[i * 3 + j] += MA[i * 3 + l] * M[l * 3 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int s = 0; s < 3; ++s)
          acc[(i * 3 + j) * 3 + s] += z[s] * F[i * 3 + j] - T[s] * M[i * 3 + j];
  }
  double f = (2.0 * PI / nphi) / (8.0 * PI * PI * r2);
  for (int i = 0; i < 27; ++i) D[i] = f * acc[i];
}

/* ---------------------------------------------------------------------- */
/* Green's-function derivative of the medium with the non-singular core.  */
/* Isotropic medium: Eq. k_iso with R_a.  Cubic medium: the Voigt-average  */
/* isotropic derivative with core a, plus the anisotropic correction       */
/* (dG_circle - dG_iso_Voigt with a = 0) damped by (R/R_a)^3, which tends  */
/* to the singular anisotropic derivative for R >> a, vanishes at R = 0    */
/* and reduces exactly to the isotropic form when the medium is isotropic. */
void or_dG_medium(const double* x, const double* prm, double* D) {
  double a = prm[3];
  int nphi = (int)prm[4];
  if (is_isotropic(prm)) {
    double mu = prm[2], lam = prm[1];
    double nu = lam / (2.0 * (lam + mu));
    or_dG_iso(x, mu, nu, a, D);
    return;
  }
  double mu, nu;
  or_voigt(prm, &mu, &nu);
  or_dG_iso(x, mu, nu, a, D);
  double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  if (r2 == 0.0) return;
  double C[81], Dc[27], Di[27];
  or_stiffness(prm[0], prm[1], prm[2], C);
  or_dG_circle(x, C, nphi, Dc);
  or_dG_iso(x, mu, nu, 0.0, Di);
  double damp = pow(r2 / (r2 + a * a), 1.5);
  for (int i = 0; i < 27; ++i) D[i] += damp * (Dc[i] - Di[i]);
}

/* ---------------------------------------------------------------------- */
/* K[ab*9 + w*3 + r] = - eps_ngr C_{ab vg} C_{pqwn} d_qG_vp  (Eq. kernel,   */
/* negated), ab in Voigt order.  Evaluated as three successive contractions */
/* of the same expression.                                                  */
void or_kernel54(const double* D, const double* C, double* K) {
  double X[27]; /* X[v][w][n] = sum_pq C_pqwn D_vpq */
  for (int v = 0; v < 3; ++v)
    for (int w = 0; w < 3; ++w)
      for (int n = 0; n < 3; ++n) {
        double s = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) s += C[C4(p, q, w, n)] * D[(v * 3 + p) * 3 + q];
        X[(v * 3 + w) * 3 + n] = s;
      }
  double Y[81]; /* Y[v][g][w][r] = sum_n eps_ngr X[v][w][n] */
  for (int v = 0; v < 3; ++v)
    for (int g = 0; g < 3; ++g)
      for (int w = 0; w < 3; ++w)
        for (int r = 0; r < 3; ++r) {
          double s = 0.0;
          for (int n = 0; n < 3; ++n) s += levi(n, g, r) * X[(v * 3 + w) * 3 + n];
          Y[((v * 3 + g) * 3 + w) * 3 + r] = s;
        }
  for (int ab = 0; ab < 6; ++ab)
    for (int w = 0; w < 3; ++w)
      for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int v = 0; v < 3; ++v)
          for (int g = 0; g < 3; ++g)
            s += C[C4(VA[ab], VB[ab], v, g)] * Y[((v * 3 + g) * 3 + w) * 3 + r];
        K[ab * 9 + w * 3 + r] = -s;
      }
}

/* K at n displacement vectors x[n][3] for the medium prm. */
void or_kernel_batch(int64_t n, const double* x, const double* prm, double* K) {
  double C[81];
  or_stiffness(prm[0], prm[1], prm[2], C);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double D[27];
    or_dG_medium(x + 3 * i, prm, D);
    or_kernel54(D, C, K + 54 * i);
  }
}

/* ---------------------------------------------------------------------- */
/* Neumaier-compensated running sum.                                       */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double t) {
  double u = a->s + t;
  if (fabs(a->s) >= fabs(t)) a->c += (a->s - u) + t;
  else a->c += (t - u) + a->s;
  a->s = u;
}

/* Stress s(x_i) = sum_j K(x_i - y_j) q_j, Eq. stress3, at n_t targets     */
/* from n_s sources with 9-component strengths q[j][w*3+r].  The sources   */
/* are taken in fixed chunks of OR_CHUNK; each chunk is summed in order     */
/* with Neumaier compensation and the chunk sums are combined in order, so  */
/* the result does not depend on the number of threads or of targets.      */
#define OR_CHUNK 8192
void or_stress(int64_t n_t, const double* xt, int64_t n_s, const double* ys,
               const double* q, const double* prm, double* sigma) {
  double C[81];
  or_stiffness(prm[0], prm[1], prm[2], C);
  int64_t nch = (n_s + OR_CHUNK - 1) / OR_CHUNK;
  if (nch < 1) nch = 1;
  int64_t tb = (int64_t)(1 << 22) / nch; /* targets per batch: bounded scratch */
  if (tb < 1) tb = 1;
  nsum* part = (nsum*)malloc(sizeof(nsum) * 6 * nch * (tb < n_t ? tb : n_t));
  for (int64_t t0 = 0; t0 < n_t; t0 += tb) {
    int64_t nb = (n_t - t0 < tb) ? n_t - t0 : tb;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int64_t ii = 0; ii < nb; ++ii)
      for (int64_t ch = 0; ch < nch; ++ch) {
        int64_t i = t0 + ii;
        nsum acc[6];
        memset(acc, 0, sizeof(acc));
        int64_t j1 = (ch + 1) * OR_CHUNK < n_s ? (ch + 1) * OR_CHUNK : n_s;
        for (int64_t j = ch * OR_CHUNK; j < j1; ++j) {
          double d[3] = {xt[3 * i] - ys[3 * j], xt[3 * i + 1] - ys[3 * j + 1],
                         xt[3 * i + 2] - ys[3 * j + 2]};
          double D[27], K[54];
          or_dG_medium(d, prm, D);
          or_kernel54(D, C, K);
          for (int ab = 0; ab < 6; ++ab) {
            double s = 0.0;
            for (int k = 0; k < 9; ++k) s += K[ab * 9 + k] * q[9 * j + k];
            nadd(&acc[ab], s);
          }
        }
        memcpy(part + (ii * nch + ch) * 6, acc, sizeof(acc));
      }
    for (int64_t ii = 0; ii < nb; ++ii) {
      nsum tot[6];
      memset(tot, 0, sizeof(tot));
      for (int64_t ch = 0; ch < nch; ++ch)
        for (int ab = 0; ab < 6; ++ab) {
          nadd(&tot[ab], part[(ii * nch + ch) * 6 + ab].s);
          nadd(&tot[ab], part[(ii * nch + ch) * 6 + ab].c);
        }
      for (int ab = 0; ab < 6; ++ab) sigma[6 * (t0 + ii) + ab] = tot[ab].s + tot[ab].c;
    }
  }
  free(part);
}

/* Quadrature points y_ik = x1 + (1+u_k)/2 dS_i and strengths               */
/* q_ik[w*3+r] = (1/2) omega_k b_w dS_r, Eq. stress_discrete.               */
void or_points(int64_t n_seg, const double* seg, const double* burg, int nq,
               double* y, double* q) {
  double u[64], w[64];
  or_gauss_legendre(nq, u, w);
  for (int64_t i = 0; i < n_seg; ++i) {
    const double* x1 = seg + 6 * i;
    const double* x2 = seg + 6 * i + 3;
    double dS[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
    for (int k = 0; k < nq; ++k) {
      int64_t j = i * nq + k;
      for (int c = 0; c < 3; ++c) y[3 * j + c] = x1[c] + 0.5 * (1.0 + u[k]) * dS[c];
      for (int ww = 0; ww < 3; ++ww)
        for (int r = 0; r < 3; ++r) q[9 * j + ww * 3 + r] = 0.5 * w[k] * burg[3 * i + ww] * dS[r];
    }
  }
}

/* Forces at both ends of the target segments from the stress at their    */
/* quadrature points: f^(1) = sum_k (omega_k/2)(1-s_k) (sigma_k.b) x dS,   */
/* f^(2) = sum_k (omega_k/2) s_k (sigma_k.b) x dS, s_k = (1+u_k)/2.         */
/* sig_t[(t*nq+k)*6 + ab] is the stress at point k of target t.            */
void or_assemble_forces(int64_t n_t, const int64_t* tgt, const double* seg,
                        const double* burg, int nq, const double* sig_t, double* f) {
  double u[64], w[64];
  or_gauss_legendre(nq, u, w);
  for (int64_t t = 0; t < n_t; ++t) {
    int64_t i = tgt[t];
    const double* x1 = seg + 6 * i;
    const double* x2 = seg + 6 * i + 3;
    const double* b = burg + 3 * i;
    double dS[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
    double f1[3] = {0, 0, 0}, f2[3] = {0, 0, 0};
    for (int k = 0; k < nq; ++k) {
      const double* s = sig_t + (t * nq + k) * 6;
      double S[3][3] = {{s[0], s[5], s[4]}, {s[5], s[1], s[3]}, {s[4], s[3], s[2]}};
      double sb[3];
      for (int c = 0; c < 3; ++c) sb[c] = S[c][0] * b[0] + S[c][1] * b[1] + S[c][2] * b[2];
      double fx[3] = {sb[1] * dS[2] - sb[2] * dS[1], sb[2] * dS[0] - sb[0] * dS[2],
                      sb[0] * dS[1] - sb[1] * dS[0]};
      double sk = 0.5 * (1.0 + u[k]);
      for (int c = 0; c < 3; ++c) {
        f1[c] += 0.5 * w[k] * (1.0 - sk) * fx[c];
        f2[c] += 0.5 * w[k] * sk * fx[c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      f[6 * t + c] = f1[c];
      f[6 * t + 3 + c] = f2[c];
    }
  }
}

/* Direct O(N^2) forces on the target segments tgt[0..n_t) from all n_seg  */
/* segments (every quadrature point of every segment is a source, the      */
/* segment's own points included).  f[t][2][3].                             */
int or_forces(int64_t n_seg, const double* seg, const double* burg, const double* prm,
              int nq, int64_t n_t, const int64_t* tgt, double* f) {
  int64_t N = n_seg * nq;
  double* y = (double*)malloc(sizeof(double) * 3 * N);
  double* q = (double*)malloc(sizeof(double) * 9 * N);
  double* xt = (double*)malloc(sizeof(double) * 3 * n_t * nq);
  double* sg = (double*)malloc(sizeof(double) * 6 * n_t * nq);
  if (!y || !q || !xt || !sg) { free(y); free(q); free(xt); free(sg); return -1; }
  or_points(n_seg, seg, burg, nq, y, q);
  for (int64_t t = 0; t < n_t; ++t)
    for (int k = 0; k < nq; ++k)
      for (int c = 0; c < 3; ++c) xt[3 * (t * nq + k) + c] = y[3 * (tgt[t] * nq + k) + c];
  or_stress(n_t * nq, xt, N, y, q, prm, sg);
  or_assemble_forces(n_t, tgt, seg, burg, nq, sg, f);
  free(y); free(q); free(xt); free(sg);
  return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
