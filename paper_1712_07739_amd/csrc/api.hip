// C ABI of libdfmm: argument checking, object lifetime, error reporting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace dfmm {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

// Gauss-Legendre nodes and weights on [-1, 1] from the Jacobi matrix of the
// Legendre polynomials (zero diagonal, off-diagonal b_k = k / sqrt(4k^2 - 1)):
// the nodes are its eigenvalues, found one by one by bisection on the Sturm
// count of the LDL^T pivots of J - x I; the weight of a node x is the
// Christoffel number 1 / sum_k phi_k(x)^2 over the orthonormal polynomials
// phi_0 .. phi_{n-1}, which the same b_k generate.
static void gauss_legendre(int n, double* u, double* w) {
  auto beta = [](int k) { return k / std::sqrt(4.0 * k * k - 1.0); };
  auto below = [&](double x) {  // eigenvalues of J smaller than x
    int c = 0;
    double d = -x;
    for (int k = 0; k < n; ++k) {
      if (k > 0) d = -x - beta(k) * beta(k) / d;
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++c;
    }
    return c;
  };
  for (int i = 0; i < n; ++i) {
    double lo = -1.0, hi = 1.0;  // the i-th smallest eigenvalue lies in [lo, hi)
    while (hi - lo > 0.0) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (below(mid) > i)
        hi = mid;
      else
        lo = mid;
    }
    const double x = 0.5 * (lo + hi);
    double prev = 0.0, cur = 1.0 / std::sqrt(2.0), sum = cur * cur;
    for (int k = 0; k + 1 < n; ++k) {
      const double next = (x * cur - (k > 0 ? beta(k) * prev : 0.0)) / beta(k + 1);
      prev = cur;
      cur = next;
      sum += cur * cur;
    }
    u[i] = x;
    w[i] = 1.0 / sum;
  }
}
}  // namespace dfmm

using namespace dfmm;

extern "C" {

void dfmm_default_params(dfmm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->order = 5;
  p->depth = 4;
  double mu = 1.0, nu = 0.3, lam = 2 * mu * nu / (1 - 2 * nu);
  p->c11 = lam + 2 * mu;
  p->c12 = lam;
  p->c44 = mu;
  p->core_a = 1e-3;
  p->box_lo[0] = p->box_lo[1] = p->box_lo[2] = -0.05;
  p->box_size = 1.1;
  p->n_quad = 3;
  p->n_circle = 64;
  p->precision = DFMM_FP64;
  p->m2l_mode = DFMM_M2L_FFT;
  p->aniso_kernel = DFMM_KERNEL_EXACT;
  p->lsq_degree = 0;
  p->leaf_max = 0;
  p->freq_chunks = 0;
}

const char* dfmm_status_string(int s) {
  switch (s) {
    case DFMM_OK: return "ok";
    case DFMM_E_ARG: return "invalid argument";
    case DFMM_E_NOMEM: return "out of memory";
    case DFMM_E_HIP: return "HIP error";
    case DFMM_E_OUT_OF_BOX: return "point outside the root cube";
    case DFMM_E_NONFINITE: return "non-finite coordinate";
    case DFMM_E_STATE: return "objects do not belong together";
    default: return "unknown status";
  }
}

const char* dfmm_last_error(void) { return g_err.c_str(); }

int dfmm_fmm_setup(const dfmm_params* prm, void* stream, dfmm_plan** out) {
  if (!prm || !out) { set_error("fmm_setup: null argument"); return DFMM_E_ARG; }
  *out = nullptr;
  const dfmm_params& q = *prm;
  if (q.order < 2 || q.order > kMaxOrder) { set_error("fmm_setup: order must be in [2, 8]"); return DFMM_E_ARG; }
  if (q.depth < 2 || q.depth > 10) { set_error("fmm_setup: depth must be in [2, 10]"); return DFMM_E_ARG; }
  if (q.n_quad < 1 || q.n_quad > kMaxQuad) { set_error("fmm_setup: n_quad must be in [1, 8]"); return DFMM_E_ARG; }
  if (q.n_circle < 8 || q.n_circle > 256 || (q.n_circle & 1)) {
    set_error("fmm_setup: n_circle must be even and in [8, 256]");
    return DFMM_E_ARG;
  }
  if (!(q.box_size > 0) || !std::isfinite(q.box_size) || !std::isfinite(q.box_lo[0]) ||
      !std::isfinite(q.box_lo[1]) || !std::isfinite(q.box_lo[2])) {
    set_error("fmm_setup: invalid root cube");
    return DFMM_E_ARG;
  }
  if (!(q.core_a >= 0) || !std::isfinite(q.core_a)) { set_error("fmm_setup: core_a must be >= 0"); return DFMM_E_ARG; }
  // cubic stiffness positive definite: c44 > 0, c11 - c12 > 0, c11 + 2 c12 > 0
  if (!(q.c44 > 0 && q.c11 - q.c12 > 0 && q.c11 + 2 * q.c12 > 0)) {
    set_error("fmm_setup: stiffness is not positive definite");
    return DFMM_E_ARG;
  }
  if (q.precision != DFMM_FP64 && q.precision != DFMM_MIXED && q.precision != DFMM_MIXED_F16) {
    set_error("fmm_setup: precision must be DFMM_FP64, DFMM_MIXED or DFMM_MIXED_F16");
    return DFMM_E_ARG;
  }
  if (q.m2l_mode != DFMM_M2L_FFT && q.m2l_mode != DFMM_M2L_FFT_SYM) {
    set_error("fmm_setup: m2l_mode must be DFMM_M2L_FFT or DFMM_M2L_FFT_SYM");
    return DFMM_E_ARG;
  }
  if (q.leaf_max < 0) { set_error("fmm_setup: leaf_max must be >= 0"); return DFMM_E_ARG; }
  if (q.freq_chunks < 0) { set_error("fmm_setup: freq_chunks must be >= 0"); return DFMM_E_ARG; }
  if (q.leaf_max > 0 && (q.lsq_degree != 0 || q.aniso_kernel != DFMM_KERNEL_EXACT)) {
    set_error("fmm_setup: the adaptive tree (leaf_max > 0) takes Lagrange interpolation and the exact kernel");
    return DFMM_E_ARG;
  }
  if (q.lsq_degree < DFMM_LSQ_AUTO || q.lsq_degree > q.order - 1) {
    set_error("fmm_setup: lsq_degree must be DFMM_LSQ_AUTO, 0 (Lagrange) or in [1, order - 1]");
    return DFMM_E_ARG;
  }
  if (q.aniso_kernel != DFMM_KERNEL_EXACT && q.aniso_kernel != DFMM_KERNEL_SURROGATE) {
    set_error("fmm_setup: aniso_kernel must be DFMM_KERNEL_EXACT or DFMM_KERNEL_SURROGATE");
    return DFMM_E_ARG;
  }
  auto t0 = std::chrono::steady_clock::now();
  dfmm_plan* pl = new dfmm_plan();
  pl->prm = q;
  pl->p = q.order;
  pl->n = 2 * q.order - 1;
  pl->nf = pl->n * pl->n * q.order;
  pl->D = q.depth;
  pl->mixed = q.precision != DFMM_FP64;
  pl->h16 = q.precision == DFMM_MIXED_F16;
  if (q.lsq_degree == DFMM_LSQ_AUTO) {  // largest d < 2 sqrt(p)
    int d = 0;
    while ((d + 1) * (d + 1) < 4 * q.order) ++d;
    pl->lsq = std::min(d, q.order - 1);
  } else {
    pl->lsq = q.lsq_degree;
  }
  if (pl->lsq == q.order - 1) pl->lsq = 0;  // the fit through all p nodes is the interpolant
  pl->sym = q.m2l_mode == DFMM_M2L_FFT_SYM;
  pl->iso = std::fabs(2.0 * q.c44 - (q.c11 - q.c12)) <= 1e-12 * std::fabs(q.c44);
  if (pl->iso) {
    pl->mu = q.c44;
    pl->nu = q.c12 / (2.0 * (q.c12 + q.c44));
  } else {
    double mv = (q.c11 - q.c12 + 3 * q.c44) / 5.0, lv = (q.c11 + 4 * q.c12 - 2 * q.c44) / 5.0;
    pl->mu = mv;
    pl->nu = lv / (2.0 * (lv + mv));
  }
  pl->quad.n = q.n_quad;
  gauss_legendre(q.n_quad, pl->quad.u, pl->quad.w);
  hipGetDevice(&pl->device);
  int rc = setup_tables(pl, (hipStream_t)stream);
  if (rc == DFMM_OK && q.aniso_kernel == DFMM_KERNEL_SURROGATE && !pl->iso) {
    dfmm_surrogate_cfg cfg;
    dfmm_surrogate_default_cfg(&cfg);
    rc = surrogate_train(pl, cfg, (hipStream_t)stream);
    if (rc == DFMM_OK) {
      pl->sur.in_use = 1;
      rc = build_spectra(pl, (hipStream_t)stream);
    }
  }
  if (rc) {
    dfmm_plan_destroy(pl);
    return rc;
  }
  pl->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = pl;
  return DFMM_OK;
}

void dfmm_plan_destroy(dfmm_plan* pl) {
  if (!pl) return;
  hipFree(pl->sur.w); hipFree(pl->sur.g); hipFree(pl->sur.m); hipFree(pl->sur.v); hipFree(pl->sur.mask);
  hipFree(pl->sur.wi); hipFree(pl->sur.bi); hipFree(pl->sur.split);
  for (auto& l : pl->lev) hipFree(l.khat);
  hipFree(pl->t64.S); hipFree(pl->t64.cs); hipFree(pl->t64.tw); hipFree(pl->t64.Pm); hipFree(pl->t32.Pm);
  hipFree(pl->t32.S); hipFree(pl->t32.cs); hipFree(pl->t32.tw);
  hipFree(pl->oid343); hipFree(pl->off158); hipFree(pl->cls16); hipFree(pl->symtab);
  delete pl;
}

int dfmm_build_tree(dfmm_plan* plan, const double* seg, int64_t n_seg, void* stream, dfmm_tree** out) {
  if (!plan || !seg || !out || n_seg < 1) { set_error("build_tree: invalid argument"); return DFMM_E_ARG; }
  *out = nullptr;
  dfmm_tree* t = new dfmm_tree();
  int rc = build_tree_impl(plan, seg, n_seg, (hipStream_t)stream, t);
  if (rc) {
    dfmm_tree_destroy(t);
    return rc;
  }
  *out = t;
  return DFMM_OK;
}

void dfmm_tree_destroy(dfmm_tree* t) {
  if (!t) return;
  if (t->done_set) hipEventSynchronize(t->done);
  if (t->done) hipEventDestroy(t->done);
  if (t->side) {
    hipStreamSynchronize(t->side);
    hipStreamDestroy(t->side);
  }
  if (t->fork) hipEventDestroy(t->fork);
  if (t->join) hipEventDestroy(t->join);
  hipFree(t->perm); hipFree(t->inv); hipFree(t->nbr);
  for (auto& L : t->lv) {
    hipFree(L.key); hipFree(L.first); hipFree(L.count); hipFree(L.parent); hipFree(L.il_start); hipFree(L.il); hipFree(L.order);
    hipFree(L.ilw); hipFree(L.wbase); hipFree(L.lenq);
  }
  hipFree(t->cstart); hipFree(t->cpair); hipFree(t->cval); hipFree(t->part); hipFree(t->cuni); hipFree(t->bigp);
  hipFree(t->pos0); hipFree(t->chk);
  hipFree(t->pts); hipFree(t->pleaf); hipFree(t->W); hipFree(t->s); hipFree(t->What); hipFree(t->Shat); hipFree(t->sig);
  hipFree(t->kexp); hipFree(t->wmax);
  hipFree(t->gl_cell); hipFree(t->gl_pf); hipFree(t->gl_pc); hipFree(t->gkey); hipFree(t->glev); hipFree(t->gord);
  hipFree(t->ustart); hipFree(t->usrc); hipFree(t->wstart); hipFree(t->wsrc); hipFree(t->xstart); hipFree(t->xsrc);
  hipFree(t->xcells); hipFree(t->wleaves); hipFree(t->gsf); hipFree(t->gsn); hipFree(t->dstart); hipFree(t->drange);
  delete t;
}

int dfmm_fmm_forces(const dfmm_plan* plan, dfmm_tree* tree, const double* seg, const double* burgers,
                    double* forces, void* stream) {
  if (!plan || !tree || !seg || !burgers || !forces) { set_error("fmm_forces: null argument"); return DFMM_E_ARG; }
  if (tree->plan != plan) { set_error("fmm_forces: tree was built with another plan"); return DFMM_E_STATE; }
  return fmm_forces_impl(plan, tree, seg, burgers, forces, (hipStream_t)stream);
}

int dfmm_tree_check_positions(const dfmm_plan* plan, dfmm_tree* tree, const double* seg, void* stream) {
  if (!plan || !tree || !seg) { set_error("tree_check_positions: null argument"); return DFMM_E_ARG; }
  if (tree->plan != plan) { set_error("tree_check_positions: tree was built with another plan"); return DFMM_E_STATE; }
  return check_positions_impl(plan, tree, seg, (hipStream_t)stream);
}

int dfmm_direct_forces(const dfmm_plan* plan, const double* seg, const double* burgers, int64_t n_seg,
                       const int64_t* targets, int64_t n_targets, double* forces, int fp32, void* stream) {
  if (!plan || !seg || !burgers || !forces || n_seg < 1 || n_targets < 1) {
    set_error("direct_forces: invalid argument");
    return DFMM_E_ARG;
  }
  if (!targets && n_targets != n_seg) {
    set_error("direct_forces: without a target list n_targets must equal n_seg");
    return DFMM_E_ARG;
  }
  return direct_forces_impl(plan, seg, burgers, n_seg, targets, n_targets, forces, fp32 ? 1 : 0,
                            (hipStream_t)stream);
}

int dfmm_direct_forces_noalloc(const dfmm_plan* plan, const double* seg, const double* burgers, int64_t n_seg,
                               const int64_t* targets, int64_t n_targets, double* forces, int fp32, void* stream) {
  if (!plan || !seg || !burgers || !forces || n_seg < 1 || n_targets < 1) {
    set_error("direct_forces_noalloc: invalid argument");
    return DFMM_E_ARG;
  }
  if (!targets && n_targets != n_seg) {
    set_error("direct_forces_noalloc: without a target list n_targets must equal n_seg");
    return DFMM_E_ARG;
  }
  return direct_forces_noalloc_impl(plan, seg, burgers, n_seg, targets, n_targets, forces, fp32 ? 1 : 0,
                                    (hipStream_t)stream);
}

size_t dfmm_direct_noalloc_bytes(const dfmm_plan* plan, int64_t n_seg, int64_t n_targets) {
  if (!plan || n_seg < 1 || n_targets < 1) return 0;
  return direct_noalloc_bytes(plan, n_seg, n_targets);
}

int dfmm_tree_set_timing(dfmm_tree* t, int on) {
  if (!t) { set_error("tree_set_timing: null tree"); return DFMM_E_ARG; }
  t->timing = on ? 1 : 0;
  for (double& x : t->stage_ms) x = 0;
  t->timed_calls = 0;
  return DFMM_OK;
}

int dfmm_tree_stage_times(dfmm_tree* t, double* ms, int* n_calls) {
  if (!t || !ms) { set_error("tree_stage_times: null argument"); return DFMM_E_ARG; }
  if (t->done_set) DFMM_HIP(hipEventSynchronize(t->done));
  for (int i = 0; i < DFMM_N_STAGES; ++i) ms[i] = t->stage_ms[i];
  if (n_calls) *n_calls = t->timed_calls;
  return DFMM_OK;
}

void dfmm_surrogate_default_cfg(dfmm_surrogate_cfg* c) {
  if (!c) return;
  c->hidden = 128;
  c->epochs = 20;
  c->batch = 4096;
  c->bins = 32;
  c->n_samples = 2000000;
  c->lr = 1e-3;
  c->tol = 1e-5;
  c->seed = 1;
}

// The plan's operator spectra must always come from the kernel the near
// field uses: whenever the surrogate is switched off because its network
// changes, the spectra are rebuilt with the exact kernel.
static int surrogate_off(dfmm_plan* pl, hipStream_t st) {
  const bool was = pl->sur.in_use && pl->sur.trained && pl->sur.pass_frac > 0;
  pl->sur.in_use = 0;
  return was ? build_spectra(pl, st) : DFMM_OK;
}

int dfmm_surrogate_train(dfmm_plan* pl, const dfmm_surrogate_cfg* cfg, void* stream) {
  if (!pl || !cfg) { set_error("surrogate_train: null argument"); return DFMM_E_ARG; }
  if (pl->iso) { set_error("surrogate_train: the plan's medium is isotropic (closed form)"); return DFMM_E_ARG; }
  int rc = surrogate_off(pl, (hipStream_t)stream);
  if (rc) return rc;
  return surrogate_train(pl, *cfg, (hipStream_t)stream);
}

int dfmm_surrogate_use(dfmm_plan* pl, int on, void* stream) {
  if (!pl) { set_error("surrogate_use: null plan"); return DFMM_E_ARG; }
  if (on && (!pl->sur.trained || pl->iso)) { set_error("surrogate_use: no trained surrogate"); return DFMM_E_STATE; }
  pl->sur.in_use = on ? 1 : 0;
  return build_spectra(pl, (hipStream_t)stream);
}

int dfmm_surrogate_info(const dfmm_plan* pl, char* json, size_t cap) {
  if (!pl || !json || cap == 0) { set_error("surrogate_info: invalid argument"); return DFMM_E_ARG; }
  const Surrogate& S = pl->sur;
  auto num = [](double x) {
    char b[40];
    std::snprintf(b, sizeof b, "%.9g", x);
    return std::string(b);
  };
  std::string s = "{\"trained\": " + std::to_string(S.trained) + ", \"in_use\": " + std::to_string(S.in_use) +
                  ", \"n_params\": " + std::to_string(S.L.total) + ", \"n_samples\": " + std::to_string(S.n_samples) +
                  ", \"epochs\": " + std::to_string(S.epochs) + ", \"bins\": " + std::to_string(S.bins) +
                  ", \"tol\": " + num(S.tol) + ", \"pass_frac\": " + num(S.pass_frac) +
                  ", \"max_bin_err\": " + num(S.max_err) + ", \"median_bin_err\": " + num(S.med_err) +
                  ", \"yscale\": " + num(S.yscale) + ", \"features\": [" + num(S.ft.f[0]) + ", " + num(S.ft.f[1]) +
                  ", " + num(S.ft.f[2]) + "], \"train_ms\": " + num(S.train_ms) + ", \"loss\": [";
  for (size_t i = 0; i < S.loss_hist.size(); ++i) s += (i ? ", " : "") + num(S.loss_hist[i]);
  s += "]}";
  if (s.size() + 1 > cap) { set_error("surrogate_info: buffer too small"); return DFMM_E_ARG; }
  std::memcpy(json, s.c_str(), s.size() + 1);
  return DFMM_OK;
}

int dfmm_surrogate_get_params(const dfmm_plan* pl, float* host, int64_t cap, int64_t* n) {
  if (!pl || !n) { set_error("surrogate_get_params: null argument"); return DFMM_E_ARG; }
  if (!pl->sur.w) { set_error("surrogate_get_params: no network"); return DFMM_E_STATE; }
  *n = pl->sur.L.total;
  if (host && cap >= *n) DFMM_HIP(hipMemcpy(host, pl->sur.w, sizeof(float) * (*n), hipMemcpyDeviceToHost));
  return DFMM_OK;
}

int dfmm_surrogate_set_params(dfmm_plan* pl, const float* host, int64_t n) {
  if (!pl || !host) { set_error("surrogate_set_params: null argument"); return DFMM_E_ARG; }
  if (pl->iso) { set_error("surrogate_set_params: the plan's medium is isotropic (closed form)"); return DFMM_E_ARG; }
  int rc = surrogate_off(pl, nullptr);
  if (rc) return rc;
  if (n != sur_layout(kSurHidden).total) { set_error("surrogate_set_params: wrong parameter count"); return DFMM_E_ARG; }
  if ((rc = surrogate_alloc(pl, 1, nullptr))) return rc;
  DFMM_HIP(hipMemcpy(pl->sur.w, host, sizeof(float) * n, hipMemcpyHostToDevice));
  if ((rc = surrogate_pack(pl, nullptr))) return rc;
  DFMM_HIP(hipStreamSynchronize(nullptr));
  pl->sur.trained = 0;
  return DFMM_OK;
}

int dfmm_surrogate_get_gate(const dfmm_plan* pl, unsigned char* host, int64_t cap, int* bins) {
  if (!pl || !bins) { set_error("surrogate_get_gate: null argument"); return DFMM_E_ARG; }
  if (!pl->sur.mask || pl->sur.bins < 1) { set_error("surrogate_get_gate: no gate"); return DFMM_E_STATE; }
  *bins = pl->sur.bins;
  const int64_t nb = 6LL * pl->sur.bins * pl->sur.bins;
  if (host && cap >= nb) DFMM_HIP(hipMemcpy(host, pl->sur.mask, nb, hipMemcpyDeviceToHost));
  return DFMM_OK;
}

// File layout (little-endian): "DFMMSUR1", int32 version, hidden, n_params,
// bins; float features[3], yscale; double tol, pass_frac, max_err, med_err,
// train_ms; int64 n_samples; int32 epochs, n_loss; double loss[n_loss];
// float params[n_params]; uint8 gate[6 bins^2].
static const char kSurMagic[8] = {'D', 'F', 'M', 'M', 'S', 'U', 'R', '1'};

int dfmm_surrogate_save(const dfmm_plan* pl, const char* path) {
  if (!pl || !path) { set_error("surrogate_save: null argument"); return DFMM_E_ARG; }
  const Surrogate& S = pl->sur;
  if (!S.trained || !S.w || !S.mask) { set_error("surrogate_save: no trained surrogate"); return DFMM_E_STATE; }
  std::vector<float> w(S.L.total);
  const int64_t nb = 6LL * S.bins * S.bins;
  std::vector<unsigned char> mask(nb);
  DFMM_HIP(hipMemcpy(w.data(), S.w, sizeof(float) * w.size(), hipMemcpyDeviceToHost));
  DFMM_HIP(hipMemcpy(mask.data(), S.mask, nb, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) { set_error(std::string("surrogate_save: cannot open ") + path); return DFMM_E_ARG; }
  const int32_t hdr[4] = {1, kSurHidden, (int32_t)S.L.total, S.bins};
  const float fl[4] = {S.ft.f[0], S.ft.f[1], S.ft.f[2], S.yscale};
  const double db[5] = {S.tol, S.pass_frac, S.max_err, S.med_err, S.train_ms};
  const int64_t ns = S.n_samples;
  const int32_t ep[2] = {S.epochs, (int32_t)S.loss_hist.size()};
  bool ok = std::fwrite(kSurMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
            std::fwrite(fl, sizeof fl, 1, f) == 1 && std::fwrite(db, sizeof db, 1, f) == 1 &&
            std::fwrite(&ns, sizeof ns, 1, f) == 1 && std::fwrite(ep, sizeof ep, 1, f) == 1 &&
            (S.loss_hist.empty() || std::fwrite(S.loss_hist.data(), sizeof(double), S.loss_hist.size(), f) == S.loss_hist.size()) &&
            std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size() &&
            std::fwrite(mask.data(), 1, mask.size(), f) == mask.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) { set_error(std::string("surrogate_save: write failed: ") + path); return DFMM_E_ARG; }
  return DFMM_OK;
}

int dfmm_surrogate_load(dfmm_plan* pl, const char* path, void* stream) {
  if (!pl || !path) { set_error("surrogate_load: null argument"); return DFMM_E_ARG; }
  if (pl->iso) { set_error("surrogate_load: the plan's medium is isotropic (closed form)"); return DFMM_E_ARG; }
  hipStream_t st = (hipStream_t)stream;
  FILE* f = std::fopen(path, "rb");
  if (!f) { set_error(std::string("surrogate_load: cannot open ") + path); return DFMM_E_ARG; }
  char magic[8];
  int32_t hdr[4], ep[2];
  float fl[4];
  double db[5];
  int64_t ns = 0;
  std::vector<double> loss;
  std::vector<float> w;
  std::vector<unsigned char> mask;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kSurMagic, 8) == 0 &&
            std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 1 && hdr[1] == kSurHidden &&
            hdr[2] == (int32_t)sur_layout(kSurHidden).total && hdr[3] >= 1 && hdr[3] <= 256 &&
            std::fread(fl, sizeof fl, 1, f) == 1 && std::fread(db, sizeof db, 1, f) == 1 &&
            std::fread(&ns, sizeof ns, 1, f) == 1 && std::fread(ep, sizeof ep, 1, f) == 1 && ep[1] >= 0 &&
            ep[1] <= (1 << 20);
  if (ok) {
    loss.resize(ep[1]);
    w.resize(hdr[2]);
    mask.resize(6LL * hdr[3] * hdr[3]);
    ok = (loss.empty() || std::fread(loss.data(), sizeof(double), loss.size(), f) == loss.size()) &&
         std::fread(w.data(), sizeof(float), w.size(), f) == w.size() &&
         std::fread(mask.data(), 1, mask.size(), f) == mask.size();
  }
  std::fclose(f);
  if (!ok) { set_error(std::string("surrogate_load: not a surrogate file of this library: ") + path); return DFMM_E_ARG; }
  const double csum = pl->prm.c11 + pl->prm.c12 + pl->prm.c44;
  if (fl[0] != (float)(pl->prm.c11 / csum) || fl[1] != (float)(pl->prm.c12 / csum) ||
      fl[2] != (float)(pl->prm.c44 / csum)) {
    set_error("surrogate_load: the network was trained for another medium");
    return DFMM_E_STATE;
  }
  int rc = surrogate_off(pl, st);
  if (rc) return rc;
  pl->sur.trained = 0;
  if ((rc = surrogate_alloc(pl, 1, st))) return rc;
  Surrogate& S = pl->sur;
  DFMM_HIP(hipMemcpy(S.w, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice));
  if ((rc = surrogate_pack(pl, st))) return rc;
  hipFree(S.mask);
  S.mask = nullptr;
  DFMM_HIP(hipMalloc(&S.mask, mask.size()));
  DFMM_HIP(hipMemcpy(S.mask, mask.data(), mask.size(), hipMemcpyHostToDevice));
  DFMM_HIP(hipStreamSynchronize(st));
  S.bins = hdr[3];
  S.yscale = fl[3];
  S.tol = db[0];
  S.pass_frac = db[1];
  S.max_err = db[2];
  S.med_err = db[3];
  S.train_ms = db[4];
  S.n_samples = ns;
  S.epochs = ep[0];
  S.loss_hist = loss;
  S.trained = 1;
  return DFMM_OK;
}

int dfmm_surrogate_loss_grad(dfmm_plan* pl, const float* X, const float* Y, int64_t n, float* grad, double* loss,
                             void* stream) {
  if (!pl || !X || !Y || !grad || n < 1 || n > (1 << 24)) { set_error("surrogate_loss_grad: invalid argument"); return DFMM_E_ARG; }
  if (!pl->sur.w) { set_error("surrogate_loss_grad: no network"); return DFMM_E_STATE; }
  return surrogate_loss_grad(pl, X, Y, n, grad, loss, (hipStream_t)stream);
}

int dfmm_surrogate_forward(const dfmm_plan* pl, const float* X, int64_t n, float* Y, void* stream) {
  if (!pl || !X || !Y || n < 1 || n > (1 << 24)) { set_error("surrogate_forward: invalid argument"); return DFMM_E_ARG; }
  if (!pl->sur.w) { set_error("surrogate_forward: no network"); return DFMM_E_STATE; }
  return surrogate_forward(pl, X, n, Y, (hipStream_t)stream);
}

int dfmm_plan_info(const dfmm_plan* pl, char* json, size_t cap) {
  if (!pl || !json || cap == 0) { set_error("plan_info: invalid argument"); return DFMM_E_ARG; }
  const int p = pl->p;
  double mem_unif = 54.0 * 316.0 * std::pow(2.0 * p - 1, 3) * 8.0;
  int w = std::snprintf(
      json, cap,
      "{\"order\": %d, \"depth\": %d, \"n_fft\": %d, \"n_freq\": %d, \"isotropic\": %d, \"mixed\": %d, "
      "\"mu\": %.17g, \"nu\": %.17g, \"mem_unif_fp64_bytes_per_level\": %.0f, "
      "\"m2l_mode\": %d, \"stored_offsets\": %d, \"generator_fp64_bytes_per_level\": %zu, "
      "\"spectra_bytes\": %zu, \"levels_stored\": %d, \"setup_ms\": %.3f, \"n_quad\": %d, \"n_circle\": %d, "
      "\"n_circle_float\": %d, \"float_rule_err\": %.3g, \"surrogate_in_use\": %d, \"lsq_degree\": %d}",
      p, pl->D, pl->n, pl->nf, pl->iso, pl->mixed, pl->mu, pl->nu, mem_unif, pl->sym,
      pl->sym ? kNumSymClass : kNumCanon, pl->gen_bytes / (size_t)std::max(1, pl->D - 1), pl->khat_bytes, pl->D - 1,
      pl->setup_ms, pl->quad.n, pl->prm.n_circle, 2 * pl->nhalf32, pl->float_rule_err, sur_dev(pl).on, pl->lsq);
  if (w < 0 || (size_t)w >= cap) { set_error("plan_info: buffer too small"); return DFMM_E_ARG; }
  return DFMM_OK;
}

int dfmm_tree_info(const dfmm_tree* t, char* json, size_t cap) {
  if (!t || !json || cap == 0) { set_error("tree_info: invalid argument"); return DFMM_E_ARG; }
  std::string s = "{\"n_seg\": " + std::to_string(t->nseg) + ", \"n_points\": " + std::to_string(t->N) +
                  ", \"depth\": " + std::to_string(t->D) + ", \"m2l_pairs\": " + std::to_string(t->npairs) +
                  ", \"near_pairs\": " + std::to_string(t->near_pairs) +
                  ", \"max_leaf_points\": " + std::to_string(t->max_leaf_pts) +
                  ", \"symmetric_near\": " + std::to_string(t->part != nullptr ? 1 : 0) +
                  ", \"workspace_bytes\": " + std::to_string(t->bytes) + ", \"adaptive\": " +
                  std::to_string(t->adaptive) + ", \"leaves\": " +
                  std::to_string(t->adaptive ? t->nleaf : (t->D >= 2 ? t->lv[t->D].n : 0)) +
                  ", \"u_pairs\": " + std::to_string(t->nu) + ", \"w_pairs\": " + std::to_string(t->nw) +
                  ", \"x_pairs\": " + std::to_string(t->nx) + ", \"direct_ranges\": " + std::to_string(t->nd) +
                  ", \"freq_chunks\": " + std::to_string(t->fchunks) +
                  ", \"levels\": [";
  for (int l = 2; l <= t->D; ++l) {
    if (l > 2) s += ", ";
    s += "{\"level\": " + std::to_string(l) + ", \"cells\": " + std::to_string(t->lv[l].n) +
         ", \"leaves\": " + std::to_string(t->adaptive ? t->leaf_n[l] : (l == t->D ? t->lv[l].n : 0)) +
         ", \"m2l_pairs\": " + std::to_string(t->lv[l].npairs) + "}";
  }
  s += "]}";
  if (s.size() + 1 > cap) { set_error("tree_info: buffer too small"); return DFMM_E_ARG; }
  std::memcpy(json, s.c_str(), s.size() + 1);
  return DFMM_OK;
}

}  // extern "C"
