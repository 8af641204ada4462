// C ABI of libdfmm: argument checking, object lifetime, error reporting.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace dfmm {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

// Gauss-Legendre nodes/weights on [-1, 1]: eigenvalue-free Newton iteration
// on P_n (three-term recurrence).
static void gauss_legendre(int n, double* u, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), d = 1.0;
    for (int it = 0; it < 100; ++it) {
      double a = 1.0, b = x;
      for (int k = 2; k <= n; ++k) {
        double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
      }
      d = n * (x * b - a) / (x * x - 1.0);
      double dx = b / d;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    u[n - 1 - i] = x;
    w[n - 1 - i] = 2.0 / ((1.0 - x * x) * d * d);
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
  if (q.precision != DFMM_FP64 && q.precision != DFMM_MIXED) {
    set_error("fmm_setup: precision must be DFMM_FP64 or DFMM_MIXED");
    return DFMM_E_ARG;
  }
  auto t0 = std::chrono::steady_clock::now();
  dfmm_plan* pl = new dfmm_plan();
  pl->prm = q;
  pl->p = q.order;
  pl->n = 2 * q.order - 1;
  pl->nf = pl->n * pl->n * q.order;
  pl->D = q.depth;
  pl->mixed = q.precision == DFMM_MIXED;
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
  for (auto& l : pl->lev) hipFree(l.khat);
  hipFree(pl->t64.S); hipFree(pl->t64.cs); hipFree(pl->t64.tw);
  hipFree(pl->t32.S); hipFree(pl->t32.cs); hipFree(pl->t32.tw);
  hipFree(pl->oid343); hipFree(pl->off158);
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
  hipFree(t->pts); hipFree(t->pleaf); hipFree(t->W); hipFree(t->s); hipFree(t->What); hipFree(t->Shat); hipFree(t->sig);
  delete t;
}

int dfmm_fmm_forces(const dfmm_plan* plan, dfmm_tree* tree, const double* seg, const double* burgers,
                    double* forces, void* stream) {
  if (!plan || !tree || !seg || !burgers || !forces) { set_error("fmm_forces: null argument"); return DFMM_E_ARG; }
  if (tree->plan != plan) { set_error("fmm_forces: tree was built with another plan"); return DFMM_E_STATE; }
  return fmm_forces_impl(plan, tree, seg, burgers, forces, (hipStream_t)stream);
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

int dfmm_surrogate_train(dfmm_plan* pl, const dfmm_surrogate_cfg* cfg, void* stream) {
  if (!pl || !cfg) { set_error("surrogate_train: null argument"); return DFMM_E_ARG; }
  if (pl->iso) { set_error("surrogate_train: the plan's medium is isotropic (closed form)"); return DFMM_E_ARG; }
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
  std::string s = "{\"trained\": " + std::to_string(S.trained) + ", \"in_use\": " + std::to_string(S.in_use) +
                  ", \"n_params\": " + std::to_string(S.L.total) + ", \"n_samples\": " + std::to_string(S.n_samples) +
                  ", \"epochs\": " + std::to_string(S.epochs) + ", \"bins\": " + std::to_string(S.bins) +
                  ", \"tol\": " + std::to_string(S.tol) + ", \"pass_frac\": " + std::to_string(S.pass_frac) +
                  ", \"max_bin_err\": " + std::to_string(S.max_err) + ", \"median_bin_err\": " +
                  std::to_string(S.med_err) + ", \"yscale\": " + std::to_string(S.yscale) +
                  ", \"train_ms\": " + std::to_string(S.train_ms) + ", \"loss\": [";
  for (size_t i = 0; i < S.loss_hist.size(); ++i) {
    char b[32];
    std::snprintf(b, sizeof b, "%s%.6g", i ? ", " : "", S.loss_hist[i]);
    s += b;
  }
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
  int rc = surrogate_alloc(pl, 1, nullptr);
  if (rc) return rc;
  if (n != pl->sur.L.total) { set_error("surrogate_set_params: wrong parameter count"); return DFMM_E_ARG; }
  DFMM_HIP(hipMemcpy(pl->sur.w, host, sizeof(float) * n, hipMemcpyHostToDevice));
  pl->sur.trained = 0;
  pl->sur.in_use = 0;
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
      "\"spectra_bytes\": %zu, \"levels_stored\": %d, \"setup_ms\": %.3f, \"n_quad\": %d, \"n_circle\": %d, "
      "\"n_circle_float\": %d, \"float_rule_err\": %.3g}",
      p, pl->D, pl->n, pl->nf, pl->iso, pl->mixed, pl->mu, pl->nu, mem_unif, pl->khat_bytes, pl->D - 1,
      pl->setup_ms, pl->quad.n, pl->prm.n_circle, 2 * pl->nhalf32, pl->float_rule_err);
  if (w < 0 || (size_t)w >= cap) { set_error("plan_info: buffer too small"); return DFMM_E_ARG; }
  return DFMM_OK;
}

int dfmm_tree_info(const dfmm_tree* t, char* json, size_t cap) {
  if (!t || !json || cap == 0) { set_error("tree_info: invalid argument"); return DFMM_E_ARG; }
  std::string s = "{\"n_seg\": " + std::to_string(t->nseg) + ", \"n_points\": " + std::to_string(t->N) +
                  ", \"depth\": " + std::to_string(t->D) + ", \"m2l_pairs\": " + std::to_string(t->npairs) +
                  ", \"near_pairs\": " + std::to_string(t->near_pairs) +
                  ", \"max_leaf_points\": " + std::to_string(t->max_leaf_pts) +
                  ", \"workspace_bytes\": " + std::to_string(t->bytes) + ", \"levels\": [";
  for (int l = 2; l <= t->D; ++l) {
    if (l > 2) s += ", ";
    s += "{\"level\": " + std::to_string(l) + ", \"cells\": " + std::to_string(t->lv[l].n) +
         ", \"m2l_pairs\": " + std::to_string(t->lv[l].npairs) + "}";
  }
  s += "]}";
  if (s.size() + 1 > cap) { set_error("tree_info: buffer too small"); return DFMM_E_ARG; }
  std::memcpy(json, s.c_str(), s.size() + 1);
  return DFMM_OK;
}

}  // extern "C"
