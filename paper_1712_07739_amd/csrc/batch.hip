// Many independent configurations in one graph launch, and the depth
// autotuner built on the cost model of App. B (refined by measuring the
// model's choice and its neighbours).
#include <algorithm>
#include <numeric>

#include "internal.h"

struct dfmm_batch {
  int n = 0, lanes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* stamps = nullptr;  // device [n + 1]: [0] = graph start, [1 + i] = configuration i done
  double clk_khz = 0;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  hipStream_t origin = nullptr;  // capture origin (capture is not allowed on the null stream)
  hipStream_t last = nullptr;
};

namespace dfmm {

// Device wall-clock timestamp of the moment this (one-thread) kernel runs.
__global__ void k_stamp(uint64_t* slot) {
  if (threadIdx.x == 0) slot[0] = wall_clock64();
}

static void batch_free(dfmm_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (auto s : b->side) hipStreamDestroy(s);
  if (b->origin) hipStreamDestroy(b->origin);
  for (auto e : b->ev) hipEventDestroy(e);
  hipFree(b->stamps);
  delete b;
}

}  // namespace dfmm

using namespace dfmm;

// Wall time (device events) of one dfmm_fmm_forces at depth d after one
// untimed call; plan, tree and output are made and freed here.
static int time_depth(const dfmm_params* prm, int d, const double* seg, const double* burgers, int64_t n_seg,
                      hipStream_t st, double* ms) {
  dfmm_params q = *prm;
  q.depth = d;
  dfmm_plan* pl = nullptr;
  int rc = dfmm_fmm_setup(&q, st, &pl);
  if (rc) return rc;
  dfmm_tree* t = nullptr;
  double* f = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = dfmm_build_tree(pl, seg, n_seg, st, &t);
  if (rc == DFMM_OK && hipMalloc(&f, sizeof(double) * 6 * n_seg) != hipSuccess) rc = DFMM_E_NOMEM;
  if (rc == DFMM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = DFMM_E_HIP;
  if (rc == DFMM_OK) rc = fmm_forces_impl(pl, t, seg, burgers, f, st);
  if (rc == DFMM_OK && hipEventRecord(e0, st) != hipSuccess) rc = DFMM_E_HIP;
  if (rc == DFMM_OK) rc = fmm_forces_impl(pl, t, seg, burgers, f, st);
  if (rc == DFMM_OK && hipEventRecord(e1, st) != hipSuccess) rc = DFMM_E_HIP;
  if (rc == DFMM_OK && hipEventSynchronize(e1) != hipSuccess) rc = DFMM_E_HIP;
  float m = 0.f;
  if (rc == DFMM_OK && hipEventElapsedTime(&m, e0, e1) != hipSuccess) rc = DFMM_E_HIP;
  *ms = m;
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(f);
  dfmm_tree_destroy(t);
  dfmm_plan_destroy(pl);
  return rc;
}

extern "C" {

int dfmm_batch_create(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                      const double* const* burgers, double* const* forces, int n_cfg, int n_lanes, void* stream,
                      dfmm_batch** out) {
  if (!plans || !trees || !seg || !burgers || !forces || !out || n_cfg < 1 || n_lanes < 1 || n_lanes > 16) {
    set_error("batch_create: invalid argument");
    return DFMM_E_ARG;
  }
  *out = nullptr;
  for (int i = 0; i < n_cfg; ++i) {
    if (!plans[i] || !trees[i] || !seg[i] || !burgers[i] || !forces[i]) {
      set_error("batch_create: null entry " + std::to_string(i));
      return DFMM_E_ARG;
    }
    if (trees[i]->plan != plans[i]) {
      set_error("batch_create: tree " + std::to_string(i) + " was built with another plan");
      return DFMM_E_STATE;
    }
    if (trees[i]->timing) {
      set_error("batch_create: stage timing is on for tree " + std::to_string(i));
      return DFMM_E_STATE;
    }
  }
  (void)stream;
  dfmm_batch* b = new dfmm_batch();
  b->n = n_cfg;
  b->lanes = std::min(n_lanes, n_cfg);
  int dev = 0, khz = 0;
  hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
    batch_free(b);
    set_error("batch_create: no device wall-clock rate");
    return DFMM_E_HIP;
  }
  b->clk_khz = khz;
  if (hipMalloc(&b->stamps, sizeof(uint64_t) * (n_cfg + 1)) != hipSuccess) {
    batch_free(b);
    set_error("batch_create: cannot allocate timestamps");
    return DFMM_E_NOMEM;
  }
  b->side.resize(b->lanes);
  b->ev.resize(b->lanes + 1);
  if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    set_error("batch_create: stream creation failed");
    return DFMM_E_HIP;
  }
  hipStream_t st = b->origin;
  for (int l = 0; l < b->lanes; ++l)
    if (hipStreamCreateWithFlags(&b->side[l], hipStreamNonBlocking) != hipSuccess) {
      batch_free(b);
      set_error("batch_create: stream creation failed");
      return DFMM_E_HIP;
    }
  for (auto& e : b->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      set_error("batch_create: event creation failed");
      return DFMM_E_HIP;
    }
  // longest first onto the least loaded lane, by the number of quadrature points
  std::vector<int> order(n_cfg);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return trees[a]->N > trees[c]->N; });
  std::vector<double> load(b->lanes, 0.0);
  std::vector<int> lane_of(n_cfg);
  for (int i : order) {
    int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane_of[i] = l;
    load[l] += (double)trees[i]->N;
  }
  for (int i = 0; i < n_cfg; ++i) fmm_prepare(plans[i]);
  int rc = DFMM_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    batch_free(b);
    set_error("batch_create: stream capture could not start");
    return DFMM_E_HIP;
  }
  k_stamp<<<1, 64, 0, st>>>(b->stamps);
  hipEventRecord(b->ev[b->lanes], st);
  for (int l = 0; l < b->lanes; ++l) hipStreamWaitEvent(b->side[l], b->ev[b->lanes], 0);
  for (int i : order) {
    hipStream_t s = b->side[lane_of[i]];
    rc = fmm_forces_impl(plans[i], trees[i], seg[i], burgers[i], forces[i], s);
    if (rc) break;
    k_stamp<<<1, 64, 0, s>>>(b->stamps + 1 + i);
  }
  for (int l = 0; l < b->lanes; ++l) {
    hipEventRecord(b->ev[l], b->side[l]);
    hipStreamWaitEvent(st, b->ev[l], 0);
  }
  hipError_t e = hipStreamEndCapture(st, &b->graph);
  if (rc == DFMM_OK && e != hipSuccess) {
    set_error(std::string("batch_create: capture failed: ") + hipGetErrorString(e));
    rc = DFMM_E_HIP;
  }
  if (rc == DFMM_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    set_error("batch_create: graph instantiation failed");
    rc = DFMM_E_HIP;
  }
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return DFMM_OK;
}

int dfmm_batch_run(dfmm_batch* b, void* stream) {
  if (!b || !b->exec) { set_error("batch_run: invalid batch"); return DFMM_E_ARG; }
  DFMM_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
  b->last = (hipStream_t)stream;
  return DFMM_OK;
}

int dfmm_batch_latencies(dfmm_batch* b, double* ms, int n_cfg) {
  if (!b || !ms || n_cfg != b->n) { set_error("batch_latencies: invalid argument"); return DFMM_E_ARG; }
  std::vector<uint64_t> h(b->n + 1);
  hipStream_t st = b->last;
  DFMM_HIP(hipStreamSynchronize(st));
  DFMM_HIP(hipMemcpy(h.data(), b->stamps, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->n; ++i) ms[i] = (double)(h[1 + i] - h[0]) / b->clk_khz;
  return DFMM_OK;
}

void dfmm_batch_destroy(dfmm_batch* b) {
  if (b && b->last) hipStreamSynchronize(b->last);
  batch_free(b);
}

int dfmm_autotune_batch_lanes(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                              const double* const* burgers, double* const* forces, int n_cfg, int reps, void* stream,
                              int* best, double* ms) {
  if (!best || reps < 1 || n_cfg < 1) {
    set_error("autotune_batch_lanes: invalid argument");
    return DFMM_E_ARG;
  }
  const hipStream_t st = (hipStream_t)stream;
  const int cand[4] = {1, 2, 4, 8};
  double best_ms = 0;
  *best = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    set_error("autotune_batch_lanes: cannot create events");
    return DFMM_E_HIP;
  }
  int rc = DFMM_OK;
  for (int k = 0; k < 4 && rc == DFMM_OK; ++k) {
    if (ms) ms[k] = 0;
    if (cand[k] > n_cfg && k > 0) continue;
    dfmm_batch* b = nullptr;
    rc = dfmm_batch_create(plans, trees, seg, burgers, forces, n_cfg, cand[k], stream, &b);
    if (rc) break;
    rc = dfmm_batch_run(b, stream);  // warm-up
    if (rc == DFMM_OK && hipEventRecord(e0, st) != hipSuccess) rc = DFMM_E_HIP;
    for (int r = 0; r < reps && rc == DFMM_OK; ++r) rc = dfmm_batch_run(b, stream);
    if (rc == DFMM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      rc = DFMM_E_HIP;
    float t = 0.f;
    if (rc == DFMM_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = DFMM_E_HIP;
    dfmm_batch_destroy(b);
    if (rc) break;
    const double per = t / reps;
    if (ms) ms[k] = per;
    if (*best == 0 || per < best_ms) {
      best_ms = per;
      *best = cand[k];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == DFMM_E_HIP) set_error("autotune_batch_lanes: a HIP call failed");
  return rc;
}

int dfmm_forces_batched(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                        const double* const* burgers, double* const* forces, int n_cfg, void* stream) {
  dfmm_batch* b = nullptr;
  int rc = dfmm_batch_create(plans, trees, seg, burgers, forces, n_cfg, std::min(4, std::max(1, n_cfg)), stream, &b);
  if (rc) return rc;
  rc = dfmm_batch_run(b, stream);
  if (rc == DFMM_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
    set_error("forces_batched: stream synchronisation failed");
    rc = DFMM_E_HIP;
  }
  dfmm_batch_destroy(b);
  return rc;
}

int dfmm_autotune_depth(const dfmm_params* prm, const double* seg, const double* burgers, int64_t n_seg, int d_min,
                        int d_max, void* stream, int* best, double* pred_ms, double* meas_ms) {
  if (!prm || !seg || !burgers || !best || n_seg < 1 || d_min < 2 || d_max > 10 || d_min > d_max ||
      prm->depth < d_min || prm->depth > d_max) {
    set_error("autotune_depth: invalid argument (the plan depth must lie in [d_min, d_max])");
    return DFMM_E_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  dfmm_plan* pl = nullptr;
  int rc = dfmm_fmm_setup(prm, stream, &pl);
  if (rc) return rc;
  dfmm_tree* t0 = nullptr;
  rc = dfmm_build_tree(pl, seg, n_seg, stream, &t0);
  double* f = nullptr;
  if (rc == DFMM_OK && hipMalloc(&f, sizeof(double) * 6 * n_seg) != hipSuccess) rc = DFMM_E_NOMEM;
  double ms[DFMM_N_STAGES] = {};
  if (rc == DFMM_OK) {
    // one untimed call, then one timed call at the plan's depth
    rc = fmm_forces_impl(pl, t0, seg, burgers, f, st);
    if (rc == DFMM_OK) {
      t0->timing = 1;
      rc = fmm_forces_impl(pl, t0, seg, burgers, f, st);
      t0->timing = 0;
      for (int i = 0; i < DFMM_N_STAGES; ++i) ms[i] = t0->stage_ms[i];
    }
  }
  if (rc == DFMM_OK) {
    // App. B: near cost C_n x (near pairs), far cost C_f x (M2L translations);
    // the remaining stages scale with the number of cells and points.
    const double near_ms = ms[6], far_ms = ms[2] + ms[3] + ms[4];
    const double other_ms = ms[0] + ms[1] + ms[5] + ms[7];
    const double cn = near_ms / std::max<int64_t>(1, t0->near_pairs);
    const double cf = far_ms / std::max<int64_t>(1, t0->npairs);
    const double cc = other_ms / std::max<int64_t>(1, t0->ncell_total + t0->N);
    double best_ms = 1e300;
    for (int d = d_min; d <= d_max && rc == DFMM_OK; ++d) {
      dfmm_plan tmp = *pl;  // same tables; only the depth differs for the partition
      tmp.D = d;
      dfmm_tree* t = new dfmm_tree();
      rc = build_tree_impl(&tmp, seg, n_seg, st, t, /*workspaces=*/false);
      if (rc == DFMM_OK) {
        double pm = cn * t->near_pairs + cf * t->npairs + cc * (t->ncell_total + t->N);
        if (pred_ms) pred_ms[d - d_min] = pm;
        if (pm < best_ms) {
          best_ms = pm;
          *best = d;
        }
      }
      t->plan = nullptr;
      dfmm_tree_destroy(t);
    }
  }
  hipFree(f);
  dfmm_tree_destroy(t0);
  dfmm_plan_destroy(pl);
  if (meas_ms)
    for (int d = d_min; d <= d_max; ++d) meas_ms[d - d_min] = 0.0;
  if (rc) return rc;
  // measurement of the model's choice and its neighbours
  const int pick = *best;
  double best_meas = 1e300;
  for (int d = std::max(d_min, pick - 1); d <= std::min(d_max, pick + 1) && rc == DFMM_OK; ++d) {
    double ms_d = 0.0;
    rc = time_depth(prm, d, seg, burgers, n_seg, st, &ms_d);
    if (rc) break;
    if (meas_ms) meas_ms[d - d_min] = ms_d;
    if (ms_d < best_meas) {
      best_meas = ms_d;
      *best = d;
    }
  }
  return rc;
}

}  // extern "C"
