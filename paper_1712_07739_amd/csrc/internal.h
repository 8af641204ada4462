// Internal declarations of libdfmm (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dfmm.h"
#include "kernel_eval.h"
#include "mlp_eval.h"

namespace dfmm {

constexpr int kMaxOrder = 8;
constexpr int kMaxLevels = 10;  // deepest leaf level (30-bit Morton keys)
constexpr int kMaxQuad = 8;
constexpr int kNumOffsets = 316;  // M2L offsets in [-3,3]^3 outside [-1,1]^3
// Targets per M2L block (one window of Morton-consecutive targets), two lanes
// per target: 768 threads in single precision (two blocks per CU), 1024 in
// double, whose spectra (139 KB) leave room for one block per CU.  Both are
// whole multiples of four waves, so a CU's four SIMDs get equal shares.
// (Windows four times as large, whose waves take 32 targets at a time from a
// counter, made the product 8-18% slower: sorted by list length, a larger
// window's waves draw their sources from further apart.)
constexpr int kM2LWindowF = 384;
constexpr int kM2LWindowD = 512;
inline int m2l_window(bool mixed) { return mixed ? kM2LWindowF : kM2LWindowD; }
constexpr int kNumCanon = 158;    // one of each pair (o, -o): the kernel is odd, so the
                                  // spectrum of -o is minus the conjugate of that of o
constexpr int kNumFar = 189;      // interaction-list size of an interior cell
// Scratch of the allocation-free direct sum (one copy per GPU) and the
// devices it supports.
constexpr long long kScratchBytes = DFMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The M2L Hadamard kernels split a target's 6x9 product between its two
// lanes by source component, so that no source value crosses lanes: lane h
// loads components 4h..4h+3 and 8 of the source and takes components
// 4h..4h+3 for all six stress rows and component 8 for rows 3h..3h+2 (27
// complex multiply-adds each), keeping row R in accumulator (R - 3h) mod 6;
// the rows a lane writes (3h..3h+2, its accumulators 0..2) receive the
// partner's accumulators 3..5 once per target.  The spectra are stored in
// the order in which a lane reads them: per frequency and offset, lane h's 27
// entries (f_unit_of, d_unit_of, h16_word_of) start a half of its own.
// Single precision: two halves of kKHalfF complex entries (16-byte aligned;
// the pads are zero), 29 16-byte units per offset: lanes read the spectra of
// unrelated offsets at once, and an odd stride spreads those reads evenly
// over the LDS banks (an even one leaves half of them idle and doubles up the
// rest).
constexpr int kKHalfF = 28;
constexpr int kKOffsetF = 2 * kKHalfF + 2;
// Entry of stress row R (0..5), source component C (0..8) in an offset's
// single-precision spectra: lane h's 27 entries (components 4h..4h+3 for
// accumulators a = 0..5, then component 8 for rows 3h..3h+2) start at entry
// 28 h.
__host__ __device__ constexpr int f_unit_of(int R, int C) {
  return C == 8 ? kKHalfF * (R / 3) + 24 + R % 3
                : kKHalfF * (C >> 2) + 4 * ((R - 3 * (C >> 2) + 6) % 6) + (C & 3);
}
constexpr bool f_layout_ok() {
  bool seen[kKOffsetF] = {};
  for (int R = 0; R < 6; ++R)
    for (int C = 0; C < 9; ++C) {
      const int w = f_unit_of(R, C);
      if (w < 0 || w >= 2 * kKHalfF || w % kKHalfF >= 27 || seen[w]) return false;
      seen[w] = true;
    }
  return true;
}
static_assert(f_layout_ok(), "single-precision spectrum entries");
// The f16 product: one 32-bit word (f16 real, f16 imaginary) per complex
// value; lane h's 27 words, in the order it reads them (accumulator-major for
// components 4h..4h+3, then component 8), start at word 28 h; per offset two
// halves of 28 words and 4 pad words, 15 16-byte units (odd, for the same
// reason).
constexpr int kKHalfH = 28;
constexpr int kKOffsetH = 2 * kKHalfH + 4;
// Word of stress row R (0..5), source component C (0..8) in an offset's
// f16 spectra.
__host__ __device__ constexpr int h16_word_of(int R, int C) {
  return C == 8 ? kKHalfH * (R / 3) + 24 + R % 3
                : kKHalfH * (C >> 2) + 4 * ((R - 3 * (C >> 2) + 6) % 6) + (C & 3);
}
// every (row, component) has its own word, the first 27 of a half
constexpr bool h16_layout_ok() {
  bool seen[kKOffsetH] = {};
  for (int R = 0; R < 6; ++R)
    for (int C = 0; C < 9; ++C) {
      const int w = h16_word_of(R, C);
      if (w < 0 || w >= 2 * kKHalfH || w % kKHalfH >= 27 || seen[w]) return false;
      seen[w] = true;
    }
  return true;
}
static_assert(h16_layout_ok(), "f16 spectrum words");
// Double precision: one complex value per 16-byte LDS unit, the two halves of
// 27 values back to back and one pad unit, 55 units per offset (odd).
constexpr int kKHalfD = 27;
constexpr int kKOffsetD = 2 * kKHalfD + 1;
// The double product splits the 6x9 product between a target's two lanes by
// source component as the f16 product does: lane h's 27 values (components
// 4h..4h+3 for accumulators a = 0..5, stress row (3h + a) mod 6, then
// component 8 for rows 3h..3h+2) start at unit 27 h.  Unit of stress row R
// (0..5), source component C (0..8) in an offset's double spectra:
__host__ __device__ constexpr int d_unit_of(int R, int C) {
  return C == 8 ? kKHalfD * (R / 3) + 24 + R % 3
                : kKHalfD * (C >> 2) + 4 * ((R - 3 * (C >> 2) + 6) % 6) + (C & 3);
}
constexpr bool d_layout_ok() {
  bool seen[kKOffsetD] = {};
  for (int R = 0; R < 6; ++R)
    for (int C = 0; C < 9; ++C) {
      const int w = d_unit_of(R, C);
      if (w < 0 || w >= 2 * kKHalfD || seen[w]) return false;
      seen[w] = true;
    }
  return true;
}
static_assert(d_layout_ok(), "double spectrum units");
// The single-precision M2L kernel walks the lists of 32 consecutive targets
// of the processing order in one wave; their entries are stored step-major per
// wave (see Level::ilw), and the entry after a list's end is read.
// Largest leaf (points) for the symmetric near field, both precisions (its
// LDS holds four accumulators per point in single precision, two in FP64);
// trees with larger leaves use the one-sided kernel.
constexpr int kSymMaxLeaf = 1024;
constexpr int kWaveTargets = 32;
constexpr int kIlwPad = 2;  // the f16 product reads entries two steps ahead
// Target (0..31 within the wave) of lane pair lp (lanes 2 lp, 2 lp + 1) in
// the M2L kernels.  LDS has 64 four-byte banks and serves a wave's 16-byte
// read in four passes of 16 lanes, which are not runs of consecutive lanes:
// one-wave reads counted with SQ_LDS_BANK_CONFLICT put lanes 0-3, 12-15 and
// 20-27 in one pass and 4-11, 16-19, 28-31 in another (the same again for
// lanes 32-63), i.e. lane l's pass is 2 (l >> 5) plus the parity of bits
// 2..5 of l.  This map gives the 8 lane pairs of pass k the consecutive
// targets 8k..8k+7, so the lists' bank-aware order (tree build), which packs
// the bank groups of 8 consecutive targets, packs each pass.
__host__ __device__ constexpr int pass_target(int lp) {
  const int par = ((lp >> 1) ^ (lp >> 2) ^ (lp >> 3) ^ (lp >> 4)) & 1;
  return (lp & 16) | (par << 3) | ((lp >> 1) & 6) | (lp & 1);
}
constexpr bool pass_target_ok() {
  bool seen[32] = {};
  for (int lp = 0; lp < 32; ++lp) {
    const int t = pass_target(lp);
    if (t < 0 || t >= 32 || seen[t]) return false;
    seen[t] = true;
  }
  // lanes 0-3, 12-15, 20-27 (pairs 0, 1, 6, 7, 10..13) hold targets 0..7
  return pass_target(0) == 0 && pass_target(1) == 1 && pass_target(6) == 2 && pass_target(7) == 3 &&
         pass_target(10) == 4 && pass_target(13) == 7 && pass_target(2) == 8 && pass_target(18) == 16 &&
         pass_target(16) == 24;
}
static_assert(pass_target_ok(), "lane pair -> target map");

struct Quad {
  double u[kMaxQuad], w[kMaxQuad];
  int n;
};

// Quadrature point k of segment s: position x = x1 + (1 + u_k)/2 (x2 - x1)
// and weight vector t = (w_k / 2)(x2 - x1).  The tree build (which finds the
// near-coincident pairs) and every force call (which skips them in the
// single-precision near field) form the positions with this one function,
// with explicit fused multiply-adds, so both see the same bits.
__device__ __forceinline__ void quad_point(const double* seg, int64_t s, int k, const Quad& qd, double* x,
                                           double* t) {
  const double* p = seg + 6 * s;
  const double c = 0.5 * (1.0 + qd.u[k]), hw = 0.5 * qd.w[k];
  for (int d = 0; d < 3; ++d) {
    const double dS = p[3 + d] - p[d];
    x[d] = fma(c, dS, p[d]);
    t[d] = hw * dS;
  }
}

// Device-resident float/double copies of the small constant tables.
template <typename T>
struct Tables {
  T* S = nullptr;   // [2][p][p]: S[b][i][m] = parent basis i at child node m of octant bit b
  T* cs = nullptr;  // circle cos/sin [nhalf][2]
  T* tw = nullptr;  // DFT twiddles [n][2]: exp(-2 pi i k / n)
  T* Pm = nullptr;  // [p][p] least-squares projector of the node values (stabilised interpolation)
};

// Trained network of the anisotropic-kernel surrogate and its residual gate.
struct Surrogate {
  int trained = 0, in_use = 0;
  SurLayout L = {};
  SurFeat ft = {};
  float yscale = 1.f;
  float* w = nullptr;  // f32 master parameters (device), layout SurLayout
  float* g = nullptr;  // gradient
  float* m = nullptr;  // Adam moments
  float* v = nullptr;
  uint16_t* wi = nullptr;  // inference copy: f16 fragments (mlp_eval.h)
  float* bi = nullptr;     // inference biases
  float* split = nullptr;  // split-K partials of the training products
  size_t split_n = 0;
  unsigned char* mask = nullptr;  // [6][bins][bins]
  int bins = 0;
  double tol = 0, pass_frac = 0, max_err = 0, med_err = 0, train_ms = 0;
  int64_t n_samples = 0;
  int epochs = 0;
  std::vector<double> loss_hist;
};

struct LevelTables {
  float kscale = 1.f;    // DFMM_MIXED_F16: power of two the f16 operator spectra are scaled by
  void* khat = nullptr;  // DFT of the circulant embedding of each stored offset's
                         // generator.  DFMM_M2L_FFT: the 158 canonical offsets,
                         // double [nf][158][54] complex (row-major 6 x 9), float
                         // [nf][158][kKOffsetF] complex in reading order (DFMM_MIXED_F16:
                         // [nf][158][kKOffsetH] f16 pairs, scaled by kscale).
                         // DFMM_M2L_FFT_SYM: the 16 symmetry classes, [nf][16][54]
                         // complex (row-major 6 x 9) in the plan's precision.
};

// Symmetry reduction of the M2L operators: the 316 offsets fall into 16
// classes under the 48 signed permutations R of the axes (the cube's
// symmetry group, which maps a cubic or isotropic medium onto itself).  The
// kernel obeys K(R x) = det(R) rho(R) K(x) with rho(R) acting on each of its
// four indices, so the spectrum of offset R o_c is
//   Khat_{R o_c}(f)[a b w r] = det(R) s_a s_b s_w s_r Khat_{o_c}(R^T f)[pi(a) pi(b) pi(w) pi(r)]
// with R_ij = s_i [j == pi(i)].  Per canonical id: class, pi, s and det(R).
constexpr int kNumSymClass = 16;
struct SymEntry {
  int cls;
  int pi[3];
  int sg[3];
  int det;
};

}  // namespace dfmm

struct dfmm_plan {
  dfmm_params prm;
  int p = 0, n = 0, nf = 0, D = 0;
  int mixed = 0;
  int iso = 0;
  double mu = 0, nu = 0;  // isotropic (or Voigt) moduli
  int nhalf32 = 0;         // circle angles on [0, pi) of the float evaluation
  double float_rule_err = 0;
  dfmm::Quad quad;
  dfmm::Tables<double> t64;
  dfmm::Tables<float> t32;
  int* oid343 = nullptr;   // device [343]: offset (o+3) lex index -> 2*canonical id + mirrored, or -1
  int* off158 = nullptr;   // device [158][3]: canonical id -> offset
  int sym = 0;             // operator store: 0 = 158 offset spectra, 1 = 16 class spectra
  int h16 = 0;             // DFMM_MIXED_F16: f16 operands in the M2L product
  int lsq = 0;             // least-squares degree of the stabilised interpolation (0: Lagrange)
  int* cls16 = nullptr;    // device [16][3]: class representatives (|o| sorted, descending)
  dfmm::SymEntry* symtab = nullptr;  // device [158]: class and R of each canonical id
  size_t gen_bytes = 0;    // kernel values behind the stored spectra (real generators, FP64)
  std::vector<dfmm::LevelTables> lev;  // index = level (0..D); used for 2..D
  double setup_ms = 0;
  size_t khat_bytes = 0;
  dfmm::Surrogate sur;
  int device = 0;
  template <typename T>
  dfmm::Med<T> med() const;
};

struct dfmm_tree {
  const dfmm_plan* plan = nullptr;
  int64_t nseg = 0, N = 0;
  int D = 0;
  // sorted points: perm[sorted] = point id (= seg*nq + k), inv[point id] = sorted
  uint32_t* perm = nullptr;
  uint32_t* inv = nullptr;
  // occupied cells of one level (level-local indices), levels 2..D
  struct Level {
    int64_t n = 0;             // occupied cells
    int64_t off = 0;           // first global cell index (W, s are global over levels 2..D)
    uint32_t* key = nullptr;   // Morton key at this level, ascending
    int* first = nullptr;      // leaves: first sorted point; others: first child (level l+1 index)
    int* count = nullptr;      // leaves: #points; others: #children
    int* parent = nullptr;     // parent index at level l-1 (levels 3..D)
    int* il_start = nullptr;   // [n+1] interaction-list CSR
    int2* il = nullptr;        // (source index at this level, 2*canonical offset id + mirrored);
                               // double-precision plans only
    uint32_t* order = nullptr; // targets in M2L processing order (list length buckets, then Morton)
    // Single-precision plans: the lists laid out for the M2L kernel, one block
    // per wave of kWaveTargets consecutive targets of the processing order.
    // Entry s of the target in slot k of wave w is ilw[kWaveTargets *
    // (wbase[w] + s) + k] = source | id << 23 | mirrored << 31 (cells < 2^23);
    // a block has the wave's longest list + kIlwPad steps, the unused entries
    // zero (a valid entry).
    uint32_t* ilw = nullptr;
    int* wbase = nullptr;      // [waves + 1] first step of each wave's block
    int* lenq = nullptr;       // [n] list length by processing position
    int64_t npairs = 0;
  };
  std::vector<Level> lv;
  int64_t ncell_total = 0, max_level_cells = 0;
  int* nbr = nullptr;            // leaves: [n][27] neighbour leaf index or -1
  int* pleaf = nullptr;          // [N] leaf of each sorted point
  int64_t npairs = 0;            // M2L pairs over all levels
  int64_t near_pairs = 0;        // point pairs in the near field
  int max_leaf_pts = 0;
  // workspaces
  double* pts = nullptr;    // sorted point data [9][N]: x, y, z, bx, by, bz, tx, ty, tz
  double* pos0 = nullptr;   // [3][N] the sorted points' positions at build time
  unsigned long long* chk = nullptr;  // [2] position check: mismatches, first mismatching segment
  void* W = nullptr;        // [ncell_total][9][p^3]  (float or double)
  void* s = nullptr;        // [ncell_total][6][p^3]
  int fchunk = 0;           // first frequency indices per chunk of the spectra (n: whole)
  int fchunks = 1;          // chunks per level
  void* What = nullptr;     // [chunk frequencies][max level cells][9] complex (f16 pairs or T)
  void* Shat = nullptr;     // [chunk frequencies][max level cells][6] complex
  double* sig = nullptr;    // [N][6] stress at sorted points
  unsigned* wmax = nullptr; // DFMM_MIXED_F16: per level, the largest |W| (float bits), for the f16 scale
  void* kexp = nullptr;     // symmetry-reduced plans: one level's 158 offset spectra, expanded
                            // from the 16 classes before that level's Hadamard product
  void* part = nullptr;     // cubic medium: [N][27][6] near-field partial (float or double) per
                            // neighbour slot (the symmetric near field)
  int* bigp = nullptr;      // leaf pairs with more than 64 points on a side, A * 14 + (q - 13)
  int64_t nbig = 0;
  size_t bytes = 0;
  // per-stage timing
  int timing = 0;
  hipEvent_t ev[DFMM_N_STAGES + 1] = {};
  double stage_ms[DFMM_N_STAGES] = {};
  int timed_calls = 0;
  // Single-precision plans: the near-coincident pairs (closer than 2a, left
  // to a double-precision pass), found once per tree.  Per sorted target
  // point, the CSR of its sources in the order the near field visits them.
  int64_t nclose = 0;
  int* cstart = nullptr;   // [N + 1]
  int2* cpair = nullptr;   // [nclose] (target, source), sorted point indices
  double* cval = nullptr;  // [nclose][6] per-pair stress, written by every call
  int64_t nuni = 0;
  int2* cuni = nullptr;     // [nuni] unordered pairs: (entry (i, j) with i < j, entry (j, i))
  // Adaptive tree (plan leaf_max > 0): cells below a leaf are pruned and the
  // levels' arrays hold the cells that remain (first/count: children, zero for
  // a leaf).  Leaves of all levels are numbered level by level ("ordinals").
  int adaptive = 0;
  int64_t nleaf = 0;
  int64_t leaf_off[dfmm::kMaxLevels + 1] = {}, leaf_n[dfmm::kMaxLevels + 1] = {};  // ordinals of each level's leaves
  int* gl_cell = nullptr;        // [nleaf] global cell index (over levels 2..D)
  int* gl_pf = nullptr;          // [nleaf] first sorted point
  int* gl_pc = nullptr;          // [nleaf] points
  uint32_t* gkey = nullptr;      // [ncell_total] Morton key at the cell's level
  unsigned char* glev = nullptr; // [ncell_total] level
  int* gord = nullptr;           // [ncell_total] leaf ordinal, or -1
  int* ustart = nullptr;         // [nleaf + 1] U lists: adjacent leaves (ordinals), any level
  int* usrc = nullptr;
  int64_t nu = 0;
  int* wstart = nullptr;         // [nleaf + 1] W lists: source cells (global) acting on a leaf's points
  int* wsrc = nullptr;
  int64_t nw = 0;
  int* xstart = nullptr;         // [ncell_total + 1] X lists: source leaves acting on a cell's nodes
  int* xsrc = nullptr;
  int64_t nx = 0;
  int* xcells = nullptr;         // cells whose X list goes through their nodes (more than p^3 points below)
  int64_t nxcell = 0;
  int* gsf = nullptr;            // [ncell_total] first sorted point below the cell
  int* gsn = nullptr;            // [ncell_total] points below the cell
  int* dstart = nullptr;         // [nleaf + 1] direct sources of a leaf's points: the U leaves, then the
  int2* drange = nullptr;        //   W cells and (for its ancestors) X leaves of pairs whose finer cell
  int64_t nd = 0;                //   holds at most p^3 points, as point ranges (first, count)
  int* wleaves = nullptr;        // leaves with a non-empty W list
  int64_t nwleaf = 0;
  // recorded at the end of every call that is not being captured into a
  // graph: destroy and the query calls wait on it (an event the tree owns,
  // valid whatever becomes of the caller's streams)
  hipEvent_t done = nullptr;
  bool done_set = false;
  // second stream for the near field, which runs beside the far-field
  // pipeline (fork after the point gather, join before L2P)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace dfmm {

void set_error(const std::string& msg);

// setup.hip
int setup_tables(dfmm_plan* plan, hipStream_t st);
int build_spectra(dfmm_plan* plan, hipStream_t st);  // exact, or with the surrogate when in use
SurDev sur_dev(const dfmm_plan* plan);

// mlp.hip
SurLayout sur_layout(int hidden);
int surrogate_pack(dfmm_plan* pl, hipStream_t st);   // f16 inference copy of the master weights
int surrogate_gate(dfmm_plan* pl, int bins, double tol, hipStream_t st);
int surrogate_infer(const dfmm_plan* pl, const float* X, int64_t n, float* Y, hipStream_t st);
int sur_grid(int device);
int surrogate_train(dfmm_plan* pl, const dfmm_surrogate_cfg& cfg, hipStream_t st);
int surrogate_alloc(dfmm_plan* pl, uint64_t seed, hipStream_t st);
int surrogate_loss_grad(dfmm_plan* pl, const float* X, const float* Y, int64_t n, float* grad, double* loss,
                        hipStream_t st);
int surrogate_forward(const dfmm_plan* pl, const float* X, int64_t n, float* Yout, hipStream_t st);

// tree.hip
// Exclusive scan of in[0..n) (n >= 1) into out, the total in *total (host).
int scan_excl(const int* in, int* out, int64_t n, hipStream_t st, int64_t* total);
// Stable LSD radix sort of (keys, vals) (n >= 1) by the low `bits` bits of keys.
int radix_sort(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t st);
int check_positions_impl(const dfmm_plan* plan, dfmm_tree* t, const double* seg, hipStream_t st);
int build_tree_impl(dfmm_plan* plan, const double* seg, int64_t nseg, hipStream_t st, dfmm_tree* t,
                    bool workspaces = true);

// adaptive.hip
int adapt_prune(const dfmm_plan* plan, dfmm_tree* t, hipStream_t st);  // levels -> adaptive levels, leaves
int adapt_lists(const dfmm_plan* plan, dfmm_tree* t, hipStream_t st);  // U, W, X lists, point leaves
// near-coincident pairs over the U lists: counts (fill = false) or the pairs
int adapt_close_find(const dfmm_plan* plan, dfmm_tree* t, bool fill, int* cnt, const int* cstart, int2* cpair,
                     hipStream_t st);
template <typename T>
int adapt_near(const dfmm_plan* plan, dfmm_tree* t, hipStream_t st);    // U lists (writes sig)
template <typename T>
int adapt_m2p(const dfmm_plan* plan, dfmm_tree* t, const T* W, hipStream_t st);  // W lists (adds to sig)
template <typename T>
int adapt_p2l(const dfmm_plan* plan, dfmm_tree* t, T* s, hipStream_t st);        // X lists (adds to s)
template <typename T>
int adapt_l2p(const dfmm_plan* plan, dfmm_tree* t, const T* s, hipStream_t st);  // adds to sig

// fmm.hip
void fmm_prepare(const dfmm_plan* plan);  // one-time kernel attributes (outside graph capture)
int fmm_forces_impl(const dfmm_plan* plan, dfmm_tree* t, const double* seg, const double* burg,
                    double* forces, hipStream_t st);
int direct_forces_impl(const dfmm_plan* plan, const double* seg, const double* burg, int64_t nseg,
                       const int64_t* targets, int64_t ntgt, double* forces, int fp32, hipStream_t st);
int direct_forces_noalloc_impl(const dfmm_plan* plan, const double* seg, const double* burg, int64_t nseg,
                               const int64_t* targets, int64_t ntgt, double* forces, int fp32, hipStream_t st);
size_t direct_noalloc_bytes(const dfmm_plan* plan, int64_t nseg, int64_t ntgt);

}  // namespace dfmm

#define DFMM_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      dfmm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                 \
      return DFMM_E_HIP;                                                                 \
    }                                                                                    \
  } while (0)

#define DFMM_D2H(dst, src, bytes, st)                                                   \
  do {                                                                                   \
    DFMM_HIP(hipMemcpyAsync((dst), (src), (bytes), hipMemcpyDeviceToHost, (st)));        \
    DFMM_HIP(hipStreamSynchronize(st));                                                  \
  } while (0)

#define DFMM_LAUNCH_CHECK()                                                              \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess) {                                                              \
      dfmm::set_error(std::string("kernel launch: ") + hipGetErrorString(e_) + " at " +   \
                      __FILE__ + ":" + std::to_string(__LINE__));                        \
      return DFMM_E_HIP;                                                                 \
    }                                                                                    \
  } while (0)
