// Adaptive octree (the partition step of Sec. 3 taken until every leaf cell
// holds at most leaf_max points) and the FMM kernels that only such a tree
// needs.
//
// The uniform build gives the occupied cells of every level down to D.  The
// adaptive tree keeps a cell when its parent is kept and is not a leaf (every
// cell of level 2 is kept: the M2L starts there); a kept cell is a leaf when
// it holds at most leaf_max points or lies on level D.  On the kept cells
// P2M (at every leaf), M2M, the M2L over the interaction lists (children of
// the parent's neighbours that are not neighbours, now among kept cells) and
// L2L are those of Alg. lagrange.  Leaves of different levels meet in three
// more lists ("adjacent" = the closed boxes touch):
//   U(B), leaf B: the adjacent leaves of any level, B included: direct sum;
//   W(B), leaf B: the cells A finer than B, not adjacent to B, whose parent
//         is adjacent to B: A's multipole weights act on B's points as point
//         sources at A's nodes (the weights W_m of the Lagrange FMM are the
//         strengths of sources at the nodes y_m);
//   X(A): the leaves B with A in W(B): B's points act on A's nodes, whose
//         values are A's local expansion.
// Every pair is found from its finer side by looking up, on each coarser
// level, the few cells that touch a box (binary search in the level's sorted
// keys); pair arrays are sorted by target into CSR lists.
#include <algorithm>
#include <vector>

#include "internal.h"
#include "kernel_eval.h"
#include "morton.h"

namespace dfmm {

struct LevelTab {
  const uint32_t* key[kMaxLevels + 1];
  int n[kMaxLevels + 1];
  int off[kMaxLevels + 1];  // global index of the level's first cell
};

static inline unsigned nbk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------- pruning
// Points below each cell of a level and its first sorted point: at level D
// the cell's own range, above it the sum over its children (level l + 1).
__global__ void k_sub_pts(const int* first, const int* count, int n, const int* cnp, const int* cpf, int* np,
                          int* pf) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if (!cnp) {
    np[c] = count[c];
    pf[c] = first[c];
    return;
  }
  int s = 0;
  for (int k = 0; k < count[c]; ++k) s += cnp[first[c] + k];
  np[c] = s;
  pf[c] = cpf[first[c]];
}

// Kept and leaf flags of a level from its parent level's.
__global__ void k_prune(const int* parent, int n, const int* pkeep, const int* pleaf, const int* np, int leaf_max,
                        int last, int* keep, int* leaf, int* kl) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k = parent ? (pkeep[parent[c]] && !pleaf[parent[c]]) : 1;
  const int lf = k && (last || np[c] <= leaf_max);
  keep[c] = k;
  leaf[c] = lf;
  kl[c] = lf;
}

// The kept cells of a level, renumbered: key, parent (in the parent level's
// numbering), children range (in the child level's numbering; none for a
// leaf).  All children of a kept cell that is not a leaf are kept, so they
// stay contiguous.
__global__ void k_compact(int n, const int* keep, const int* leaf, const int* nidx, const uint32_t* key,
                          const int* first, const int* count, const int* parent, const int* pnidx,
                          const int* cnidx, uint32_t* key2, int* first2, int* count2, int* parent2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !keep[c]) return;
  const int i = nidx[c];
  key2[i] = key[c];
  if (parent2) parent2[i] = pnidx[parent[c]];
  if (leaf[c]) {
    first2[i] = 0;
    count2[i] = 0;
  } else {
    first2[i] = cnidx[first[c]];
    count2[i] = count[c];
  }
}

// Global per-cell arrays of a level's kept cells, and its leaves (ordinals
// lord + their rank among the level's leaves).
__global__ void k_leaf_emit(int n, const int* keep, const int* leaf, const int* nidx, const int* lidx, const int* np,
                            const int* pf, const uint32_t* key, int level, int goff, int lord, int* gl_cell,
                            int* gl_pf, int* gl_pc, uint32_t* gkey, unsigned char* glev, int* gord, int* gsf,
                            int* gsn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !keep[c]) return;
  const int g = goff + nidx[c];
  gkey[g] = key[c];
  glev[g] = (unsigned char)level;
  gsf[g] = pf[c];
  gsn[g] = np[c];
  if (leaf[c]) {
    const int o = lord + lidx[c];
    gl_cell[o] = g;
    gl_pf[o] = pf[c];
    gl_pc[o] = np[c];
    gord[g] = o;
  } else {
    gord[g] = -1;
  }
}

int adapt_prune(const dfmm_plan* pl, dfmm_tree* t, hipStream_t st) {
  const int D = t->D;
  const int lm = pl->prm.leaf_max;
  std::vector<int*> np(D + 1, nullptr), pf(D + 1, nullptr), keep(D + 1, nullptr), leaf(D + 1, nullptr),
      kl(D + 1, nullptr), nidx(D + 1, nullptr), lidx(D + 1, nullptr);
  std::vector<int64_t> nkeep(D + 1, 0), nlf(D + 1, 0);
  auto cleanup = [&]() {
    for (int l = 0; l <= D; ++l) {
      hipFree(np[l]); hipFree(pf[l]); hipFree(keep[l]); hipFree(leaf[l]); hipFree(kl[l]); hipFree(nidx[l]);
      hipFree(lidx[l]);
    }
  };
  int rc = DFMM_OK;
#define ACHK(call)                       \
  do {                                   \
    if ((call) != hipSuccess) {          \
      cleanup();                         \
      set_error("adaptive tree: " #call); \
      return DFMM_E_HIP;                 \
    }                                    \
  } while (0)
  for (int l = D; l >= 2; --l) {
    const int64_t n = t->lv[l].n;
    ACHK(hipMalloc(&np[l], sizeof(int) * (n + 1)));
    ACHK(hipMalloc(&pf[l], sizeof(int) * (n + 1)));
    k_sub_pts<<<nbk(n, 256), 256, 0, st>>>(t->lv[l].first, t->lv[l].count, (int)n, l == D ? nullptr : np[l + 1],
                                          l == D ? nullptr : pf[l + 1], np[l], pf[l]);
    ACHK(hipGetLastError());
  }
  for (int l = 2; l <= D; ++l) {
    const int64_t n = t->lv[l].n;
    ACHK(hipMalloc(&keep[l], sizeof(int) * (n + 1)));
    ACHK(hipMalloc(&leaf[l], sizeof(int) * (n + 1)));
    ACHK(hipMalloc(&kl[l], sizeof(int) * (n + 1)));
    ACHK(hipMalloc(&nidx[l], sizeof(int) * (n + 1)));
    ACHK(hipMalloc(&lidx[l], sizeof(int) * (n + 1)));
    k_prune<<<nbk(n, 256), 256, 0, st>>>(l == 2 ? nullptr : t->lv[l].parent, (int)n, keep[l - 1], leaf[l - 1],
                                        np[l], lm, l == D, keep[l], leaf[l], kl[l]);
    ACHK(hipGetLastError());
    if ((rc = scan_excl(keep[l], nidx[l], n, st, &nkeep[l])) || (rc = scan_excl(kl[l], lidx[l], n, st, &nlf[l]))) {
      cleanup();
      return rc;
    }
  }
  // deepest level with kept cells
  int De = 2;
  for (int l = 2; l <= D; ++l)
    if (nkeep[l] > 0) De = l;
  int64_t ncell = 0, nleaf = 0;
  std::vector<int64_t> goff(D + 1, 0), lord(D + 1, 0);
  for (int l = 2; l <= De; ++l) {
    goff[l] = ncell;
    lord[l] = nleaf;
    ncell += nkeep[l];
    nleaf += nlf[l];
  }
  if (ncell >= ((int64_t)1 << 31) || nleaf < 1) {
    cleanup();
    set_error("adaptive tree: unexpected cell counts");
    return DFMM_E_STATE;
  }
  ACHK(hipMalloc(&t->gl_cell, sizeof(int) * nleaf));
  ACHK(hipMalloc(&t->gl_pf, sizeof(int) * nleaf));
  ACHK(hipMalloc(&t->gl_pc, sizeof(int) * nleaf));
  ACHK(hipMalloc(&t->gkey, sizeof(uint32_t) * ncell));
  ACHK(hipMalloc(&t->glev, ncell));
  ACHK(hipMalloc(&t->gord, sizeof(int) * ncell));
  ACHK(hipMalloc(&t->gsf, sizeof(int) * ncell));
  ACHK(hipMalloc(&t->gsn, sizeof(int) * ncell));
  std::vector<dfmm_tree::Level> nl(D + 1);
  for (int l = 2; l <= De; ++l) {
    const int64_t n = t->lv[l].n, m = nkeep[l];
    auto& L = nl[l];
    L.n = m;
    ACHK(hipMalloc(&L.key, sizeof(uint32_t) * std::max<int64_t>(m, 1)));
    ACHK(hipMalloc(&L.first, sizeof(int) * std::max<int64_t>(m, 1)));
    ACHK(hipMalloc(&L.count, sizeof(int) * std::max<int64_t>(m, 1)));
    if (l > 2) ACHK(hipMalloc(&L.parent, sizeof(int) * std::max<int64_t>(m, 1)));
    k_compact<<<nbk(n, 256), 256, 0, st>>>((int)n, keep[l], leaf[l], nidx[l], t->lv[l].key, t->lv[l].first,
                                          t->lv[l].count, t->lv[l].parent, l > 2 ? nidx[l - 1] : nullptr,
                                          l < D ? nidx[l + 1] : nullptr, L.key, L.first, L.count, L.parent);
    ACHK(hipGetLastError());
    k_leaf_emit<<<nbk(n, 256), 256, 0, st>>>((int)n, keep[l], leaf[l], nidx[l], lidx[l], np[l], pf[l],
                                            t->lv[l].key, l, (int)goff[l], (int)lord[l], t->gl_cell, t->gl_pf,
                                            t->gl_pc, t->gkey, t->glev, t->gord, t->gsf, t->gsn);
    ACHK(hipGetLastError());
  }
  ACHK(hipStreamSynchronize(st));
  cleanup();
#undef ACHK
  for (int l = 2; l <= D; ++l) {
    auto& L = t->lv[l];
    hipFree(L.key); hipFree(L.first); hipFree(L.count); hipFree(L.parent);
    L = nl[l];
    t->leaf_off[l] = lord[l];
    t->leaf_n[l] = l <= De ? nlf[l] : 0;
  }
  t->lv.resize(De + 1);
  t->D = De;
  t->nleaf = nleaf;
  t->adaptive = 1;
  return DFMM_OK;
}

// ---------------------------------------------------------------- lists
// Cells of level l2 whose closed boxes touch the box of cell (x, y, z) of a
// level sh finer: per axis from floor(x / 2^sh) - 1 (only when x is a multiple
// of 2^sh) to floor((x + 1) / 2^sh), inside the level.
__device__ __forceinline__ void touch_range(int x, int sh, int ns, int& lo, int& hi) {
  const int mask = (1 << sh) - 1;
  lo = max(0, (x >> sh) - ((x & mask) ? 0 : 1));
  hi = min(ns - 1, (x + 1) >> sh);
}

// U pairs: each leaf emits (itself, C) for every leaf C of its own or a
// coarser level that touches it (itself included), and (C, itself) when C is
// coarser.  FILL = false counts per leaf.
template <bool FILL>
__global__ void k_upairs(int nleaf, const int* gl_cell, const uint32_t* gkey, const unsigned char* glev,
                         LevelTab lt, const int* gord, int* cnt, const int* start, uint32_t* tgt, uint32_t* src) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nleaf) return;
  const int c = gl_cell[o], l = glev[c];
  int xs[3];
  demorton(gkey[c], xs[0], xs[1], xs[2]);
  int k = 0;
  int64_t w = FILL ? start[o] : 0;
  for (int l2 = 2; l2 <= l; ++l2) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) touch_range(xs[d], l - l2, 1 << l2, lo[d], hi[d]);
    for (int X = lo[0]; X <= hi[0]; ++X)
      for (int Y = lo[1]; Y <= hi[1]; ++Y)
        for (int Z = lo[2]; Z <= hi[2]; ++Z) {
          const int r = bsearch_key(lt.key[l2], lt.n[l2], morton(X, Y, Z));
          if (r < 0) continue;
          const int a = gord[lt.off[l2] + r];
          if (a < 0) continue;
          if (FILL) {
            tgt[w] = (uint32_t)o;
            src[w] = (uint32_t)a;
            ++w;
            if (l2 < l) {
              tgt[w] = (uint32_t)a;
              src[w] = (uint32_t)o;
              ++w;
            }
          }
          k += l2 < l ? 2 : 1;
        }
  }
  if (!FILL) cnt[o] = k;
}

// W/X pairs: each kept cell A of level >= 3 emits (A, B) for every leaf B of
// a coarser level that touches A's parent but not A.  The emissions of a
// cell are its X list; sorted by B they are the W lists.
template <bool FILL>
__global__ void k_wxpairs(int ncell, const uint32_t* gkey, const unsigned char* glev, LevelTab lt, const int* gord,
                          int* cnt, const int* start, int* xsrc, uint32_t* wtgt, uint32_t* wsrc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int la = glev[c];
  int k = 0;
  if (la >= 3) {
    int xs[3], ps[3];
    demorton(gkey[c], xs[0], xs[1], xs[2]);
    for (int d = 0; d < 3; ++d) ps[d] = xs[d] >> 1;
    int64_t w = FILL ? start[c] : 0;
    for (int l2 = 2; l2 <= la - 1; ++l2) {
      const int sh = la - 1 - l2;
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) touch_range(ps[d], sh, 1 << l2, lo[d], hi[d]);
      for (int X = lo[0]; X <= hi[0]; ++X)
        for (int Y = lo[1]; Y <= hi[1]; ++Y)
          for (int Z = lo[2]; Z <= hi[2]; ++Z) {
            // adjacent to A itself?  boxes in units of A's level
            const int C[3] = {X, Y, Z};
            bool adj = true;
            for (int d = 0; d < 3; ++d)
              adj = adj && ((C[d] << (sh + 1)) <= xs[d] + 1) && (((C[d] + 1) << (sh + 1)) >= xs[d]);
            if (adj) continue;
            const int r = bsearch_key(lt.key[l2], lt.n[l2], morton(X, Y, Z));
            if (r < 0) continue;
            const int b = gord[lt.off[l2] + r];
            if (b < 0) continue;
            if (FILL) {
              xsrc[w] = b;
              wtgt[w] = (uint32_t)b;
              wsrc[w] = (uint32_t)c;
              ++w;
            }
            ++k;
          }
    }
  }
  if (!FILL) cnt[c] = k;
}

__global__ void k_count_tgt(const uint32_t* tgt, int64_t n, int* cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) atomicAdd(&cnt[tgt[k]], 1);
}

// Cells with an X list through their nodes (more than pmax points below),
// or (gsn == nullptr) entries with a non-empty list.
__global__ void k_nonempty(const int* start, int n, const int* gsn, int pmax, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (start[i + 1] > start[i] && (!gsn || gsn[i] > pmax)) ? 1 : 0;
}

// Direct source ranges of each leaf (FILL = false counts): its U leaves, the
// cells of its W list with at most pmax points below, and, for each of its
// cells from its own up to level 3 with at most pmax points below, the
// leaves of that cell's X list (whose points then act on all points below
// the cell).
template <bool FILL>
__global__ void k_direct_lists(int nleaf, const int* gl_cell, const int* gl_pf, const int* gl_pc,
                               const uint32_t* gkey, const unsigned char* glev, LevelTab lt, const int* ustart,
                               const int* usrc, const int* wstart, const int* wsrc, const int* xstart,
                               const int* xsrc, const int* gsf, const int* gsn, int pmax, int* cnt,
                               const int* start, int2* out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nleaf) return;
  int k = 0;
  int64_t w = FILL ? start[o] : 0;
  auto emit = [&](int f, int n) {
    if (FILL) out[w++] = make_int2(f, n);
    ++k;
  };
  for (int q = ustart[o]; q < ustart[o + 1]; ++q) emit(gl_pf[usrc[q]], gl_pc[usrc[q]]);
  for (int q = wstart[o]; q < wstart[o + 1]; ++q) {
    const int a = wsrc[q];
    if (gsn[a] <= pmax) emit(gsf[a], gsn[a]);
  }
  const int c = gl_cell[o], l = glev[c];
  const uint32_t key = gkey[c];
  for (int la = l; la >= 3; --la) {
    const int r = bsearch_key(lt.key[la], lt.n[la], key >> (3 * (l - la)));
    if (r < 0) continue;  // cannot happen: the ancestors of a kept cell are kept
    const int g = lt.off[la] + r;
    if (gsn[g] > pmax) continue;
    for (int q = xstart[g]; q < xstart[g + 1]; ++q) emit(gl_pf[xsrc[q]], gl_pc[xsrc[q]]);
  }
  if (!FILL) cnt[o] = k;
}

__global__ void k_compact_idx(const int* flag, const int* pos, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = i;
}

__global__ void k_point_leaf_ad(const int* pf, const int* pc, int nleaf, int* pleaf) {
  const int o = blockIdx.x;
  if (o >= nleaf) return;
  for (int k = threadIdx.x; k < pc[o]; k += blockDim.x) pleaf[pf[o] + k] = o;
}

// near-field point pairs of the U lists, summed (for reporting)
__global__ void k_u_pairs_sum(const int* dstart, const int2* drange, const int* pc, int nleaf,
                              unsigned long long* total) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nleaf) return;
  unsigned long long s = 0;
  for (int q = dstart[o]; q < dstart[o + 1]; ++q) s += (unsigned long long)drange[q].y;
  atomicAdd(total, s * (unsigned long long)pc[o]);
}

static LevelTab level_tab(const dfmm_tree* t) {
  LevelTab lt{};
  for (int l = 2; l <= t->D; ++l) {
    lt.key[l] = t->lv[l].key;
    lt.n[l] = (int)t->lv[l].n;
    lt.off[l] = (int)t->lv[l].off;
  }
  return lt;
}

// CSR over nt targets from (tgt, src) pairs: sorted by source, then stably by
// target; start[] from the per-target counts.  tgt/src are overwritten.
static int pairs_to_csr(uint32_t*& tgt, uint32_t*& src, int64_t np, int64_t nt, int* start, hipStream_t st) {
  int* cnt = nullptr;
  DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (nt + 1)));
  DFMM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (nt + 1), st));
  int rc = DFMM_OK;
  if (np > 0) {
    int bits = 1;
    while (((int64_t)1 << bits) < std::max<int64_t>(nt, 2)) ++bits;
    // sources are cell or leaf indices below 2^31
    rc = radix_sort(src, tgt, np, 32, st);
    if (rc == DFMM_OK) rc = radix_sort(tgt, src, np, bits, st);
    if (rc == DFMM_OK) {
      k_count_tgt<<<nbk(np, 256), 256, 0, st>>>(tgt, np, cnt);
      if (hipGetLastError() != hipSuccess) rc = DFMM_E_HIP;
    }
  }
  int64_t tot = 0;
  if (rc == DFMM_OK) rc = scan_excl(cnt, start, nt + 1, st, &tot);
  hipFree(cnt);
  if (rc == DFMM_OK && tot != np) {
    set_error("adaptive tree: list counts do not add up");
    rc = DFMM_E_STATE;
  }
  return rc;
}

int adapt_lists(const dfmm_plan* pl, dfmm_tree* t, hipStream_t st) {
  const int64_t nleaf = t->nleaf, ncell = t->ncell_total;
  const LevelTab lt = level_tab(t);
  int rc = DFMM_OK;
  // U lists
  {
    int* cnt = nullptr;
    int* start = nullptr;
    DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (nleaf + 1)));
    DFMM_HIP(hipMalloc(&start, sizeof(int) * (nleaf + 1)));
    DFMM_HIP(hipMemsetAsync(cnt + nleaf, 0, sizeof(int), st));
    k_upairs<false><<<nbk(nleaf, 128), 128, 0, st>>>((int)nleaf, t->gl_cell, t->gkey, t->glev, lt, t->gord, cnt,
                                                    nullptr, nullptr, nullptr);
    DFMM_LAUNCH_CHECK();
    int64_t np = 0;
    rc = scan_excl(cnt, start, nleaf + 1, st, &np);
    hipFree(cnt);
    if (rc) {
      hipFree(start);
      return rc;
    }
    uint32_t *tg = nullptr, *sr = nullptr;
    DFMM_HIP(hipMalloc(&tg, sizeof(uint32_t) * std::max<int64_t>(np, 1)));
    DFMM_HIP(hipMalloc(&sr, sizeof(uint32_t) * std::max<int64_t>(np, 1)));
    k_upairs<true><<<nbk(nleaf, 128), 128, 0, st>>>((int)nleaf, t->gl_cell, t->gkey, t->glev, lt, t->gord, nullptr,
                                                   start, tg, sr);
    DFMM_LAUNCH_CHECK();
    hipFree(start);
    DFMM_HIP(hipMalloc(&t->ustart, sizeof(int) * (nleaf + 1)));
    rc = pairs_to_csr(tg, sr, np, nleaf, t->ustart, st);
    hipFree(tg);
    if (rc) {
      hipFree(sr);
      return rc;
    }
    t->usrc = (int*)sr;
    t->nu = np;
  }
  // W and X lists
  {
    int* cnt = nullptr;
    DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (ncell + 1)));
    DFMM_HIP(hipMalloc(&t->xstart, sizeof(int) * (ncell + 1)));
    DFMM_HIP(hipMemsetAsync(cnt + ncell, 0, sizeof(int), st));
    k_wxpairs<false><<<nbk(ncell, 128), 128, 0, st>>>((int)ncell, t->gkey, t->glev, lt, t->gord, cnt, nullptr,
                                                     nullptr, nullptr, nullptr);
    DFMM_LAUNCH_CHECK();
    int64_t np = 0;
    rc = scan_excl(cnt, t->xstart, ncell + 1, st, &np);
    hipFree(cnt);
    if (rc) return rc;
    uint32_t *tg = nullptr, *sr = nullptr;
    DFMM_HIP(hipMalloc(&t->xsrc, sizeof(int) * std::max<int64_t>(np, 1)));
    DFMM_HIP(hipMalloc(&tg, sizeof(uint32_t) * std::max<int64_t>(np, 1)));
    DFMM_HIP(hipMalloc(&sr, sizeof(uint32_t) * std::max<int64_t>(np, 1)));
    k_wxpairs<true><<<nbk(ncell, 128), 128, 0, st>>>((int)ncell, t->gkey, t->glev, lt, t->gord, nullptr, t->xstart,
                                                    t->xsrc, tg, sr);
    DFMM_LAUNCH_CHECK();
    t->nx = np;
    t->nw = np;
    DFMM_HIP(hipMalloc(&t->wstart, sizeof(int) * (nleaf + 1)));
    rc = pairs_to_csr(tg, sr, np, nleaf, t->wstart, st);
    hipFree(tg);
    if (rc) {
      hipFree(sr);
      return rc;
    }
    t->wsrc = (int*)sr;
  }
  // A W or X pair whose finer cell holds at most p^3 points is summed
  // directly (p^3 evaluations per point through the nodes would cost more):
  // the cells whose X list goes through their nodes, the leaves with a W
  // list, and the direct source ranges of every leaf
  const int pmax = pl->p * pl->p * pl->p;
  {
    const int64_t nmax = std::max(ncell, nleaf);
    int *flag = nullptr, *pos = nullptr;
    DFMM_HIP(hipMalloc(&flag, sizeof(int) * (nmax + 1)));
    DFMM_HIP(hipMalloc(&pos, sizeof(int) * (nmax + 1)));
    for (int which = 0; which < 2 && rc == DFMM_OK; ++which) {
      const int64_t n = which ? nleaf : ncell;
      const int* start = which ? t->wstart : t->xstart;
      k_nonempty<<<nbk(n, 256), 256, 0, st>>>(start, (int)n, which ? nullptr : t->gsn, pmax, flag);
      DFMM_LAUNCH_CHECK();
      int64_t m = 0;
      rc = scan_excl(flag, pos, n, st, &m);
      if (rc) break;
      int*& out = which ? t->wleaves : t->xcells;
      DFMM_HIP(hipMalloc(&out, sizeof(int) * std::max<int64_t>(m, 1)));
      k_compact_idx<<<nbk(n, 256), 256, 0, st>>>(flag, pos, (int)n, out);
      DFMM_LAUNCH_CHECK();
      (which ? t->nwleaf : t->nxcell) = m;
    }
    hipFree(flag);
    hipFree(pos);
    if (rc) return rc;
  }
  {
    int* cnt = nullptr;
    DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (nleaf + 1)));
    DFMM_HIP(hipMalloc(&t->dstart, sizeof(int) * (nleaf + 1)));
    DFMM_HIP(hipMemsetAsync(cnt + nleaf, 0, sizeof(int), st));
    k_direct_lists<false><<<nbk(nleaf, 128), 128, 0, st>>>(
        (int)nleaf, t->gl_cell, t->gl_pf, t->gl_pc, t->gkey, t->glev, lt, t->ustart, t->usrc, t->wstart, t->wsrc,
        t->xstart, t->xsrc, t->gsf, t->gsn, pmax, cnt, nullptr, nullptr);
    DFMM_LAUNCH_CHECK();
    rc = scan_excl(cnt, t->dstart, nleaf + 1, st, &t->nd);
    hipFree(cnt);
    if (rc) return rc;
    DFMM_HIP(hipMalloc(&t->drange, sizeof(int2) * std::max<int64_t>(t->nd, 1)));
    k_direct_lists<true><<<nbk(nleaf, 128), 128, 0, st>>>(
        (int)nleaf, t->gl_cell, t->gl_pf, t->gl_pc, t->gkey, t->glev, lt, t->ustart, t->usrc, t->wstart, t->wsrc,
        t->xstart, t->xsrc, t->gsf, t->gsn, pmax, nullptr, t->dstart, t->drange);
    DFMM_LAUNCH_CHECK();
  }
  // leaf of every sorted point, and the near-field pair count
  DFMM_HIP(hipMalloc(&t->pleaf, sizeof(int) * t->N));
  k_point_leaf_ad<<<(unsigned)nleaf, 64, 0, st>>>(t->gl_pf, t->gl_pc, (int)nleaf, t->pleaf);
  DFMM_LAUNCH_CHECK();
  unsigned long long* tot = nullptr;
  DFMM_HIP(hipMalloc(&tot, sizeof(unsigned long long)));
  DFMM_HIP(hipMemsetAsync(tot, 0, sizeof(unsigned long long), st));
  k_u_pairs_sum<<<nbk(nleaf, 256), 256, 0, st>>>(t->dstart, t->drange, t->gl_pc, (int)nleaf, tot);
  DFMM_LAUNCH_CHECK();
  unsigned long long h = 0;
  DFMM_HIP(hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, st));
  DFMM_HIP(hipStreamSynchronize(st));
  hipFree(tot);
  t->near_pairs = (int64_t)h;
  return DFMM_OK;
}

// Near-coincident pairs of the direct sums (single precision): per sorted
// target point, the sources closer than 2a in its leaf's direct source
// ranges (the U leaves and the W/X pairs summed directly: cells finer than
// 2a can be closer than 2a without touching), in the order of the ranges
// and then of the points.  The relation is symmetric, as the close-pair pass
// needs: j lies in a direct range of i's leaf iff i lies in one of j's.
template <bool FILL>
__global__ void k_close_find_u(const double* pts, int64_t N, const int* pleaf, const int* dstart,
                               const int2* drange, double a2x4, int* cnt, const int* cstart, int2* cpair) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int g = pleaf[i];
  const double x0 = pts[i], x1 = pts[N + i], x2 = pts[2 * N + i];
  int c = 0;
  int64_t w = FILL ? cstart[i] : 0;
  for (int q = dstart[g]; q < dstart[g + 1]; ++q) {
    const int2 rg = drange[q];
    for (int jj = 0; jj < rg.y; ++jj) {
      const int64_t j = rg.x + jj;
      const double d0 = x0 - pts[j], d1 = x1 - pts[N + j], d2 = x2 - pts[2 * N + j];
      if (j != i && d0 * d0 + d1 * d1 + d2 * d2 < a2x4) {
        if (FILL)
          cpair[w++] = make_int2((int)i, (int)j);
        else
          ++c;
      }
    }
  }
  if (!FILL) cnt[i] = c;
}

int adapt_close_find(const dfmm_plan* pl, dfmm_tree* t, bool fill, int* cnt, const int* cstart, int2* cpair,
                     hipStream_t st) {
  const double a2x4 = 4.0 * pl->prm.core_a * pl->prm.core_a;
  if (fill)
    k_close_find_u<true><<<nbk(t->N, 128), 128, 0, st>>>(t->pts, t->N, t->pleaf, t->dstart, t->drange, a2x4,
                                                         nullptr, cstart, cpair);
  else
    k_close_find_u<false><<<nbk(t->N, 128), 128, 0, st>>>(t->pts, t->N, t->pleaf, t->dstart, t->drange, a2x4, cnt,
                                                          nullptr, nullptr);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

// ----------------------------------------------------------- FMM kernels
// sig[6] -= (general 9-component strength q[w*3 + r]) seen through dG (D):
// contract_b_t is bilinear in (b, t), so a general q = sum_w e_w (x) q[w, :]
// is three rank-one terms; E_v(b) is linear in b, and F_v = sum_w q[w,:] x E_v(e_w).
template <typename T>
__device__ __forceinline__ void contract_q(const T* D, T c12, T c44, T hh, const T* q, T* sig) {
  T F[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = T(0);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const T* Dv = D + v * 9;  // Dv[p*3+q] = d_q G_vp
    const T tr = Dv[0] + Dv[4] + Dv[8];
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      T E[3];
#pragma unroll
      for (int n = 0; n < 3; ++n)
        E[n] = (n == w ? c12 * tr + hh * Dv[n * 3 + n] : T(0)) + c44 * (Dv[w * 3 + n] + Dv[n * 3 + w]);
      const T* t = q + 3 * w;
      F[v * 3 + 0] += t[1] * E[2] - t[2] * E[1];
      F[v * 3 + 1] += t[2] * E[0] - t[0] * E[2];
      F[v * 3 + 2] += t[0] * E[1] - t[1] * E[0];
    }
  }
  const T trF = F[0] + F[4] + F[8];
  sig[0] -= c12 * trF + (T(2) * c44 + hh) * F[0];
  sig[1] -= c12 * trF + (T(2) * c44 + hh) * F[4];
  sig[2] -= c12 * trF + (T(2) * c44 + hh) * F[8];
  sig[3] -= c44 * (F[5] + F[7]);
  sig[4] -= c44 * (F[2] + F[6]);
  sig[5] -= c44 * (F[1] + F[3]);
}

__device__ __forceinline__ void cell_origin(uint32_t key, int level, const double* lo, double L, double* o,
                                            double* s) {
  int c[3];
  demorton(key, c[0], c[1], c[2]);
  *s = ldexp(L, -level);
  for (int d = 0; d < 3; ++d) o[d] = lo[d] + c[d] * *s;
}

// Lanes of a wave over a block of nt targets: passes of 64 targets with one
// lane each, then the remainder in power-of-two chunks with S = 64 / chunk
// lanes per target splitting its sources (as the uniform near field).
// (the loop below: c0 steps over the targets, S lanes per target in a pass)

// Direct sums: one wave per leaf, over its direct source ranges (the U
// leaves, and the W/X pairs with few points on the finer side).
// Single precision leaves pairs closer than 2a to the double-precision
// close-pair pass and accumulates with compensation.  Writes sig.
template <typename T, bool MIXED, bool ISO>
__global__ void __launch_bounds__(64) k_leaf_u(const double* pts, int64_t N, const int* gl_pf, const int* gl_pc,
                                               const int* dstart, const int2* drange, Med<T> m, double a2x4,
                                               double* sig) {
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int t0 = gl_pf[leaf], nt = gl_pc[leaf];
  const int u0 = dstart[leaf], nu = dstart[leaf + 1] - u0;
  __shared__ int nb_first[64], nb_cnt[64];
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
    for (int q0 = 0; q0 < nu; q0 += 64) {
      const int nq = min(64, nu - q0);
      __syncthreads();
      if (lane < nq) {
        const int2 rg = drange[u0 + q0 + lane];
        nb_first[lane] = rg.x;
        nb_cnt[lane] = rg.y;
      }
      __syncthreads();
      for (int q = 0; q < nq; ++q) {
        const int fj = nb_first[q], cj = nb_cnt[q];
        if (act) {
          for (int jj = (slice - (base % S) + S) % S; jj < cj; jj += S) {
            const int64_t j = fj + jj;
            const double d0 = xt0 - pts[j], d1 = xt1 - pts[N + j], d2 = xt2 - pts[2 * N + j];
            if (MIXED && d0 * d0 + d1 * d1 + d2 * d2 < a2x4) continue;  // left to the close-pair pass
            T D[27], b[3], tt[3];
            for (int c = 0; c < 3; ++c) b[c] = (T)pts[(3 + c) * N + j], tt[c] = (T)pts[(6 + c) * N + j];
            dg_medium_t<T, ISO>((T)d0, (T)d1, (T)d2, m, D);
            if (MIXED) {
              T ds[6] = {0, 0, 0, 0, 0, 0};
              contract_b_t<T>(D, m.c12, m.c44, m.hh, b, tt, ds);
#pragma unroll
              for (int c = 0; c < 6; ++c) {
                const T y = ds[c] - cmp[c];
                const T z = acc[c] + y;
                cmp[c] = (z - acc[c]) - y;
                acc[c] = z;
              }
            } else {
              contract_b_t<T>(D, m.c12, m.c44, m.hh, b, tt, acc);
            }
          }
        }
        base += cj;
      }
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

// W lists: one wave per leaf with a W list; the multipole weights of each W
// cell act on the leaf's points as point sources at that cell's p^3 nodes.
// Adds to sig.
template <typename T, bool ISO>
__global__ void __launch_bounds__(64) k_m2p(const double* pts, int64_t N, const int* wleaves, const int* gl_pf,
                                            const int* gl_pc, const int* wstart, const int* wsrc,
                                            const uint32_t* gkey, const unsigned char* glev, const int* gsn,
                                            const T* W, Med<T> m, double lo0, double lo1, double lo2, double L,
                                            int p, double* sig) {
  const int leaf = wleaves[blockIdx.x], lane = threadIdx.x;
  const int t0 = gl_pf[leaf], nt = gl_pc[leaf];
  const int p3 = p * p * p;
  const double lo[3] = {lo0, lo1, lo2};
  const double h = 1.0 / (p - 1);
  for (int c0 = 0, per = 64; c0 < nt; c0 += per) {
    const int rem = nt - c0;
    per = 64;
    while (per > rem) per >>= 1;
    const int S = 64 / per;
    const int ti = c0 + lane / S, slice = lane % S;
    const bool act = ti < nt;
    const int64_t i = t0 + (act ? ti : 0);
    const double x[3] = {pts[i], pts[N + i], pts[2 * N + i]};
    T acc[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
      for (int e = wstart[leaf]; e < wstart[leaf + 1]; ++e) {
        const int c = wsrc[e];
        if (gsn[c] <= p3) continue;  // summed directly with the leaf's other sources
        double o[3], s;
        cell_origin(gkey[c], glev[c], lo, L, o, &s);
        const T* Wc = W + (int64_t)c * 9 * p3;
        for (int nd = slice; nd < p3; nd += S) {
          const int a = nd / (p * p), b = (nd / p) % p, cc = nd % p;
          const double y0 = o[0] + s * (a * h), y1 = o[1] + s * (b * h), y2 = o[2] + s * (cc * h);
          T D[27], q[9];
          dg_medium_t<T, ISO>((T)(x[0] - y0), (T)(x[1] - y1), (T)(x[2] - y2), m, D);
#pragma unroll
          for (int k = 0; k < 9; ++k) q[k] = Wc[k * p3 + nd];
          contract_q<T>(D, m.c12, m.c44, m.hh, q, acc);
        }
      }
    }
    double tot[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tot[c] = (double)acc[c];
    for (int o2 = S / 2; o2 >= 1; o2 >>= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) tot[c] += __shfl_xor(tot[c], o2, 64);
    if (act && slice == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sig[i * 6 + c] += tot[c];
    }
  }
}

// X lists: one block per cell with an X list; the points of each X leaf act
// on the cell's nodes (thread = node), staged through LDS in chunks.  Adds to
// the cell's local values s.
constexpr int kP2LThreads = 256;
template <typename T, bool ISO>
__global__ void __launch_bounds__(kP2LThreads) k_p2l(const double* pts, int64_t N, const int* xcells,
                                                     const int* xstart, const int* xsrc, const int* gl_pf,
                                                     const int* gl_pc, const uint32_t* gkey,
                                                     const unsigned char* glev, Med<T> m, double lo0, double lo1,
                                                     double lo2, double L, int p, T* s) {
  __shared__ double sp[kP2LThreads][9];
  const int c = xcells[blockIdx.x];
  const int p3 = p * p * p;
  const double lo[3] = {lo0, lo1, lo2};
  double o[3], sz;
  cell_origin(gkey[c], glev[c], lo, L, o, &sz);
  const double h = 1.0 / (p - 1);
  // nodes tid and tid + 256 (p^3 <= 512)
  T acc[2][6] = {};
  double y[2][3];
  for (int r = 0; r < 2; ++r) {
    const int nd = threadIdx.x + r * kP2LThreads;
    const int a = nd / (p * p), b = (nd / p) % p, cc = nd % p;
    y[r][0] = o[0] + sz * (a * h);
    y[r][1] = o[1] + sz * (b * h);
    y[r][2] = o[2] + sz * (cc * h);
  }
  for (int e = xstart[c]; e < xstart[c + 1]; ++e) {
    const int a = xsrc[e];
    const int f = gl_pf[a], n = gl_pc[a];
    for (int j0 = 0; j0 < n; j0 += kP2LThreads) {
      const int nc = min(kP2LThreads, n - j0);
      __syncthreads();
      if ((int)threadIdx.x < nc)
        for (int k = 0; k < 9; ++k) sp[threadIdx.x][k] = pts[k * N + f + j0 + threadIdx.x];
      __syncthreads();
      for (int r = 0; r < 2; ++r) {
        if ((int)threadIdx.x + r * kP2LThreads >= p3) break;
        for (int j = 0; j < nc; ++j) {
          T D[27], b[3], tt[3];
          for (int k = 0; k < 3; ++k) b[k] = (T)sp[j][3 + k], tt[k] = (T)sp[j][6 + k];
          dg_medium_t<T, ISO>((T)(y[r][0] - sp[j][0]), (T)(y[r][1] - sp[j][1]), (T)(y[r][2] - sp[j][2]), m, D);
          contract_b_t<T>(D, m.c12, m.c44, m.hh, b, tt, acc[r]);
        }
      }
    }
  }
  for (int r = 0; r < 2; ++r) {
    const int nd = threadIdx.x + r * kP2LThreads;
    if (nd >= p3) break;
    T* sc = s + (int64_t)c * 6 * p3;
    for (int k = 0; k < 6; ++k) sc[k * p3 + nd] += acc[r][k];
  }
}

// L2P on an adaptive tree: the local values of each point's leaf (any
// level), interpolated at the point.  Adds to sig.
template <typename T, int P>
__global__ void k_l2p_ad(const double* pts, int64_t N, const int* pleaf, const int* gl_cell, const uint32_t* gkey,
                         const unsigned char* glev, const T* s, double lo0, double lo1, double lo2, double L,
                         double* sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = gl_cell[pleaf[i]];
  const double lo[3] = {lo0, lo1, lo2};
  double o[3], sz;
  cell_origin(gkey[c], glev[c], lo, L, o, &sz);
  constexpr int p3 = P * P * P;
  const T* sl = s + (int64_t)c * 6 * p3;
  T Lb[3][P];
  for (int d = 0; d < 3; ++d) {
    const T t = (T)((pts[d * N + i] - o[d]) / sz);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      // ell_k(t) on the nodes j / (P - 1): numerator product, one division
      T v = T(1);
      int den = 1;
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (j != k) {
          v *= t * T(P - 1) - T(j);
          den *= k - j;
        }
      Lb[d][k] = v / T(den);
    }
  }
  T far[6] = {0, 0, 0, 0, 0, 0};
  for (int l1 = 0; l1 < P; ++l1)
#pragma unroll
    for (int l2 = 0; l2 < P; ++l2) {
      const T w12 = Lb[0][l1] * Lb[1][l2];
#pragma unroll
      for (int l3 = 0; l3 < P; ++l3) {
        const T w = w12 * Lb[2][l3];
        const int node = (l1 * P + l2) * P + l3;
#pragma unroll
        for (int c2 = 0; c2 < 6; ++c2) far[c2] = fma(w, sl[c2 * p3 + node], far[c2]);
      }
    }
#pragma unroll
  for (int c2 = 0; c2 < 6; ++c2) sig[i * 6 + c2] += (double)far[c2];
}

// ----------------------------------------------------------- launchers
template <typename T>
int adapt_near(const dfmm_plan* pl, dfmm_tree* t, hipStream_t st) {
  const Med<T> m = pl->med<T>();
  const double a2x4 = 4.0 * pl->prm.core_a * pl->prm.core_a;
  const unsigned g = (unsigned)t->nleaf;
  if constexpr (std::is_same<T, float>::value) {
    if (pl->iso)
      k_leaf_u<T, true, true><<<g, 64, 0, st>>>(t->pts, t->N, t->gl_pf, t->gl_pc, t->dstart, t->drange, m, a2x4, t->sig);
    else
      k_leaf_u<T, true, false><<<g, 64, 0, st>>>(t->pts, t->N, t->gl_pf, t->gl_pc, t->dstart, t->drange, m, a2x4, t->sig);
  } else {
    if (pl->iso)
      k_leaf_u<T, false, true><<<g, 64, 0, st>>>(t->pts, t->N, t->gl_pf, t->gl_pc, t->dstart, t->drange, m, a2x4, t->sig);
    else
      k_leaf_u<T, false, false><<<g, 64, 0, st>>>(t->pts, t->N, t->gl_pf, t->gl_pc, t->dstart, t->drange, m,
                                                 a2x4, t->sig);
  }
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

template <typename T>
int adapt_m2p(const dfmm_plan* pl, dfmm_tree* t, const T* W, hipStream_t st) {
  if (t->nwleaf == 0) return DFMM_OK;
  const Med<T> m = pl->med<T>();
  const double* lo = pl->prm.box_lo;
  const unsigned g = (unsigned)t->nwleaf;
  if (pl->iso)
    k_m2p<T, true><<<g, 64, 0, st>>>(t->pts, t->N, t->wleaves, t->gl_pf, t->gl_pc, t->wstart, t->wsrc, t->gkey,
                                     t->glev, t->gsn, W, m, lo[0], lo[1], lo[2], pl->prm.box_size, pl->p, t->sig);
  else
    k_m2p<T, false><<<g, 64, 0, st>>>(t->pts, t->N, t->wleaves, t->gl_pf, t->gl_pc, t->wstart, t->wsrc, t->gkey,
                                      t->glev, t->gsn, W, m, lo[0], lo[1], lo[2], pl->prm.box_size, pl->p, t->sig);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

template <typename T>
int adapt_p2l(const dfmm_plan* pl, dfmm_tree* t, T* s, hipStream_t st) {
  if (t->nxcell == 0) return DFMM_OK;
  const Med<T> m = pl->med<T>();
  const double* lo = pl->prm.box_lo;
  const unsigned g = (unsigned)t->nxcell;
  if (pl->iso)
    k_p2l<T, true><<<g, kP2LThreads, 0, st>>>(t->pts, t->N, t->xcells, t->xstart, t->xsrc, t->gl_pf, t->gl_pc,
                                              t->gkey, t->glev, m, lo[0], lo[1], lo[2], pl->prm.box_size, pl->p, s);
  else
    k_p2l<T, false><<<g, kP2LThreads, 0, st>>>(t->pts, t->N, t->xcells, t->xstart, t->xsrc, t->gl_pf, t->gl_pc,
                                               t->gkey, t->glev, m, lo[0], lo[1], lo[2], pl->prm.box_size, pl->p, s);
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

template <typename T>
int adapt_l2p(const dfmm_plan* pl, dfmm_tree* t, const T* s, hipStream_t st) {
  const double* lo = pl->prm.box_lo;
  const unsigned blocks = nbk(t->N, 256);
#define L2PA(P_)                                                                                              \
  k_l2p_ad<T, P_><<<blocks, 256, 0, st>>>(t->pts, t->N, t->pleaf, t->gl_cell, t->gkey, t->glev, s, lo[0], lo[1], \
                                          lo[2], pl->prm.box_size, t->sig)
  switch (pl->p) {
    case 2: L2PA(2); break;
    case 3: L2PA(3); break;
    case 4: L2PA(4); break;
    case 5: L2PA(5); break;
    case 6: L2PA(6); break;
    case 7: L2PA(7); break;
    default: L2PA(8); break;
  }
#undef L2PA
  DFMM_LAUNCH_CHECK();
  return DFMM_OK;
}

template int adapt_near<float>(const dfmm_plan*, dfmm_tree*, hipStream_t);
template int adapt_near<double>(const dfmm_plan*, dfmm_tree*, hipStream_t);
template int adapt_m2p<float>(const dfmm_plan*, dfmm_tree*, const float*, hipStream_t);
template int adapt_m2p<double>(const dfmm_plan*, dfmm_tree*, const double*, hipStream_t);
template int adapt_p2l<float>(const dfmm_plan*, dfmm_tree*, float*, hipStream_t);
template int adapt_p2l<double>(const dfmm_plan*, dfmm_tree*, double*, hipStream_t);
template int adapt_l2p<float>(const dfmm_plan*, dfmm_tree*, const float*, hipStream_t);
template int adapt_l2p<double>(const dfmm_plan*, dfmm_tree*, const double*, hipStream_t);

}  // namespace dfmm
