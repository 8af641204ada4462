// Octree build (partition step of the FMM, Sec. 3 and Sec. 4.3).
//
// Quadrature points get 3D Morton keys of their leaf (every point is binned by
// its own position into half-open cells; points on the upper face of the root
// are clamped in).  A stable LSD radix sort orders (key, point id); run-length
// encoding of the sorted keys gives the occupied leaves, and of the parent
// keys (key >> 3) the occupied cells of each coarser level down to level 2.
// Neighbour lists (27 cells, self included) of the leaves and interaction
// lists (children of the parent's neighbours that are not neighbours, at most
// 189) of every level >= 2 are found by binary search in the sorted keys.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "internal.h"
#include "morton.h"

namespace dfmm {

// --------------------------------------------------------------- points
__global__ void k_make_keys(const double* seg, int64_t nseg, Quad qd, double lo0, double lo1, double lo2,
                            double size, int D, uint32_t* keys, uint32_t* vals, int* err) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = nseg * qd.n;
  if (j >= N) return;
  int64_t i = j / qd.n;
  int k = (int)(j - i * qd.n);
  const double* s = seg + 6 * i;
  double x1[3] = {s[0], s[1], s[2]}, x2[3] = {s[3], s[4], s[5]};
  double lo[3] = {lo0, lo1, lo2};
  int c[3];
  int e = 0;
  const int nside = 1 << D;
  const double sD = size / nside;
  for (int d = 0; d < 3; ++d) {
    if (!isfinite(x1[d]) || !isfinite(x2[d])) e |= 1;
    double y = x1[d] + 0.5 * (1.0 + qd.u[k]) * (x2[d] - x1[d]);
    if (!(y >= lo[d] && y <= lo[d] + size)) e |= 2;
    double f = floor((y - lo[d]) / sD);
    int ci = isfinite(f) ? (int)fmin(fmax(f, 0.0), (double)(nside - 1)) : 0;
    c[d] = ci;
  }
  if (e) atomicOr(err, e);
  keys[j] = morton(c[0], c[1], c[2]);
  vals[j] = (uint32_t)j;
}

// ----------------------------------------------------------------- scan
constexpr int SC_T = 256, SC_I = 8, SC_TILE = SC_T * SC_I;

__device__ __forceinline__ int block_excl_scan(int v, int& total) {
  __shared__ int wsum[SC_T / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
  for (int i = 0; i < SC_T / 64; ++i) {
    if (i < w) pre += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__global__ void k_scan_tiles(const int* in, int* out, int64_t n, int* sums) {
  int64_t base = (int64_t)blockIdx.x * SC_TILE + threadIdx.x * SC_I;
  int v[SC_I], s = 0;
#pragma unroll
  for (int i = 0; i < SC_I; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_excl_scan(s, tot);
#pragma unroll
  for (int i = 0; i < SC_I; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_add_tile_offsets(int* out, int64_t n, const int* offs) {
  int64_t base = (int64_t)blockIdx.x * SC_TILE;
  int add = offs[blockIdx.x];
  for (int i = threadIdx.x; i < SC_TILE; i += SC_T)
    if (base + i < n) out[base + i] += add;
}

// Exclusive scan of in[0..n) into out; returns the total in *total (host).
int scan_excl(const int* in, int* out, int64_t n, hipStream_t st, int64_t* total) {
  int64_t nt = (n + SC_TILE - 1) / SC_TILE;
  int* sums = nullptr;
  int* sums_ex = nullptr;
  DFMM_HIP(hipMalloc(&sums, sizeof(int) * (nt + 1)));
  DFMM_HIP(hipMalloc(&sums_ex, sizeof(int) * (nt + 1)));
  k_scan_tiles<<<(unsigned)nt, SC_T, 0, st>>>(in, out, n, sums);
  DFMM_LAUNCH_CHECK();
  int64_t tot = 0;
  int rc = DFMM_OK;
  if (nt > 1) {
    rc = scan_excl(sums, sums_ex, nt, st, &tot);
    if (rc == DFMM_OK) {
      k_add_tile_offsets<<<(unsigned)nt, SC_T, 0, st>>>(out, n, sums_ex);
      DFMM_LAUNCH_CHECK();
    }
  } else {
    int h = 0;
    DFMM_HIP(hipMemcpyAsync(&h, sums, sizeof(int), hipMemcpyDeviceToHost, st));
    DFMM_HIP(hipStreamSynchronize(st));
    tot = h;
  }
  hipFree(sums);
  hipFree(sums_ex);
  *total = tot;
  return rc;
}

// ----------------------------------------------------------- radix sort
constexpr int RS_T = 256, RS_I = 16, RS_TILE = RS_T * RS_I;

__global__ void k_rs_hist(const uint32_t* keys, int64_t n, int shift, int nblk, int* hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = threadIdx.x; i < RS_TILE; i += RS_T)
    if (base + i < n) atomicAdd(&h[(keys[base + i] >> shift) & 255], 1);
  __syncthreads();
  hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items of a tile are ranked in index order (round, wave, lane).
__global__ void k_rs_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                             int64_t n, int shift, int nblk, const int* offs) {
  __shared__ int run[256];
  __shared__ int wcnt[RS_T / 64][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  run[threadIdx.x] = offs[threadIdx.x * nblk + blockIdx.x];
  for (int i = 0; i < RS_T / 64; ++i) wcnt[i][threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int r = 0; r < RS_I; ++r) {
    int64_t idx = base + (int64_t)r * RS_T + threadIdx.x;
    bool valid = idx < n;
    uint32_t k = valid ? kin[idx] : 0u;
    uint32_t v = valid ? vin[idx] : 0u;
    int d = (k >> shift) & 255;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      uint64_t m = __ballot((d >> bit) & 1);
      peers &= ((d >> bit) & 1) ? m : ~m;
    }
    int rank = __popcll(peers & lt);
    int leader = __ffsll((unsigned long long)peers) - 1;
    if (valid && lane == leader) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pre = 0;
      for (int i = 0; i < w; ++i) pre += wcnt[i][d];
      int64_t pos = (int64_t)run[d] + pre + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    int tot = 0;
    for (int i = 0; i < RS_T / 64; ++i) {
      tot += wcnt[i][threadIdx.x];
      wcnt[i][threadIdx.x] = 0;
    }
    run[threadIdx.x] += tot;
    __syncthreads();
  }
}

// Sort (keys, vals) by the low `bits` bits of keys; result in keys/vals.
int radix_sort(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t st) {
  int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
  uint32_t *k2 = nullptr, *v2 = nullptr;
  int *hist = nullptr, *offs = nullptr;
  DFMM_HIP(hipMalloc(&k2, sizeof(uint32_t) * n));
  DFMM_HIP(hipMalloc(&v2, sizeof(uint32_t) * n));
  DFMM_HIP(hipMalloc(&hist, sizeof(int) * 256 * nblk));
  DFMM_HIP(hipMalloc(&offs, sizeof(int) * 256 * nblk));
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  int rc = DFMM_OK;
  for (int shift = 0; shift < bits && rc == DFMM_OK; shift += 8) {
    k_rs_hist<<<nblk, RS_T, 0, st>>>(ka, n, shift, nblk, hist);
    DFMM_LAUNCH_CHECK();
    int64_t tot;
    rc = scan_excl(hist, offs, (int64_t)256 * nblk, st, &tot);
    if (rc) break;
    k_rs_scatter<<<nblk, RS_T, 0, st>>>(ka, va, kb, vb, n, shift, nblk, offs);
    DFMM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (rc == DFMM_OK && ka != keys) {
    DFMM_HIP(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
    DFMM_HIP(hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
  }
  DFMM_HIP(hipStreamSynchronize(st));
  hipFree(k2);
  hipFree(v2);
  hipFree(hist);
  hipFree(offs);
  return rc;
}

// ---------------------------------------------------------------- cells
__global__ void k_run_flags(const uint32_t* keys, int64_t n, int shift, int* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_run_emit(const uint32_t* keys, int64_t n, int shift, const int* flags, const int* idx,
                           uint32_t* okey, int* ofirst, int* elem_cell) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = idx[i] + flags[i] - 1;
  if (flags[i]) {
    okey[c] = keys[i] >> shift;
    ofirst[c] = (int)i;
  }
  if (elem_cell) elem_cell[i] = c;
}

__global__ void k_run_counts(const int* first, int nc, int64_t n, int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int nx = (i + 1 < nc) ? first[i + 1] : (int)n;
  cnt[i] = nx - first[i];
}

__global__ void k_inverse_perm(const uint32_t* perm, int64_t n, uint32_t* inv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[perm[i]] = (uint32_t)i;
}

__global__ void k_point_leaf(const int* first, const int* count, int nleaf, int* pleaf) {
  const int leaf = blockIdx.x;
  if (leaf >= nleaf) return;
  for (int k = threadIdx.x; k < count[leaf]; k += blockDim.x) pleaf[first[leaf] + k] = leaf;
}

// ---------------------------------------------------------------- lists
__global__ void k_leaf_nbrs(const uint32_t* keys, int nc, int lvl, int* nbr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int x, y, z;
  demorton(keys[i], x, y, z);
  const int ns = 1 << lvl;
  int k = 0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c, ++k) {
        int X = x + a, Y = y + b, Z = z + c;
        int r = -1;
        if (X >= 0 && X < ns && Y >= 0 && Y < ns && Z >= 0 && Z < ns) r = bsearch_key(keys, nc, morton(X, Y, Z));
        nbr[(int64_t)i * 27 + k] = r;
      }
}

// Count (fill == nullptr) or fill the interaction list of every cell of a
// level, in lexicographic order of the source cell (so neighbouring targets
// walk their offsets in the same order).  Entry = (source, 2*canonical id +
// mirrored).
__global__ void k_ilist(const uint32_t* keys, int nc, int lvl, const int* oid343, const int* start, int* cnt,
                        int2* fill) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int x, y, z;
  demorton(keys[i], x, y, z);
  const int ns = 1 << lvl;
  int px = 2 * ((x >> 1) - 1), py = 2 * ((y >> 1) - 1), pz = 2 * ((z >> 1) - 1);
  int k = 0;
  int pos = fill ? start[i] : 0;
  for (int a = 0; a < 6; ++a) {
    int X = px + a;
    if (X < 0 || X >= ns) continue;
    for (int b = 0; b < 6; ++b) {
      int Y = py + b;
      if (Y < 0 || Y >= ns) continue;
      for (int c = 0; c < 6; ++c) {
        int Z = pz + c;
        if (Z < 0 || Z >= ns) continue;
        int ox = x - X, oy = y - Y, oz = z - Z;
        if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
        int r = bsearch_key(keys, nc, morton(X, Y, Z));
        if (r < 0) continue;
        if (fill) fill[pos++] = make_int2(r, oid343[((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3)]);
        ++k;
      }
    }
  }
  if (!fill) cnt[i] = k;
}

// M2L processing order: windows of `win` Morton-consecutive targets (one
// block each, spatially compact), longest lists first inside a window.  The
// length that orders a target is the longest list among its siblings, so that
// siblings (which draw on the same source cells, in the same lexicographic
// order) stay next to each other in a wave.
__global__ void k_sib_len(const int* il_start, const int* parent, int n, int* pmax) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicMax(&pmax[parent[i]], il_start[i + 1] - il_start[i]);
}

__global__ void k_len_keys(const int* il_start, const int* parent, const int* pmax, int n, int win, uint32_t* key,
                           uint32_t* val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int len = parent ? pmax[parent[i]] : il_start[i + 1] - il_start[i];
  key[i] = ((uint32_t)(i / win) << 8) | (uint32_t)(kNumFar - min(len, kNumFar));
  val[i] = (uint32_t)i;
}

// Per wave of kWaveTargets consecutive targets of the
// processing order, the longest list (+ the prefetch pad), and each target's
// list length by processing position.
__global__ void k_wave_len(const uint32_t* order, const int* il_start, int n, int* lenq, int* wlen) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const uint32_t t = order[q];
  const int len = il_start[t + 1] - il_start[t];
  lenq[q] = len;
  atomicMax(&wlen[q / kWaveTargets], len + kIlwPad);
}

// Copy each target's list into its wave's block, step-major, one 32-bit word
// per entry: source cell in bits 0..22, canonical offset in bits 23..30,
// mirror flag in bit 31 (CODE9, the f16 product: offset code 2 id + mirror
// in bits 23..31, its slot among the 316 offsets' spectra).
template <bool CODE9>
__global__ void k_il_wave(const uint32_t* order, const int* il_start, const int2* il, const int* wbase, int n,
                          uint32_t* ilw) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const uint32_t t = order[q];
  const int b = il_start[t], len = il_start[t + 1] - b;
  uint32_t* dst = ilw + (int64_t)kWaveTargets * wbase[q / kWaveTargets] + q % kWaveTargets;
  for (int i = 0; i < len; ++i) {
    const int2 v = il[b + i];
    dst[(int64_t)kWaveTargets * i] = CODE9 ? (uint32_t)v.x | ((uint32_t)v.y << 23)
                                           : (uint32_t)v.x | ((uint32_t)(v.y >> 1) << 23) | ((uint32_t)(v.y & 1) << 31);
  }
}

// Order of the entries inside each list, for the LDS banks of the M2L kernel.
// A 16-byte LDS read is served 16 lanes at a time, and in the kernel those
// lanes are the two lanes of each of 8 consecutive targets of a wave (the
// kernels' lane pair -> target map, pass_target), which at one step read the
// spectra of 8 unrelated offsets: lane h of a target with
// offset id c reads 16-byte unit 29 c + 14 h + i (29 units per offset, lane 1
// from unit 14), bank group (29 c + 14 h + i) mod 16.  Reads of one address are a broadcast; reads of different
// addresses in one bank group are served one after another.  So step by step,
// each group of 8 targets picks, per target, an entry of its remaining list
// whose two bank groups are free or already taken by the same offset (the same
// offset first, then the earliest such entry, else the earliest entry).  This
// only permutes each target's list: 228 -> 208.6 ms of M2L on 1M segments,
// for about 6 ms of tree build.  One wave per group of 8 targets.
template <int kUnits, int kHalf, bool CODE9>
__global__ void k_il_bank(const int* lenq, const int* wbase, int64_t n, int64_t ngroups, uint32_t* ilw) {
  __shared__ uint32_t ent[8][kNumFar + 1];
  __shared__ int used[16];
  const int64_t G = blockIdx.x;
  if (G >= ngroups) return;
  static_assert(kWaveTargets % 8 == 0, "groups of 8 targets per wave");
  constexpr int kGroups = kWaveTargets / 8;
  const int64_t w = G / kGroups;
  const int p = (int)(G % kGroups), lane = threadIdx.x;
  const int64_t base = (int64_t)kWaveTargets * wbase[w];
  int len[8];
  int maxlen = 0;
  for (int j = 0; j < 8; ++j) {
    const int64_t q = w * kWaveTargets + 8 * p + j;
    len[j] = q < n ? lenq[q] : 0;
    maxlen = max(maxlen, len[j]);
    for (int s = lane; s < len[j]; s += 64) ent[j][s] = ilw[base + (int64_t)kWaveTargets * s + 8 * p + j];
  }
  __syncthreads();
  for (int s = 0; s < maxlen; ++s) {
    if (lane < 16) used[lane] = -1;
    __syncthreads();
    for (int j = 0; j < 8; ++j) {
      if (s >= len[j]) continue;
      int best = -1;  // key: priority * 256 + (255 - offset from s)
      for (int c = s + lane; c < len[j]; c += 64) {
        const int code = (int)((ent[j][c] >> 23) & (CODE9 ? 0x1FFu : 0xFFu));
        const int g0 = (kUnits * code) & 15, g1 = (g0 + kHalf) & 15;
        const int u0 = used[g0], u1 = used[g1];
        int pr = 0;
        if ((u0 == -1 || u0 == code) && (u1 == -1 || u1 == code)) pr = (u0 == code) ? 2 : 1;
        best = max(best, pr * 256 + (255 - (c - s)));
      }
      for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
      const int pick = s + (255 - (best & 255));
      __syncthreads();
      if (lane == 0) {
        const uint32_t e = ent[j][pick];
        ent[j][pick] = ent[j][s];
        ent[j][s] = e;
        const int code = (int)((e >> 23) & (CODE9 ? 0x1FFu : 0xFFu));
        const int g0 = (kUnits * code) & 15;
        used[g0] = code;
        used[(g0 + kHalf) & 15] = code;
      }
      __syncthreads();
    }
  }
  for (int j = 0; j < 8; ++j)
    for (int s = lane; s < len[j]; s += 64) ilw[base + (int64_t)kWaveTargets * s + 8 * p + j] = ent[j][s];
}

// Positions of the sorted points (rows 0..2 of the points array), formed as
// the force call's gather forms them.
__global__ void k_gather_pos(const double* seg, const uint32_t* perm, Quad qd, int64_t N, double* pts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t j = perm[i];
  const int64_t s = j / qd.n;
  double x[3], t[3];
  quad_point(seg, s, (int)(j - s * qd.n), qd, x, t);
  for (int d = 0; d < 3; ++d) pts[d * N + i] = x[d];
}

// Debug check that seg holds the positions a tree was built from: every
// sorted point formed again as the force call's gather forms it, compared bit
// for bit with the build's copy; chk[0] counts the points that differ, chk[1]
// keeps the smallest segment index among them.
__global__ void k_pos_check(const double* seg, const uint32_t* perm, Quad qd, int64_t N, const double* pos0,
                            unsigned long long* chk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t j = perm[i];
  const int64_t s = j / qd.n;
  double x[3], t[3];
  quad_point(seg, s, (int)(j - s * qd.n), qd, x, t);
  bool bad = false;
  for (int d = 0; d < 3; ++d) bad |= __double_as_longlong(x[d]) != __double_as_longlong(pos0[d * N + i]);
  if (bad) {
    atomicAdd(&chk[0], 1ull);
    atomicMin(&chk[1], (unsigned long long)s);
  }
}

int check_positions_impl(const dfmm_plan* pl, dfmm_tree* t, const double* seg, hipStream_t st) {
  const int64_t N = t->N;
  const unsigned long long init[2] = {0ull, ~0ull};
  DFMM_HIP(hipMemcpyAsync(t->chk, init, sizeof(init), hipMemcpyHostToDevice, st));
  k_pos_check<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(seg, t->perm, pl->quad, N, t->pos0, t->chk);
  DFMM_LAUNCH_CHECK();
  unsigned long long h[2];
  DFMM_D2H(h, t->chk, sizeof(h), st);
  if (h[0] > 0) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "tree_check_positions: %llu of %lld quadrature points differ from the positions the tree was "
                  "built from (first at segment %llu)",
                  h[0], (long long)N, h[1]);
    set_error(msg);
    return DFMM_E_STATE;
  }
  return DFMM_OK;
}

// Near-coincident pairs of each sorted target point: the sources closer than
// 2a in its leaf's 27 neighbour leaves (the point itself excluded: its own
// term is zero), in the order the near field visits them (neighbour by
// neighbour, then by sorted index).  A neighbour leaf is
// skipped only if its box lies at least 2a from the target (with a relative
// margin of 1e-9 against rounding).  FILL = false counts, true writes.
template <bool FILL>
__global__ void k_close_find(const double* pts, int64_t N, const int* pleaf, const int* first, const int* count,
                             const uint32_t* key, const int* nbr, double lo0, double lo1, double lo2, double sD,
                             double a2x4, int* cnt, const int* cstart, int2* cpair) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int leaf = pleaf[i];
  int cx, cy, cz;
  demorton(key[leaf], cx, cy, cz);
  const double x0 = pts[i], x1 = pts[N + i], x2 = pts[2 * N + i];
  const double r[3] = {x0 - (lo0 + cx * sD), x1 - (lo1 + cy * sD), x2 - (lo2 + cz * sD)};
  const double lim = a2x4 * (1.0 + 1e-9);
  int c = 0;
  int64_t w = FILL ? cstart[i] : 0;
  for (int q = 0; q < 27; ++q) {
    const int o[3] = {q / 9 - 1, q / 3 % 3 - 1, q % 3 - 1};
    double gap = 0.0;
    for (int d = 0; d < 3; ++d)
      if (o[d] < 0)
        gap += r[d] * r[d];
      else if (o[d] > 0)
        gap += (sD - r[d]) * (sD - r[d]);
    const int nl = nbr[(int64_t)leaf * 27 + q];
    if (nl < 0 || gap >= lim) continue;
    const int f = first[nl], n = count[nl];
    for (int jj = 0; jj < n; ++jj) {
      const int64_t j = f + jj;
      const double d0 = x0 - pts[j], d1 = x1 - pts[N + j], d2 = x2 - pts[2 * N + j];
      if (j != i && d0 * d0 + d1 * d1 + d2 * d2 < a2x4) {  // a point's own pair is zero (odd kernel)
        if (FILL)
          cpair[w++] = make_int2((int)i, (int)j);
        else
          ++c;
      }
    }
  }
  if (!FILL) cnt[i] = c;
}

// The close pairs are symmetric ((i, j) listed iff (j, i) is).  One thread
// per listed pair with i < j finds the mirror entry (j, i) in j's list; the
// pair is then evaluated once for both directions (flag pass, then fill).
__global__ void k_close_uni(const int2* cpair, const int* cstart, int64_t nclose, const int* upos, int* flag,
                            int2* cuni) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nclose) return;
  const int2 pr = cpair[k];
  if (!cuni) {
    flag[k] = pr.x < pr.y ? 1 : 0;
    return;
  }
  if (pr.x >= pr.y) return;
  int mk = -1;
  for (int r = cstart[pr.y]; r < cstart[pr.y + 1]; ++r)
    if (cpair[r].y == pr.x) {
      mk = r;
      break;
    }
  cuni[upos[k]] = make_int2((int)k, mk);
}

static inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int build_tree_impl(dfmm_plan* pl, const double* seg, int64_t nseg, hipStream_t st, dfmm_tree* t, bool workspaces) {
  int D = pl->D;
  const int nq = pl->quad.n;
  const int64_t N = nseg * nq;
  if (N >= (int64_t)1 << 31) {
    set_error("build_tree: too many quadrature points (limit 2^31)");
    return DFMM_E_ARG;
  }
  t->plan = pl;
  t->nseg = nseg;
  t->N = N;
  t->D = D;
  t->lv.assign(D + 1, dfmm_tree::Level());
  uint32_t* keys = nullptr;
  int* err = nullptr;
  DFMM_HIP(hipMalloc(&keys, sizeof(uint32_t) * N));
  DFMM_HIP(hipMalloc(&t->perm, sizeof(uint32_t) * N));
  DFMM_HIP(hipMalloc(&t->inv, sizeof(uint32_t) * N));
  DFMM_HIP(hipMalloc(&err, sizeof(int)));
  DFMM_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
  k_make_keys<<<nb(N, 256), 256, 0, st>>>(seg, nseg, pl->quad, pl->prm.box_lo[0], pl->prm.box_lo[1],
                                         pl->prm.box_lo[2], pl->prm.box_size, D, keys, t->perm, err);
  DFMM_LAUNCH_CHECK();
  int herr = 0;
  DFMM_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  DFMM_HIP(hipStreamSynchronize(st));
  hipFree(err);
  if (herr & 1) {
    hipFree(keys);
    set_error("build_tree: non-finite segment coordinate");
    return DFMM_E_NONFINITE;
  }
  if (herr & 2) {
    hipFree(keys);
    set_error("build_tree: a quadrature point lies outside the root cube");
    return DFMM_E_OUT_OF_BOX;
  }
  int rc = radix_sort(keys, t->perm, N, 3 * D, st);
  if (rc) return rc;
  k_inverse_perm<<<nb(N, 256), 256, 0, st>>>(t->perm, N, t->inv);
  DFMM_LAUNCH_CHECK();

  // occupied cells, level D from the points, coarser levels from their children
  int* flags = nullptr;
  int* idx = nullptr;
  DFMM_HIP(hipMalloc(&flags, sizeof(int) * N));
  DFMM_HIP(hipMalloc(&idx, sizeof(int) * N));
  const uint32_t* in_keys = keys;
  int64_t n_in = N;
  for (int l = D; l >= 2; --l) {
    int shift = (l == D) ? 0 : 3;
    k_run_flags<<<nb(n_in, 256), 256, 0, st>>>(in_keys, n_in, shift, flags);
    DFMM_LAUNCH_CHECK();
    int64_t nc;
    rc = scan_excl(flags, idx, n_in, st, &nc);
    if (rc) return rc;
    auto& L = t->lv[l];
    L.n = nc;
    DFMM_HIP(hipMalloc(&L.key, sizeof(uint32_t) * nc));
    DFMM_HIP(hipMalloc(&L.first, sizeof(int) * nc));
    DFMM_HIP(hipMalloc(&L.count, sizeof(int) * nc));
    int* elem_cell = nullptr;
    if (l < D) elem_cell = t->lv[l + 1].parent;
    k_run_emit<<<nb(n_in, 256), 256, 0, st>>>(in_keys, n_in, shift, flags, idx, L.key, L.first, elem_cell);
    DFMM_LAUNCH_CHECK();
    k_run_counts<<<nb(nc, 256), 256, 0, st>>>(L.first, (int)nc, n_in, L.count);
    DFMM_LAUNCH_CHECK();
    if (l > 2) DFMM_HIP(hipMalloc(&L.parent, sizeof(int) * nc));
    in_keys = L.key;
    n_in = nc;
  }
  hipFree(flags);
  hipFree(idx);
  hipFree(keys);
  // adaptive tree: cells below a leaf pruned, leaves on several levels; the
  // tree's depth becomes its deepest level
  if (pl->prm.leaf_max > 0) {
    rc = adapt_prune(pl, t, st);
    if (rc) return rc;
    D = t->D;
  }
  // global cell numbering over levels 2..D
  t->ncell_total = 0;
  t->max_level_cells = 0;
  for (int l = 2; l <= D; ++l) {
    t->lv[l].off = t->ncell_total;
    t->ncell_total += t->lv[l].n;
    t->max_level_cells = std::max<int64_t>(t->max_level_cells, t->lv[l].n);
  }
  // neighbours of the leaves (uniform tree)
  auto& LD = t->lv[D];
  if (!t->adaptive) {
    DFMM_HIP(hipMalloc(&t->nbr, sizeof(int) * 27 * LD.n));
    k_leaf_nbrs<<<nb(LD.n, 128), 128, 0, st>>>(LD.key, (int)LD.n, D, t->nbr);
    DFMM_LAUNCH_CHECK();
  }
  // interaction lists
  t->npairs = 0;
  for (int l = 2; l <= D; ++l) {
    auto& L = t->lv[l];
    int* cnt = nullptr;
    DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (L.n + 1)));
    DFMM_HIP(hipMalloc(&L.il_start, sizeof(int) * (L.n + 1)));
    k_ilist<<<nb(L.n, 128), 128, 0, st>>>(L.key, (int)L.n, l, pl->oid343, nullptr, cnt, nullptr);
    DFMM_LAUNCH_CHECK();
    DFMM_HIP(hipMemsetAsync(cnt + L.n, 0, sizeof(int), st));
    int64_t tot;
    rc = scan_excl(cnt, L.il_start, L.n + 1, st, &tot);
    if (rc) return rc;
    int64_t pairs = tot;
    // The M2L kernels address a level's list and one frequency's slice of the
    // source spectra (9 complex per cell) with 32-bit byte offsets.
    if (pairs * (int64_t)sizeof(int2) >= ((int64_t)1 << 32) || L.n * 9 * 16 >= ((int64_t)1 << 32)) {
      hipFree(cnt);
      set_error("build_tree: a level's interaction list or cell count exceeds the M2L kernels' 32-bit offsets");
      return DFMM_E_ARG;
    }
    L.npairs = pairs;
    t->npairs += pairs;
    DFMM_HIP(hipMalloc(&L.il, sizeof(int2) * std::max<int64_t>(pairs, 1)));
    k_ilist<<<nb(L.n, 128), 128, 0, st>>>(L.key, (int)L.n, l, pl->oid343, L.il_start, nullptr, L.il);
    DFMM_LAUNCH_CHECK();
    // processing order of the M2L targets: similar list lengths share a wave
    uint32_t* okey = (uint32_t*)cnt;
    DFMM_HIP(hipMalloc(&L.order, sizeof(uint32_t) * L.n));
    int* pmax = nullptr;
    if (l > 2) {
      DFMM_HIP(hipMalloc(&pmax, sizeof(int) * t->lv[l - 1].n));
      DFMM_HIP(hipMemsetAsync(pmax, 0, sizeof(int) * t->lv[l - 1].n, st));
      k_sib_len<<<nb(L.n, 256), 256, 0, st>>>(L.il_start, L.parent, (int)L.n, pmax);
      DFMM_LAUNCH_CHECK();
    }
    const int win = m2l_window(pl->mixed);
    k_len_keys<<<nb(L.n, 256), 256, 0, st>>>(L.il_start, pmax ? L.parent : nullptr, pmax, (int)L.n, win, okey,
                                             L.order);
    DFMM_LAUNCH_CHECK();
    int wbits = 0;
    while (((L.n + win - 1) / win) >> wbits) ++wbits;
    rc = radix_sort(okey, L.order, L.n, 8 + wbits, st);
    hipFree(pmax);
    if (rc) return rc;
    {  // the wave-blocked lists of the M2L kernels
      const int64_t nw = (L.n + kWaveTargets - 1) / kWaveTargets;
      int* wlen = nullptr;
      DFMM_HIP(hipMalloc(&wlen, sizeof(int) * (nw + 1)));
      DFMM_HIP(hipMemsetAsync(wlen, 0, sizeof(int) * (nw + 1), st));
      DFMM_HIP(hipMalloc(&L.lenq, sizeof(int) * L.n));
      DFMM_HIP(hipMalloc(&L.wbase, sizeof(int) * (nw + 1)));
      k_wave_len<<<nb(L.n, 256), 256, 0, st>>>(L.order, L.il_start, (int)L.n, L.lenq, wlen);
      DFMM_LAUNCH_CHECK();
      int64_t steps = 0;
      rc = scan_excl(wlen, L.wbase, nw + 1, st, &steps);
      hipFree(wlen);
      if (rc) return rc;
      if (steps * kWaveTargets * (int64_t)sizeof(uint32_t) >= ((int64_t)1 << 32) || L.n >= ((int64_t)1 << 23)) {
        set_error("build_tree: a level's M2L lists exceed the kernel's 32-bit offsets, or the level has 2^23 or more cells");
        return DFMM_E_ARG;
      }
      DFMM_HIP(hipMalloc(&L.ilw, sizeof(uint32_t) * kWaveTargets * std::max<int64_t>(steps, 1)));
      DFMM_HIP(hipMemsetAsync(L.ilw, 0, sizeof(uint32_t) * kWaveTargets * std::max<int64_t>(steps, 1), st));
      if (pl->h16)
        k_il_wave<true><<<nb(L.n, 128), 128, 0, st>>>(L.order, L.il_start, L.il, L.wbase, (int)L.n, L.ilw);
      else
        k_il_wave<false><<<nb(L.n, 128), 128, 0, st>>>(L.order, L.il_start, L.il, L.wbase, (int)L.n, L.ilw);
      DFMM_LAUNCH_CHECK();
      {
        const int64_t ng = nw * (kWaveTargets / 8);
        // 16-byte units per offset and lane 1's start, in the layout of the spectra in LDS
        if (pl->h16)
          k_il_bank<kKOffsetH / 4, kKHalfH / 4, true><<<(unsigned)ng, 64, 0, st>>>(L.lenq, L.wbase, L.n, ng, L.ilw);
        else if (pl->mixed)
          k_il_bank<kKOffsetF / 2, kKHalfF / 2, false><<<(unsigned)ng, 64, 0, st>>>(L.lenq, L.wbase, L.n, ng,
                                                                                   L.ilw);
        else
          k_il_bank<kKOffsetD, kKHalfD, false><<<(unsigned)ng, 64, 0, st>>>(L.lenq, L.wbase, L.n, ng, L.ilw);
        DFMM_LAUNCH_CHECK();
      }
      DFMM_HIP(hipStreamSynchronize(st));
      hipFree(L.il);
      L.il = nullptr;
    }
    hipFree(cnt);
  }
  // near-field pair count (for reporting), and the large-leaf pairs
  std::vector<int> hbig;
  if (t->adaptive) {  // U, W, X lists, the leaf of every point, near pairs
    rc = adapt_lists(pl, t, st);
    if (rc) return rc;
  } else {
    std::vector<int> hn(27 * LD.n), hc(LD.n);
    DFMM_D2H(hn.data(), t->nbr, sizeof(int) * hn.size(), st);
    DFMM_D2H(hc.data(), LD.count, sizeof(int) * hc.size(), st);
    int64_t np = 0;
    int mx = 0;
    for (int64_t i = 0; i < LD.n; ++i) {
      int64_t s = 0;
      for (int k = 0; k < 27; ++k)
        if (hn[27 * i + k] >= 0) s += hc[hn[27 * i + k]];
      np += s * hc[i];
      mx = std::max(mx, hc[i]);
    }
    t->near_pairs = np;
    t->max_leaf_pts = mx;
    // the symmetric near field's launch for large leaves takes only these pairs
    for (int64_t a = 0; !pl->iso && mx > 64 && a < LD.n; ++a)
      for (int q = 13; q < 27; ++q) {
        const int b = hn[27 * a + q];
        if (b >= 0 && (hc[a] > 64 || hc[b] > 64)) hbig.push_back((int)(a * 14 + (q - 13)));
      }
  }
  if (!workspaces) {
    DFMM_HIP(hipStreamSynchronize(st));
    return DFMM_OK;
  }
  // workspaces
  const int p3 = pl->p * pl->p * pl->p;
  const size_t es = pl->mixed ? sizeof(float) : sizeof(double);
  size_t bW = es * 9 * p3 * t->ncell_total, bS = es * 6 * p3 * t->ncell_total;
  // Source and target spectra of one level, whole or in chunks of first
  // frequency indices: the plan's freq_chunks, or (0) as few chunks as keep
  // them within half of the device memory free once the rest is allocated.
  const size_t per_f = ((pl->h16 ? sizeof(uint32_t) : es * 2) * 9 + es * 2 * 6) * (size_t)t->max_level_cells;
  {
    const int n = pl->n;
    int chunks = pl->prm.freq_chunks;
    if (chunks <= 0) {
      size_t fr = 0, total = 0;
      DFMM_HIP(hipMemGetInfo(&fr, &total));
      const size_t rest = es * 15 * p3 * t->ncell_total + sizeof(double) * 15 * N;
      const size_t budget = fr > rest ? (fr - rest) / 2 : 0;
      const size_t whole = per_f * (size_t)pl->nf;
      chunks = 1;
      while (chunks < n && whole / chunks > budget) ++chunks;
    }
    chunks = std::min(chunks, n);
    t->fchunk = (n + chunks - 1) / chunks;
    t->fchunks = (n + t->fchunk - 1) / t->fchunk;
  }
  const size_t nfc = (size_t)t->fchunk * pl->n * pl->p;
  size_t bWh = (pl->h16 ? sizeof(uint32_t) : es * 2) * 9 * nfc * t->max_level_cells;
  size_t bSh = es * 2 * 6 * nfc * t->max_level_cells;
  DFMM_HIP(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
  DFMM_HIP(hipEventCreateWithFlags(&t->fork, hipEventDisableTiming));
  DFMM_HIP(hipEventCreateWithFlags(&t->join, hipEventDisableTiming));
  DFMM_HIP(hipEventCreateWithFlags(&t->done, hipEventDisableTiming));
  DFMM_HIP(hipMalloc(&t->pts, sizeof(double) * 9 * N));
  // the build's positions, for dfmm_tree_check_positions
  DFMM_HIP(hipMalloc(&t->pos0, sizeof(double) * 3 * N));
  DFMM_HIP(hipMalloc(&t->chk, 2 * sizeof(unsigned long long)));
  k_gather_pos<<<nb(N, 256), 256, 0, st>>>(seg, t->perm, pl->quad, N, t->pos0);
  DFMM_LAUNCH_CHECK();
  if (!t->adaptive) {
    DFMM_HIP(hipMalloc(&t->pleaf, sizeof(int) * N));
    k_point_leaf<<<(unsigned)LD.n, 64, 0, st>>>(LD.first, LD.count, (int)LD.n, t->pleaf);
    DFMM_LAUNCH_CHECK();
  }
  DFMM_HIP(hipMalloc(&t->W, bW));
  DFMM_HIP(hipMalloc(&t->s, bS));
  DFMM_HIP(hipMalloc(&t->What, bWh));
  DFMM_HIP(hipMalloc(&t->Shat, bSh));
  DFMM_HIP(hipMalloc(&t->sig, sizeof(double) * 6 * N));
  size_t bKx = 0;
  if (pl->sym) {  // one level of expanded offset spectra (the plan keeps the 16 classes)
    bKx = pl->h16 ? (size_t)pl->nf * kNumOffsets * kKOffsetH * sizeof(uint32_t)
                  : (size_t)pl->nf * kNumCanon * (pl->mixed ? kKOffsetF : kKOffsetD) * 2 * es;
    DFMM_HIP(hipMalloc(&t->kexp, bKx));
  }
  if (pl->h16) DFMM_HIP(hipMalloc(&t->wmax, sizeof(unsigned) * (D + 1)));
  const size_t part_es = pl->mixed ? sizeof(float) : sizeof(double);
  if (!t->adaptive && !pl->iso && t->max_leaf_pts <= kSymMaxLeaf) {
    DFMM_HIP(hipMalloc(&t->part, part_es * 27 * 6 * N));
    if (!hbig.empty()) {
      t->nbig = (int64_t)hbig.size();
      DFMM_HIP(hipMalloc(&t->bigp, sizeof(int) * hbig.size()));
      DFMM_HIP(hipMemcpy(t->bigp, hbig.data(), sizeof(int) * hbig.size(), hipMemcpyHostToDevice));
    }
  }
  if (pl->mixed) {  // the near-coincident pairs, evaluated in double by every call
    const double sD = pl->prm.box_size / (double)(1 << D);
    const double a2x4 = 4.0 * pl->prm.core_a * pl->prm.core_a;
    k_gather_pos<<<nb(N, 256), 256, 0, st>>>(seg, t->perm, pl->quad, N, t->pts);
    DFMM_LAUNCH_CHECK();
    int* cnt = nullptr;
    DFMM_HIP(hipMalloc(&cnt, sizeof(int) * (N + 1)));
    DFMM_HIP(hipMemsetAsync(cnt + N, 0, sizeof(int), st));
    if (t->adaptive) {
      rc = adapt_close_find(pl, t, false, cnt, nullptr, nullptr, st);
      if (rc) return rc;
    } else {
      k_close_find<false><<<nb(N, 128), 128, 0, st>>>(t->pts, N, t->pleaf, LD.first, LD.count, LD.key, t->nbr,
                                                     pl->prm.box_lo[0], pl->prm.box_lo[1], pl->prm.box_lo[2], sD,
                                                     a2x4, cnt, nullptr, nullptr);
      DFMM_LAUNCH_CHECK();
    }
    DFMM_HIP(hipMalloc(&t->cstart, sizeof(int) * (N + 1)));
    rc = scan_excl(cnt, t->cstart, N + 1, st, &t->nclose);
    hipFree(cnt);
    if (rc) return rc;
    if (t->nclose >= ((int64_t)1 << 31)) {
      set_error("build_tree: too many near-coincident pairs (limit 2^31)");
      return DFMM_E_ARG;
    }
    DFMM_HIP(hipMalloc(&t->cpair, sizeof(int2) * std::max<int64_t>(t->nclose, 1)));
    DFMM_HIP(hipMalloc(&t->cval, sizeof(double) * 6 * std::max<int64_t>(t->nclose, 1)));
    if (t->adaptive) {
      rc = adapt_close_find(pl, t, true, nullptr, t->cstart, t->cpair, st);
      if (rc) return rc;
    } else {
      k_close_find<true><<<nb(N, 128), 128, 0, st>>>(t->pts, N, t->pleaf, LD.first, LD.count, LD.key, t->nbr,
                                                    pl->prm.box_lo[0], pl->prm.box_lo[1], pl->prm.box_lo[2], sD,
                                                    a2x4, nullptr, t->cstart, t->cpair);
      DFMM_LAUNCH_CHECK();
    }
    if (t->nclose > 0) {  // the unordered pairs with their two list entries
      int *flag = nullptr, *upos = nullptr;
      DFMM_HIP(hipMalloc(&flag, sizeof(int) * (t->nclose + 1)));
      DFMM_HIP(hipMalloc(&upos, sizeof(int) * (t->nclose + 1)));
      DFMM_HIP(hipMemsetAsync(flag + t->nclose, 0, sizeof(int), st));
      k_close_uni<<<nb(t->nclose, 256), 256, 0, st>>>(t->cpair, t->cstart, t->nclose, nullptr, flag, nullptr);
      DFMM_LAUNCH_CHECK();
      rc = scan_excl(flag, upos, t->nclose + 1, st, &t->nuni);
      if (rc == DFMM_OK && hipMalloc(&t->cuni, sizeof(int2) * std::max<int64_t>(t->nuni, 1)) != hipSuccess)
        rc = DFMM_E_NOMEM;
      if (rc == DFMM_OK) {
        k_close_uni<<<nb(t->nclose, 256), 256, 0, st>>>(t->cpair, t->cstart, t->nclose, upos, nullptr, t->cuni);
        DFMM_LAUNCH_CHECK();
        DFMM_HIP(hipStreamSynchronize(st));
      }
      hipFree(flag);
      hipFree(upos);
      if (rc) {
        set_error("build_tree: cannot allocate the close-pair tables");
        return rc;
      }
      if (2 * t->nuni != t->nclose) {  // the lists are symmetric by construction
        set_error("build_tree: the near-coincident pair lists are not symmetric");
        return DFMM_E_STATE;
      }
      DFMM_HIP(hipMemsetAsync(t->cval, 0, sizeof(double) * 6 * t->nclose, st));
    }
  }
  t->bytes = sizeof(double) * 18 * N + sizeof(int) * N + bW + bS + bWh + bSh +
             (sizeof(int2) + 6 * sizeof(double)) * t->nclose + sizeof(int2) * t->nuni +
             (t->cstart ? sizeof(int) * (N + 1) : 0) +
             (t->part ? part_es * 27 * 6 * N : 0) + sizeof(int) * t->nbig + bKx +
             (t->adaptive ? sizeof(int) * (3 * t->nleaf + 2 * (t->nleaf + 1) + t->nu + 2 * t->nw + t->nwleaf +
                                           t->nxcell + 2 * t->ncell_total + 1) +
                                5 * t->ncell_total
                          : 0);
  DFMM_HIP(hipStreamSynchronize(st));
  return DFMM_OK;
}

}  // namespace dfmm
