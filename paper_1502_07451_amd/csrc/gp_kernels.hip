// gp_kernels.hip - gfx950 kernels of the single-graph path and their launchers.
//
// Per level of the multilevel hierarchy:
//   matching    k_match_propose / k_match_resolve   (R rounds)
//   contraction k_contract_count -> k_contract_map -> k_contract_rows
//               -> k_contract_long -> k_contract_compact
// at the coarsest level
//   initial bisection k_init_tot -> k_init_trials (one trial per block)
// per level on the way back up
//   k_project, then P x (k_refine_gain -> k_refine_apply)
// and once at level 0 k_final_stats.  Graph checks of gp_create live at the
// end of the file.
#include "gp_dev.h"
#include "gp_launch.h"

namespace gpk {

// ------------------------------------------------------------------ helpers
// clears the per-level coarsening counters; on levels below the input graph
// the largest balance weight measured by the previous contraction becomes
// the current one
__global__ void k_level_reset(Ctrl* ctrl, int promote) {
  for (int i = threadIdx.x; i < kMaxRounds; i += blockDim.x) ctrl->made[i] = 0;
  if (threadIdx.x == 0) {
    if (promote) ctrl->maxb = ctrl->maxb_next;
    ctrl->nc = 0;
    ctrl->nnz_c = 0;
    ctrl->nlong = 0;
    ctrl->ubtot = 0;
    ctrl->maxb_next = 0;
  }
}

static int grid_for(int64_t items, int per_block, int cap = 4096) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ----------------------------------------------------------------- matching
// Edge order for matching: heavier first, then larger hash of the endpoint
// pair, then smaller endpoints.  For a fixed u, comparing (lo, hi) reduces
// to comparing the neighbour id v.
struct MatchBest {
  int64_t w;   // -1: none
  int32_t v;
};

__device__ __forceinline__ uint64_t pair_hash(uint64_t hs, int32_t u, int32_t v) {
  uint32_t lo = (uint32_t)(u < v ? u : v), hi = (uint32_t)(u < v ? v : u);
  return mix64(hs ^ (((uint64_t)lo << 32) | (uint64_t)hi));
}

// true when candidate (w, v) beats best (bw, bv) for vertex u
__device__ __forceinline__ bool match_better(int64_t w, int32_t v, int64_t bw, int32_t bv,
                                             uint64_t hs, int32_t u) {
  if (bv < 0) return v >= 0;
  if (v < 0) return false;
  if (w != bw) return w > bw;
  uint64_t h = pair_hash(hs, u, v), bh = pair_hash(hs, u, bv);
  if (h != bh) return h > bh;
  return v < bv;
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_match_propose(LevelView lv, const int32_t* match,
                                                          int32_t* prop, const Ctrl* ctrl,
                                                          int round, uint64_t hs) {
  if (round > 0 && ctrl->made[round - 1] == 0) return;
  const int64_t cap = ctrl->cap, maxb = ctrl->maxb;
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  for (int64_t uu = team; uu < lv.n; uu += nteams) {
    const int32_t u = (int32_t)uu;
    if (round > 0 && match[u] != -1) continue;
    const int64_t bu = lv.b[u];
    const bool capcheck = bu + maxb > cap;
    int64_t bw = -1;
    int32_t bv = -1;
    const int32_t e1 = lv.xadj[u + 1];
    for (int32_t e = lv.xadj[u] + lane; e < e1; e += TW) {
      const int32_t v = lv.adj[e];
      if (round > 0 && match[v] != -1) continue;
      if (capcheck && bu + lv.b[v] > cap) continue;
      const int64_t w = lv.w[e];
      if (match_better(w, v, bw, bv, hs, u)) {
        bw = w;
        bv = v;
      }
    }
#pragma unroll
    for (int o = TW / 2; o > 0; o >>= 1) {
      int64_t ow = __shfl_xor(bw, o, TW);
      int32_t ov = __shfl_xor(bv, o, TW);
      if (match_better(ow, ov, bw, bv, hs, u)) {
        bw = ow;
        bv = ov;
      }
    }
    if (lane == 0) prop[u] = bv;
  }
}

__global__ __launch_bounds__(kBlock) void k_match_resolve(int32_t n, int32_t* match,
                                                          const int32_t* prop, Ctrl* ctrl,
                                                          int round) {
  if (round > 0 && ctrl->made[round - 1] == 0) return;
  __shared__ int32_t sm[kBlock / 64];
  int32_t made = 0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * kBlock) {
    if (round == 0) {
      const int32_t p = prop[u];
      const int32_t m = (p >= 0 && prop[p] == (int32_t)u) ? p : -1;
      match[u] = m;
      made += m >= 0;
    } else if (match[u] == -1) {
      const int32_t p = prop[u];
      if (p >= 0 && prop[p] == (int32_t)u) {
        match[u] = p;
        made++;
      }
    }
  }
  made = block_sum<kBlock, int32_t>(made, sm);
  if (threadIdx.x == 0 && made) atomicAdd(&ctrl->made[round], made);
}

// --------------------------------------------------------------- two-hop pass
// hub[u] = first neighbour of an unmatched u under the edge order (-1: none);
// matched vertices get -2
template <int TW>
__global__ __launch_bounds__(kBlock) void k_hub(LevelView lv, const int32_t* match, int32_t* hub,
                                                uint64_t hs) {
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  for (int64_t uu = team; uu < lv.n; uu += nteams) {
    const int32_t u = (int32_t)uu;
    if (match[u] != -1) {
      if (lane == 0) hub[u] = -2;
      continue;
    }
    int64_t bw = -1;
    int32_t bv = -1;
    const int32_t e1 = lv.xadj[u + 1];
    for (int32_t e = lv.xadj[u] + lane; e < e1; e += TW) {
      const int32_t v = lv.adj[e];
      const int64_t w = lv.w[e];
      if (match_better(w, v, bw, bv, hs, u)) {
        bw = w;
        bv = v;
      }
    }
#pragma unroll
    for (int o = TW / 2; o > 0; o >>= 1) {
      int64_t ow = __shfl_xor(bw, o, TW);
      int32_t ov = __shfl_xor(bv, o, TW);
      if (match_better(ow, ov, bw, bv, hs, u)) {
        bw = ow;
        bv = ov;
      }
    }
    if (lane == 0) hub[u] = bv;
  }
}

// The members of h's group are the x in row h with hub[x] == h; the sorted
// row lists them in ascending id.  They are paired first-second,
// third-fourth, ... when the pair fits under the cap.  Each unmatched vertex
// has one hub, so every match[] entry is written by one team only.
template <int TW>
__global__ __launch_bounds__(kBlock) void k_twohop(LevelView lv, const int32_t* hub,
                                                   int32_t* match, const Ctrl* ctrl) {
  const int64_t cap = ctrl->cap;
  const int lane = threadIdx.x & (TW - 1);
  const int tb = lane_id() & ~(TW - 1);
  const uint64_t tmask = TW == 64 ? ~0ull : ((1ull << TW) - 1ull);
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  for (int64_t hh = team; hh < lv.n; hh += nteams) {
    const int32_t h = (int32_t)hh;
    const int32_t e1 = lv.xadj[h + 1];
    int32_t pending = -1;
    for (int32_t e0 = lv.xadj[h]; e0 < e1; e0 += TW) {
      const int32_t e = e0 + lane;
      const int32_t x = e < e1 ? lv.adj[e] : -1;
      const bool mem = x >= 0 && hub[x] == h;
      const uint64_t mask = (__ballot(mem) >> tb) & tmask;
      const int k = __popcll(mask & below);
      const int cnt = __popcll(mask);
      const int off = pending >= 0 ? 1 : 0;
      const uint64_t lower = mask & below;
      const int prev_lane = lower ? 63 - __clzll(lower) : lane;
      const int32_t prev_x = __shfl(x, prev_lane, TW);
      const int last_lane = mask ? 63 - __clzll(mask) : 0;
      const int32_t last_x = __shfl(x, last_lane, TW);
      if (mem && ((k + off) & 1)) {
        const int32_t y = k == 0 ? pending : prev_x;
        if (lv.b[x] + lv.b[y] <= cap) {
          match[x] = y;
          match[y] = x;
        }
      }
      if ((off + cnt) & 1) pending = cnt > 0 ? last_x : pending;
      else pending = -1;
    }
  }
}

// unmatched vertices without neighbours, paired in ascending id
__global__ __launch_bounds__(kBlock) void k_iso_count(LevelView lv, const int32_t* match,
                                                      Ctrl* ctrl, int32_t* tile_cnt,
                                                      int ntiles) {
  __shared__ int32_t smi[kBlock / 64];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int32_t c = 0;
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      if (u < lv.n && match[u] == -1 && lv.xadj[u + 1] == lv.xadj[u]) c++;
    }
    c = block_sum<kBlock, int32_t>(c, smi);
    if (threadIdx.x == 0) tile_cnt[t] = c;
  }
  if (!last_block(&ctrl->ctr_iso, gridDim.x)) return;
  int32_t carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += kBlock) {
    const int t = t0 + threadIdx.x;
    const int32_t x = t < ntiles ? tile_cnt[t] : 0;
    int32_t tot;
    const int32_t ex = block_exscan<kBlock, int32_t>(x, smi, &tot);
    if (t < ntiles) tile_cnt[t] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) ctrl->niso = carry;
}

__global__ __launch_bounds__(kBlock) void k_iso_list(LevelView lv, const int32_t* match,
                                                     const int32_t* tile_base, int32_t* iso,
                                                     int ntiles) {
  __shared__ int32_t smi[kBlock / 64];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    bool f[4];
    int32_t c = 0;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      f[j] = u < lv.n && match[u] == -1 && lv.xadj[u + 1] == lv.xadj[u];
      c += f[j];
    }
    int32_t tot;
    int32_t r = tile_base[t] + block_exscan<kBlock, int32_t>(c, smi, &tot);
    for (int j = 0; j < 4; j++)
      if (f[j]) iso[r++] = (int32_t)(base + j);
  }
}

__global__ __launch_bounds__(kBlock) void k_iso_pair(const int64_t* b, const int32_t* iso,
                                                     int32_t* match, const Ctrl* ctrl) {
  const int32_t npairs = ctrl->niso / 2;
  const int64_t cap = ctrl->cap;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npairs;
       i += (int64_t)gridDim.x * kBlock) {
    const int32_t x = iso[2 * i], y = iso[2 * i + 1];
    if (b[x] + b[y] <= cap) {
      match[x] = y;
      match[y] = x;
    }
  }
}

// --------------------------------------------------------------- contraction
// tile t covers fine vertices [t*kTileV, (t+1)*kTileV); each thread 4 of them
__global__ __launch_bounds__(kBlock) void k_contract_count(LevelView lv, const int32_t* match,
                                                           Ctrl* ctrl, int32_t* tile_lead,
                                                           int64_t* tile_ub, int ntiles) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ int32_t smi[kBlock / 64];
  int64_t mx = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int32_t lead = 0;
    int64_t ub = 0;
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      if (u >= lv.n) break;
      const int32_t m = match[u];
      if (m < 0 || u < m) {
        lead++;
        ub += lv.xadj[u + 1] - lv.xadj[u];
        int64_t bsum = lv.b[u];
        if (m >= 0) {
          ub += lv.xadj[m + 1] - lv.xadj[m];
          bsum += lv.b[m];
        }
        mx = bsum > mx ? bsum : mx;
      }
    }
    lead = block_sum<kBlock, int32_t>(lead, smi);
    ub = block_sum<kBlock, int64_t>(ub, sml);
    if (threadIdx.x == 0) {
      tile_lead[t] = lead;
      tile_ub[t] = ub;
    }
  }
  mx = block_max<kBlock, int64_t>(mx, sml);
  if (threadIdx.x == 0) atomicMax((long long*)&ctrl->maxb_next, (long long)mx);
  if (!last_block(&ctrl->ctr_count, gridDim.x)) return;
  // exclusive scan of the tile totals
  int32_t carry_l = 0;
  int64_t carry_u = 0;
  for (int t0 = 0; t0 < ntiles; t0 += kBlock) {
    const int t = t0 + threadIdx.x;
    int32_t l = t < ntiles ? tile_lead[t] : 0;
    int64_t u = t < ntiles ? tile_ub[t] : 0;
    int32_t tl;
    int64_t tu;
    int32_t el = block_exscan<kBlock, int32_t>(l, smi, &tl);
    int64_t eu = block_exscan<kBlock, int64_t>(u, sml, &tu);
    if (t < ntiles) {
      tile_lead[t] = carry_l + el;
      tile_ub[t] = carry_u + eu;
    }
    carry_l += tl;
    carry_u += tu;
  }
  if (threadIdx.x == 0) {
    ctrl->nc = carry_l;
    ctrl->ubtot = carry_u;
  }
}

__global__ __launch_bounds__(kBlock) void k_contract_map(LevelView lv, const int32_t* match,
                                                         const int64_t* vc, const int64_t* vg,
                                                         const int32_t* tile_lead,
                                                         const int64_t* tile_ub, int32_t* cmap,
                                                         int64_t* cvc, int64_t* cvg,
                                                         int32_t* cmem0, int32_t* cmem1,
                                                         int64_t* toff, int ntiles) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ int32_t smi[kBlock / 64];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    int32_t lead = 0;
    int64_t ub = 0;
    int32_t mm[4];
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      mm[j] = -2;
      if (u >= lv.n) continue;
      const int32_t m = match[u];
      mm[j] = m;
      if (m < 0 || u < m) {
        lead++;
        ub += lv.xadj[u + 1] - lv.xadj[u];
        if (m >= 0) ub += lv.xadj[m + 1] - lv.xadj[m];
      }
    }
    int32_t tl;
    int64_t tu;
    int32_t c = tile_lead[t] + block_exscan<kBlock, int32_t>(lead, smi, &tl);
    int64_t off = tile_ub[t] + block_exscan<kBlock, int64_t>(ub, sml, &tu);
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      const int32_t m = mm[j];
      if (m == -2 || !(m < 0 || u < m)) continue;
      cmap[u] = c;
      int64_t sc = vc[u], sg = vg[u];
      int64_t d = lv.xadj[u + 1] - lv.xadj[u];
      if (m >= 0) {
        cmap[m] = c;
        sc += vc[m];
        sg += vg[m];
        d += lv.xadj[m + 1] - lv.xadj[m];
      }
      cvc[c] = sc;
      cvg[c] = sg;
      cmem0[c] = (int32_t)u;
      cmem1[c] = m;
      toff[c] = off;
      c++;
      off += d;
    }
  }
}

// candidate i of coarse row c: entries of the first member, then the second
struct CoarseRowLoader {
  const int32_t* xadj;
  const int32_t* adj;
  const int64_t* w;
  const int32_t* cmap;
  int32_t c, e0, d0, e1;
  __device__ __forceinline__ void operator()(int i, int32_t& k, int64_t& v) const {
    const int32_t e = i < d0 ? e0 + i : e1 + (i - d0);
    const int32_t x = cmap[adj[e]];
    k = x == c ? INT_MAX : x;
    v = w[e];
  }
};

__device__ __forceinline__ CoarseRowLoader coarse_loader(const LevelView& lv, const int32_t* cmap,
                                                         const int32_t* cmem0,
                                                         const int32_t* cmem1, int32_t c,
                                                         int* L) {
  CoarseRowLoader ld;
  ld.xadj = lv.xadj;
  ld.adj = lv.adj;
  ld.w = lv.w;
  ld.cmap = cmap;
  ld.c = c;
  const int32_t m0 = cmem0[c], m1 = cmem1[c];
  ld.e0 = lv.xadj[m0];
  ld.d0 = lv.xadj[m0 + 1] - ld.e0;
  ld.e1 = m1 >= 0 ? lv.xadj[m1] : 0;
  const int d1 = m1 >= 0 ? lv.xadj[m1 + 1] - ld.e1 : 0;
  *L = ld.d0 + d1;
  return ld;
}

template <int T>
__device__ __forceinline__ void team_row(const CoarseRowLoader& ld, int L, int32_t* okey,
                                         int64_t* oval, int32_t* cnt_out) {
  const int lane = threadIdx.x & (T - 1);
  int32_t k = INT_MAX;
  int64_t v = 0;
  if (lane < L) ld(lane, k, v);
  team_bitonic<T>(k, v);
  bool dummy = false;
  int cnt = team_emit<T, true>(k, v, okey, oval, &dummy);
  if (lane == 0) *cnt_out = cnt;
}

__global__ __launch_bounds__(kBlock) void k_contract_rows(
    LevelView lv, const int32_t* cmap, const int32_t* cmem0, const int32_t* cmem1,
    const int64_t* toff, const Ctrl* ctrl, int32_t* tmpk, int64_t* tmpv, int32_t* cnt,
    int64_t* tile_cnt, int32_t* longlist, Ctrl* wctrl, int ntiles_c) {
  __shared__ int32_t sk[kSortCap];
  __shared__ int64_t sv[kSortCap];
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  const int32_t nc = ctrl->nc;
  for (int t = blockIdx.x; t < ntiles_c; t += gridDim.x) {
    const int32_t c0 = t * kTileC;
    const int32_t c1 = c0 + kTileC < nc ? c0 + kTileC : nc;
    // rows of at most 16 candidates: 16-lane teams
    for (int32_t c = c0 + (int32_t)threadIdx.x / 16; c < c1; c += kBlock / 16) {
      int L;
      CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
      if (L <= 16) team_row<16>(ld, L, tmpk + toff[c], tmpv + toff[c], &cnt[c]);
    }
    // rows of 17..64 candidates: one wave each
    for (int32_t c = c0 + (int32_t)threadIdx.x / 64; c < c1; c += kBlock / 64) {
      int L;
      CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
      if (L > 16 && L <= 64) team_row<64>(ld, L, tmpk + toff[c], tmpv + toff[c], &cnt[c]);
    }
    // longer rows: the whole block in LDS, or deferred to the dense merge
    for (int32_t c = c0; c < c1; c++) {
      int L;
      CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
      if (L <= 64) continue;
      if (L <= kSortCap) {
        bool dummy = false;
        int k = block_sort_emit<kBlock, true>(L, ld, sk, sv, tmpk + toff[c], tmpv + toff[c],
                                              &dummy, smi);
        if (threadIdx.x == 0) cnt[c] = k;
      } else if (threadIdx.x == 0) {
        int slot = atomicAdd(&wctrl->nlong, 1);
        longlist[slot] = c;
        cnt[c] = 0;
      }
    }
    __syncthreads();
    int64_t s = 0;
    for (int32_t c = c0 + threadIdx.x; c < c1; c += kBlock) s += cnt[c];
    s = block_sum<kBlock, int64_t>(s, sml);
    if (threadIdx.x == 0) tile_cnt[t] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_contract_long(LevelView lv, const int32_t* cmap,
                                                          const int32_t* cmem0,
                                                          const int32_t* cmem1,
                                                          const int64_t* toff, Ctrl* ctrl,
                                                          int32_t* tmpk, int64_t* tmpv,
                                                          int32_t* cnt, int64_t* tile_cnt,
                                                          const int32_t* longlist,
                                                          int ntiles_c) {
  extern __shared__ unsigned char dyn[];
  int64_t* acc = (int64_t*)dyn;
  int32_t* cc = (int32_t*)(acc + kWin);
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  const int32_t nlong = ctrl->nlong;
  for (int32_t i = blockIdx.x; i < nlong; i += gridDim.x) {
    const int32_t c = longlist[i];
    int L;
    CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
    bool dummy = false;
    int k = block_dense_emit<kBlock, true>(L, ld, acc, cc, smi, sml, tmpk + toff[c],
                                           tmpv + toff[c], &dummy);
    if (threadIdx.x == 0) {
      cnt[c] = k;
      atomicAdd((unsigned long long*)&tile_cnt[c / kTileC], (unsigned long long)k);
    }
  }
  if (!last_block(&ctrl->ctr_long, gridDim.x)) return;
  int64_t carry = 0;
  for (int t0 = 0; t0 < ntiles_c; t0 += kBlock) {
    const int t = t0 + threadIdx.x;
    int64_t x = t < ntiles_c ? tile_cnt[t] : 0;
    int64_t tot;
    int64_t e = block_exscan<kBlock, int64_t>(x, sml, &tot);
    if (t < ntiles_c) tile_cnt[t] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) ctrl->nnz_c = (int32_t)carry;
}

__global__ __launch_bounds__(kBlock) void k_contract_compact(const Ctrl* ctrl,
                                                             const int64_t* toff,
                                                             const int32_t* cnt,
                                                             const int64_t* tile_base,
                                                             const int32_t* tmpk,
                                                             const int64_t* tmpv, int32_t* cxadj,
                                                             int32_t* cadj, int64_t* cw,
                                                             int ntiles_c) {
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int32_t srow[kTileC + 1];
  const int32_t nc = ctrl->nc;
  for (int t = blockIdx.x; t < ntiles_c; t += gridDim.x) {
    const int32_t c0 = t * kTileC;
    const int32_t c = c0 + threadIdx.x;
    const int32_t k = (c < nc && threadIdx.x < kTileC) ? cnt[c] : 0;
    int32_t tot;
    const int32_t ex = block_exscan<kBlock, int32_t>(k, smi, &tot);
    const int64_t base = tile_base[t];
    if (c < nc && threadIdx.x < kTileC) {
      cxadj[c] = (int32_t)(base + ex);
      srow[threadIdx.x] = ex;
    }
    if (c == nc - 1) cxadj[nc] = (int32_t)(base + ex + k);
    __syncthreads();
    const int32_t rows = (c0 + kTileC < nc ? kTileC : nc - c0);
    // copy: 16-lane teams over rows
    for (int r = threadIdx.x / 16; r < rows; r += kBlock / 16) {
      const int32_t cr = c0 + r;
      const int32_t kr = cnt[cr];
      const int64_t src = toff[cr];
      const int64_t dst = base + srow[r];
      for (int j = threadIdx.x & 15; j < kr; j += 16) {
        cadj[dst + j] = tmpk[src + j];
        cw[dst + j] = tmpv[src + j];
      }
    }
    __syncthreads();
  }
  if (nc == 0 && blockIdx.x == 0 && threadIdx.x == 0) cxadj[0] = 0;
}

// ------------------------------------------------------------------ refinement
__device__ __forceinline__ void plan_pass(const RefCtl& r, int* mode, int* s) {
  if (r.pw[0] > r.maxw[0]) {
    *mode = 1;
    *s = 0;
  } else if (r.pw[1] > r.maxw[1]) {
    *mode = 1;
    *s = 1;
  } else {
    *mode = 0;
    *s = r.pass & 1;
  }
}

__device__ __forceinline__ void clear_pass_acc(RefCtl* rc) {
  rc->ext_sum = 0;
  rc->cand_b = 0;
  rc->gmin_acc = INT64_MAX;
  rc->gmax_acc = INT64_MIN;
  rc->ncand = 0;
  rc->moved_b = 0;
  rc->moved_n = 0;
}

// Called by every thread of one block once the pass totals are known.
template <int BS>
__device__ void decide_admission(RefCtl* rc, const Cand* list, uint32_t ncand, int64_t cand_b,
                                 int64_t gmin, int64_t gmax, int32_t n, SelShared* sh) {
  const int mode = rc->mode, s = rc->s, d = 1 - s;
  const int64_t budget = rc->maxw[d] - rc->pw[d];
  int admit;
  u128 thr = 0;
  int idbits = bitlen64((uint64_t)(n > 0 ? n - 1 : 0));
  if (ncand == 0) {
    admit = kAdmitNone;
  } else if (mode == 0 && cand_b <= budget) {
    admit = kAdmitAll;
  } else {
    const int tbits = bitlen64((uint64_t)(gmax - gmin)) + idbits;
    if (mode == 0) {
      thr = select_prefix<BS>(list, ncand, gmin, idbits, tbits, 0, budget, sh);
    } else {
      const int64_t excess = rc->pw[s] - rc->maxw[s];
      u128 t1 = select_prefix<BS>(list, ncand, gmin, idbits, tbits, 1, excess, sh);
      u128 t2 = 0;
      if (cand_b > budget) t2 = select_prefix<BS>(list, ncand, gmin, idbits, tbits, 0, budget, sh);
      thr = t1 > t2 ? t1 : t2;
    }
    admit = kAdmitThr;
  }
  if (threadIdx.x == 0) {
    rc->admit = admit;
    rc->idbits = idbits;
    rc->gmin = gmin;
    rc->thr_hi = (uint64_t)(thr >> 64);
    rc->thr_lo = (uint64_t)thr;
  }
}

__device__ __forceinline__ bool admitted(const RefCtl& r, const Cand& c) {
  if (r.admit == kAdmitAll) return true;
  if (r.admit == kAdmitNone) return false;
  const u128 thr = ((u128)r.thr_hi << 64) | (u128)r.thr_lo;
  return cand_key(c, r.gmin, r.idbits) >= thr;
}

__device__ __forceinline__ void finish_pass(RefCtl* rc, int64_t moved_b, int64_t moved_n) {
  const int s = rc->s, d = 1 - s;
  rc->pw[s] -= moved_b;
  rc->pw[d] += moved_b;
  rc->total_moves += moved_n;
  rc->last_cut = rc->ext_sum / 2;
  if (rc->mode == 1) rc->z = 0;
  else rc->z = moved_n == 0 ? rc->z + 1 : 0;
  rc->pass++;
  rc->done = (rc->z >= 2 || rc->pass >= rc->npass) ? 1 : 0;
  clear_pass_acc(rc);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_refine_gain(LevelView lv, const int8_t* part,
                                                        RefCtl* rc, Cand* list) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ SelShared sel;
  if (rc->done) return;
  int mode, s;
  plan_pass(*rc, &mode, &s);
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  int64_t ext_acc = 0, cb = 0, gmn = INT64_MAX, gmx = INT64_MIN;
  // every team runs the same number of iterations so that the wave-wide
  // candidate ballot sees all of its lanes
  const int64_t iters = (lv.n + nteams - 1) / nteams;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t uu = team + it * nteams;
    bool cand = false;
    Cand c;
    c.pad = 0;
    if (uu < lv.n) {
      const int32_t v = (int32_t)uu;
      const int8_t pv = part[v];
      int64_t ext = 0, in = 0;
      const int32_t e1 = lv.xadj[v + 1];
      for (int32_t e = lv.xadj[v] + lane; e < e1; e += TW) {
        const int64_t w = lv.w[e];
        if (part[lv.adj[e]] != pv) ext += w;
        else in += w;
      }
      ext = team_sum<TW>(ext);
      in = team_sum<TW>(in);
      if (lane == 0) {
        const int64_t gain = ext - in;
        ext_acc += ext;
        cand = pv == s && (mode == 1 || gain > 0);
        if (cand) {
          c.gain = gain;
          c.b = lv.b[v];
          c.v = v;
          cb += c.b;
          gmn = gain < gmn ? gain : gmn;
          gmx = gain > gmx ? gain : gmx;
        }
      }
    }
    append_cand(cand, c, list, &rc->ncand);
  }
  ext_acc = block_sum<kBlock, int64_t>(ext_acc, sml);
  cb = block_sum<kBlock, int64_t>(cb, sml);
  gmn = block_min<kBlock, int64_t>(gmn, sml);
  gmx = block_max<kBlock, int64_t>(gmx, sml);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&rc->ext_sum, (unsigned long long)ext_acc);
    atomicAdd((unsigned long long*)&rc->cand_b, (unsigned long long)cb);
    atomicMin((long long*)&rc->gmin_acc, (long long)gmn);
    atomicMax((long long*)&rc->gmax_acc, (long long)gmx);
  }
  if (!last_block(&rc->ctr_gain, gridDim.x)) return;
  if (threadIdx.x == 0) {
    rc->mode = mode;
    rc->s = s;
  }
  __syncthreads();
  decide_admission<kBlock>(rc, list, rc->ncand, rc->cand_b, rc->gmin_acc, rc->gmax_acc, lv.n,
                           &sel);
}

__global__ __launch_bounds__(kBlock) void k_refine_apply(int8_t* part, RefCtl* rc,
                                                         const Cand* list) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  const RefCtl r = *rc;
  const int d = 1 - r.s;
  int64_t mb = 0, mn = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < r.ncand;
       i += (int64_t)gridDim.x * kBlock) {
    const Cand c = list[i];
    if (admitted(r, c)) {
      part[c.v] = (int8_t)d;
      mb += c.b;
      mn++;
    }
  }
  mb = block_sum<kBlock, int64_t>(mb, sml);
  mn = block_sum<kBlock, int64_t>(mn, sml);
  if (threadIdx.x == 0 && (mb || mn)) {
    atomicAdd((unsigned long long*)&rc->moved_b, (unsigned long long)mb);
    atomicAdd((unsigned long long*)&rc->moved_n, (unsigned long long)mn);
  }
  if (!last_block(&rc->ctr_apply, gridDim.x)) return;
  if (threadIdx.x == 0) finish_pass(rc, rc->moved_b, rc->moved_n);
}

__device__ __forceinline__ void start_level(RefCtl* rc, int npass) {
  rc->pass = 0;
  rc->z = 0;
  rc->npass = npass;
  rc->done = npass <= 0 ? 1 : 0;
  rc->total_moves = 0;
  clear_pass_acc(rc);
}

__global__ __launch_bounds__(kBlock) void k_project(int32_t n, const int32_t* cmap,
                                                    const int8_t* cpart, int8_t* part, RefCtl* rc,
                                                    int npass) {
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * kBlock)
    part[u] = cpart[cmap[u]];
  if (blockIdx.x == 0 && threadIdx.x == 0) start_level(rc, npass);
}

__global__ void k_start_level(RefCtl* rc, int npass) {
  if (threadIdx.x == 0) start_level(rc, npass);
}

// cut (as sum of ext), loads and times of the final assignment
template <int TW>
__global__ __launch_bounds__(kBlock) void k_final_stats(LevelView lv, const int64_t* vc,
                                                        const int64_t* vg, const int8_t* part,
                                                        Ctrl* ctrl) {
  __shared__ int64_t sml[kBlock / 64];
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  int64_t ext_acc = 0, l0 = 0, l1 = 0, t0 = 0, t1 = 0;
  for (int64_t uu = team; uu < lv.n; uu += nteams) {
    const int32_t v = (int32_t)uu;
    const int8_t pv = part[v];
    int64_t ext = 0;
    for (int32_t e = lv.xadj[v] + lane; e < lv.xadj[v + 1]; e += TW)
      if (part[lv.adj[e]] != pv) ext += lv.w[e];
    ext = team_sum<TW>(ext);
    if (lane == 0) {
      ext_acc += ext;
      if (pv == 0) {
        l0 += lv.b[v];
        t0 += vc[v];
      } else {
        l1 += lv.b[v];
        t1 += vg[v];
      }
    }
  }
  ext_acc = block_sum<kBlock, int64_t>(ext_acc, sml);
  l0 = block_sum<kBlock, int64_t>(l0, sml);
  l1 = block_sum<kBlock, int64_t>(l1, sml);
  t0 = block_sum<kBlock, int64_t>(t0, sml);
  t1 = block_sum<kBlock, int64_t>(t1, sml);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctrl->res_ext, (unsigned long long)ext_acc);
    atomicAdd((unsigned long long*)&ctrl->res_load[0], (unsigned long long)l0);
    atomicAdd((unsigned long long*)&ctrl->res_load[1], (unsigned long long)l1);
    atomicAdd((unsigned long long*)&ctrl->res_time[0], (unsigned long long)t0);
    atomicAdd((unsigned long long*)&ctrl->res_time[1], (unsigned long long)t1);
  }
}

__global__ void k_clear_stats(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->res_ext = 0;
    ctrl->res_load[0] = ctrl->res_load[1] = 0;
    ctrl->res_time[0] = ctrl->res_time[1] = 0;
  }
}

// ------------------------------------------------------- initial bisection
__global__ __launch_bounds__(kBlock) void k_init_tot(LevelView lv, int64_t* tot) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < lv.n;
       v += (int64_t)gridDim.x * kBlock) {
    int64_t s = 0;
    for (int32_t e = lv.xadj[v]; e < lv.xadj[v + 1]; e++) s += lv.w[e];
    tot[v] = s;
  }
}

// growing key: (has a neighbour in g, gain towards g, smaller id)
struct GrowBest {
  int32_t a;
  int64_t g;
  int32_t v;  // -1: none
};

__device__ __forceinline__ bool grow_better(const GrowBest& x, const GrowBest& y) {
  if (y.v < 0) return x.v >= 0;
  if (x.v < 0) return false;
  if (x.a != y.a) return x.a > y.a;
  if (x.g != y.g) return x.g > y.g;
  return x.v < y.v;
}

template <int BS>
__device__ GrowBest block_grow_argmax(GrowBest b, GrowBest* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    GrowBest o2;
    o2.a = __shfl_xor(b.a, o, 64);
    o2.g = __shfl_xor(b.g, o, 64);
    o2.v = __shfl_xor(b.v, o, 64);
    if (grow_better(o2, b)) b = o2;
  }
  if (BS == 64) return b;
  if (lane_id() == 0) sm[threadIdx.x / 64] = b;
  __syncthreads();
  GrowBest r = sm[0];
  for (int i = 1; i < BS / 64; i++)
    if (grow_better(sm[i], r)) r = sm[i];
  __syncthreads();
  return r;
}

// Whole-graph refinement inside one block (coarsest level, per trial).
template <int BS>
__device__ void refine_block(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                             SelShared* sel, int64_t* sml, uint32_t* s_ncand) {
  for (;;) {
    __syncthreads();
    if (rc->done) break;
    int mode, s;
    plan_pass(*rc, &mode, &s);
    if (threadIdx.x == 0) *s_ncand = 0;
    __syncthreads();
    int64_t ext_acc = 0, cb = 0, gmn = INT64_MAX, gmx = INT64_MIN;
    const int iters = (lv.n + BS - 1) / BS;
    for (int it = 0; it < iters; it++) {
      const int32_t v = it * BS + threadIdx.x;
      bool cand = false;
      Cand c;
      c.pad = 0;
      if (v < lv.n) {
        const int8_t pv = part[v];
        int64_t ext = 0, in = 0;
        for (int32_t e = lv.xadj[v]; e < lv.xadj[v + 1]; e++) {
          if (part[lv.adj[e]] != pv) ext += lv.w[e];
          else in += lv.w[e];
        }
        const int64_t gain = ext - in;
        ext_acc += ext;
        cand = pv == s && (mode == 1 || gain > 0);
        if (cand) {
          c.gain = gain;
          c.b = lv.b[v];
          c.v = v;
          cb += c.b;
          gmn = gain < gmn ? gain : gmn;
          gmx = gain > gmx ? gain : gmx;
        }
      }
      append_cand(cand, c, list, s_ncand);
    }
    ext_acc = block_sum<BS, int64_t>(ext_acc, sml);
    cb = block_sum<BS, int64_t>(cb, sml);
    gmn = block_min<BS, int64_t>(gmn, sml);
    gmx = block_max<BS, int64_t>(gmx, sml);
    __threadfence_block();
    __syncthreads();
    const uint32_t ncand = *s_ncand;
    if (threadIdx.x == 0) {
      rc->mode = mode;
      rc->s = s;
      rc->ext_sum = ext_acc;
    }
    __syncthreads();
    decide_admission<BS>(rc, list, ncand, cb, gmn, gmx, lv.n, sel);
    __syncthreads();
    const RefCtl r = *rc;
    int64_t mb = 0, mn = 0;
    for (uint32_t i = threadIdx.x; i < ncand; i += BS) {
      const Cand c = list[i];
      if (admitted(r, c)) {
        part[c.v] = (int8_t)(1 - s);
        mb += c.b;
        mn++;
      }
    }
    mb = block_sum<BS, int64_t>(mb, sml);
    mn = block_sum<BS, int64_t>(mn, sml);
    if (threadIdx.x == 0) finish_pass(rc, mb, mn);
  }
}

// One block per trial: greedy growing, then refinement, then its cut.  The
// last block to finish keeps the first trial minimal in (infeasible, cut).
template <int BS>
__global__ __launch_bounds__(BS) void k_init_trials(LevelView lv, const int64_t* tot, int K,
                                                    int gs, int npass, Ctrl* ctrl, RefCtl* tctl,
                                                    int8_t* tpart, int64_t* tconn,
                                                    int32_t* tadj, Cand* tlist, int64_t* tres,
                                                    int8_t* out_part) {
  __shared__ int64_t sml[BS / 64];
  __shared__ GrowBest sgb[BS / 64];
  __shared__ SelShared sel;
  __shared__ uint32_t s_ncand;
  const int t = blockIdx.x;
  const int32_t n = lv.n;
  const int gb = 1 - gs;
  int8_t* part = tpart + (int64_t)t * n;
  int64_t* conn = tconn + (int64_t)t * n;
  int32_t* adjc = tadj + (int64_t)t * n;
  RefCtl* rc = tctl + t;
  const int64_t tg = ctrl->tgt[gs], mg = ctrl->ref.maxw[gs];
  int64_t W = 0;
  for (int32_t v = threadIdx.x; v < n; v += BS) {
    part[v] = (int8_t)gb;
    conn[v] = 0;
    adjc[v] = 0;
    W += lv.b[v];
  }
  W = block_sum<BS, int64_t>(W, sml);
  const int32_t seedv = (int32_t)(((int64_t)t * n) / K);
  int64_t pg = 0;
  bool first = true;
  __syncthreads();
  while (pg < tg) {
    int32_t pick = -1;
    if (first && pg + lv.b[seedv] <= mg) {
      pick = seedv;
    } else {
      GrowBest best;
      best.v = -1;
      best.a = 0;
      best.g = 0;
      for (int32_t v = threadIdx.x; v < n; v += BS) {
        if (part[v] != gb || pg + lv.b[v] > mg) continue;
        GrowBest x;
        x.a = adjc[v] > 0;
        x.g = 2 * conn[v] - tot[v];
        x.v = v;
        if (grow_better(x, best)) best = x;
      }
      best = block_grow_argmax<BS>(best, sgb);
      pick = best.v;
    }
    first = false;
    if (pick < 0) break;
    if (threadIdx.x == 0) part[pick] = (int8_t)gs;
    for (int32_t e = lv.xadj[pick] + threadIdx.x; e < lv.xadj[pick + 1]; e += BS) {
      const int32_t x = lv.adj[e];
      conn[x] += lv.w[e];
      adjc[x] += 1;
    }
    pg += lv.b[pick];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rc->maxw[0] = ctrl->ref.maxw[0];
    rc->maxw[1] = ctrl->ref.maxw[1];
    rc->pw[gs] = pg;
    rc->pw[gb] = W - pg;
    start_level(rc, npass);
  }
  __syncthreads();
  refine_block<BS>(lv, part, rc, tlist + (int64_t)t * (n > 0 ? n : 1), &sel, sml, &s_ncand);
  __syncthreads();
  int64_t ext = 0;
  for (int32_t v = threadIdx.x; v < n; v += BS) {
    const int8_t pv = part[v];
    for (int32_t e = lv.xadj[v]; e < lv.xadj[v + 1]; e++)
      if (part[lv.adj[e]] != pv) ext += lv.w[e];
  }
  ext = block_sum<BS, int64_t>(ext, sml);
  if (threadIdx.x == 0) {
    tres[2 * t] = ext / 2;
    tres[2 * t + 1] = (rc->pw[0] > rc->maxw[0] || rc->pw[1] > rc->maxw[1]) ? 1 : 0;
  }
  if (!last_block(&ctrl->ctr_init, gridDim.x)) return;
  __shared__ int s_best;
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < K; i++) {
      const int64_t ci = tres[2 * i], ii = tres[2 * i + 1];
      const int64_t cb = tres[2 * best], ib = tres[2 * best + 1];
      if (ii < ib || (ii == ib && ci < cb)) best = i;
    }
    s_best = best;
    ctrl->ref.pw[0] = tctl[best].pw[0];
    ctrl->ref.pw[1] = tctl[best].pw[1];
    ctrl->ref.last_cut = tres[2 * best];
  }
  __syncthreads();
  const int8_t* bp = tpart + (int64_t)s_best * n;
  for (int32_t v = threadIdx.x; v < n; v += BS) out_part[v] = bp[v];
}

// -------------------------------------------------------------- gp_create
__global__ __launch_bounds__(kBlock) void k_val_xadj(int32_t n, const int32_t* xadj, Ctrl* ctrl) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    if ((v == 0 && xadj[0] != 0) || xadj[v + 1] < xadj[v]) atomicOr(&ctrl->verr, kVInval);
  }
}

// saturating block sum of values <= 2^62 (a + b never exceeds 2^63)
__device__ __forceinline__ uint64_t sat62(uint64_t a, uint64_t b) {
  const uint64_t lim = 1ull << 62;
  uint64_t s = a + b;
  return s > lim ? lim : s;
}

template <int BS>
__device__ uint64_t block_sum_sat(uint64_t v, uint64_t* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = sat62(v, __shfl_xor(v, o, 64));
  if (lane_id() == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  uint64_t r = 0;
  for (int i = 0; i < BS / 64; i++) r = sat62(r, sm[i]);
  __syncthreads();
  return r;
}

// ranges, self loops, sortedness, weight sums; one 16-lane team per row
__global__ __launch_bounds__(kBlock) void k_val_rows(int32_t n, const int32_t* xadj,
                                                     const int32_t* adj, const int64_t* w,
                                                     const int64_t* vc, const int64_t* vg,
                                                     Ctrl* ctrl) {
  __shared__ uint64_t smu[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  const uint64_t lim = 1ull << 62;
  uint32_t err = 0, unsorted = 0;
  uint64_t sw = 0, sc = 0, sg = 0;
  int64_t mc = 0, mg = 0;
  const int lane = threadIdx.x & 15;
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 16;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / 16;
  for (int64_t uu = team; uu < n; uu += nteams) {
    const int32_t u = (int32_t)uu;
    for (int32_t e = xadj[u] + lane; e < xadj[u + 1]; e += 16) {
      const int32_t v = adj[e];
      const int64_t x = w[e];
      if (v < 0 || v >= n || x < 0) err |= kVRange;
      else if (v == u) err |= kVSelf;
      if (e + 1 < xadj[u + 1] && adj[e + 1] <= v) unsorted = 1;
      if (x >= 0) sw = sat62(sw, (uint64_t)x < lim ? (uint64_t)x : lim);
    }
    if (lane == 0) {
      const int64_t a = vc[u], b = vg[u];
      if (a < 0 || b < 0) err |= kVRange;
      if (a >= 0) {
        sc = sat62(sc, (uint64_t)a < lim ? (uint64_t)a : lim);
        mc = a > mc ? a : mc;
      }
      if (b >= 0) {
        sg = sat62(sg, (uint64_t)b < lim ? (uint64_t)b : lim);
        mg = b > mg ? b : mg;
      }
    }
  }
  sw = block_sum_sat<kBlock>(sw, smu);
  sc = block_sum_sat<kBlock>(sc, smu);
  sg = block_sum_sat<kBlock>(sg, smu);
  mc = block_max<kBlock, int64_t>(mc, sml);
  mg = block_max<kBlock, int64_t>(mg, sml);
  if (err) atomicOr(&ctrl->verr, err);
  if (unsorted) atomicOr(&ctrl->vunsorted, 1u);
  if (threadIdx.x == 0) {
    // every addend is <= 2^62; the flag is raised before a sum could wrap
    uint64_t o;
    o = atomicAdd((unsigned long long*)&ctrl->vsum_w, (unsigned long long)sw);
    if (o + sw >= lim) atomicOr(&ctrl->verr, kVOverflow);
    o = atomicAdd((unsigned long long*)&ctrl->vsum_c, (unsigned long long)sc);
    if (o + sc >= lim) atomicOr(&ctrl->verr, kVOverflow);
    o = atomicAdd((unsigned long long*)&ctrl->vsum_g, (unsigned long long)sg);
    if (o + sg >= lim) atomicOr(&ctrl->verr, kVOverflow);
    atomicMax((long long*)&ctrl->vmax_c, (long long)mc);
    atomicMax((long long*)&ctrl->vmax_g, (long long)mg);
  }
}

// sort every row by neighbour (no merging), flag repeated neighbours
struct PlainRowLoader {
  const int32_t* adj;
  const int64_t* w;
  int32_t e0;
  __device__ __forceinline__ void operator()(int i, int32_t& k, int64_t& v) const {
    k = adj[e0 + i];
    v = w[e0 + i];
  }
};

__global__ __launch_bounds__(kBlock) void k_sort_rows(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl) {
  __shared__ int32_t sk[kSortCap];
  __shared__ int64_t sv[kSortCap];
  __shared__ int32_t smi[kBlock / 64];
  bool dup = false;
  for (int64_t u0 = (int64_t)blockIdx.x * kTileC; u0 < n; u0 += (int64_t)gridDim.x * kTileC) {
    const int64_t u1 = u0 + kTileC < n ? u0 + kTileC : n;
    for (int64_t u = u0 + threadIdx.x / 16; u < u1; u += kBlock / 16) {
      const int32_t e0 = xadj[u], L = xadj[u + 1] - e0;
      if (L > 16) continue;
      const int lane = threadIdx.x & 15;
      int32_t k = INT_MAX;
      int64_t v = 0;
      if (lane < L) {
        k = adj[e0 + lane];
        v = w[e0 + lane];
      }
      team_bitonic<16>(k, v);
      team_emit<16, false>(k, v, oadj + e0, ow + e0, &dup);
    }
    for (int64_t u = u0 + threadIdx.x / 64; u < u1; u += kBlock / 64) {
      const int32_t e0 = xadj[u], L = xadj[u + 1] - e0;
      if (L <= 16 || L > 64) continue;
      const int lane = threadIdx.x & 63;
      int32_t k = INT_MAX;
      int64_t v = 0;
      if (lane < L) {
        k = adj[e0 + lane];
        v = w[e0 + lane];
      }
      team_bitonic<64>(k, v);
      team_emit<64, false>(k, v, oadj + e0, ow + e0, &dup);
    }
    for (int64_t u = u0; u < u1; u++) {
      const int32_t e0 = xadj[u], L = xadj[u + 1] - e0;
      if (L <= 64 || L > kSortCap) continue;
      PlainRowLoader ld{adj, w, e0};
      block_sort_emit<kBlock, false>(L, ld, sk, sv, oadj + e0, ow + e0, &dup, smi);
    }
  }
  if (dup) atomicOr(&ctrl->verr, kVDup);
}

// rows longer than kSortCap: dense merge over id windows, one block per row
__global__ __launch_bounds__(kBlock) void k_sort_long(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl) {
  extern __shared__ unsigned char dyn[];
  int64_t* acc = (int64_t*)dyn;
  int32_t* cc = (int32_t*)(acc + kWin);
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  bool dup = false;
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const int32_t e0 = xadj[u], L = xadj[u + 1] - e0;
    if (L <= kSortCap) continue;
    PlainRowLoader ld{adj, w, e0};
    block_dense_emit<kBlock, false>(L, ld, acc, cc, smi, sml, oadj + e0, ow + e0, &dup);
  }
  if (dup) atomicOr(&ctrl->verr, kVDup);
}

// every entry u->v must have v->u with the same weight (rows sorted)
__global__ __launch_bounds__(kBlock) void k_val_sym(int32_t n, const int32_t* xadj,
                                                    const int32_t* adj, const int64_t* w,
                                                    Ctrl* ctrl) {
  const int lane = threadIdx.x & 15;
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 16;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / 16;
  bool bad = false;
  for (int64_t uu = team; uu < n; uu += nteams) {
    const int32_t u = (int32_t)uu;
    for (int32_t e = xadj[u] + lane; e < xadj[u + 1]; e += 16) {
      const int32_t v = adj[e];
      int32_t lo = xadj[v], hi = xadj[v + 1] - 1;
      bool found = false;
      while (lo <= hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        const int32_t x = adj[mid];
        if (x == u) {
          found = w[mid] == w[e];
          break;
        }
        if (x < u) lo = mid + 1;
        else hi = mid - 1;
      }
      if (!found) bad = true;
    }
  }
  if (bad) atomicOr(&ctrl->verr, kVAsym);
}

__global__ void k_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    vc[v] = vwgt[2 * v];
    vg[v] = vwgt[2 * v + 1];
  }
}

// ================================================================ launchers
#define KCHECK()                         \
  do {                                   \
    if (hipGetLastError() != hipSuccess) \
      return false;                      \
  } while (0)

int team_width_for(int32_t n, int64_t nnz) {
  const double avg = n > 0 ? (double)nnz / n : 0.0;
  if (avg <= 6) return 4;
  if (avg <= 12) return 8;
  if (avg <= 24) return 16;
  if (avg <= 48) return 32;
  return 64;
}

bool launch_level_reset(Ctrl* ctrl, int promote, hipStream_t s) {
  k_level_reset<<<1, 64, 0, s>>>(ctrl, promote);
  KCHECK();
  return true;
}

template <int TW>
static bool propose_tw(const LevelView& lv, const int32_t* match, int32_t* prop, const Ctrl* ctrl,
                       int round, uint64_t hs, hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * TW, kBlock * 2);
  k_match_propose<TW><<<grid, kBlock, 0, s>>>(lv, match, prop, ctrl, round, hs);
  KCHECK();
  return true;
}

bool launch_match_round(const LevelView& lv, int32_t* match, int32_t* prop, Ctrl* ctrl, int round,
                        uint64_t hs, int tw, hipStream_t s) {
  bool ok;
  switch (tw) {
    case 4: ok = propose_tw<4>(lv, match, prop, ctrl, round, hs, s); break;
    case 8: ok = propose_tw<8>(lv, match, prop, ctrl, round, hs, s); break;
    case 16: ok = propose_tw<16>(lv, match, prop, ctrl, round, hs, s); break;
    case 32: ok = propose_tw<32>(lv, match, prop, ctrl, round, hs, s); break;
    default: ok = propose_tw<64>(lv, match, prop, ctrl, round, hs, s); break;
  }
  if (!ok) return false;
  k_match_resolve<<<grid_for(lv.n, kBlock * 4), kBlock, 0, s>>>(lv.n, match, prop, ctrl, round);
  KCHECK();
  return true;
}

template <int TW>
static bool twohop_tw(const LevelView& lv, int32_t* match, int32_t* hub, const Ctrl* ctrl,
                      uint64_t hs, hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * TW, kBlock * 2);
  k_hub<TW><<<grid, kBlock, 0, s>>>(lv, match, hub, hs);
  KCHECK();
  k_twohop<TW><<<grid, kBlock, 0, s>>>(lv, hub, match, ctrl);
  KCHECK();
  return true;
}

bool launch_twohop(const LevelView& lv, int32_t* match, Ctrl* ctrl, const Scratch& sc,
                   uint64_t hs, int tw, hipStream_t s) {
  bool ok;
  switch (tw) {
    case 4: ok = twohop_tw<4>(lv, match, sc.prop, ctrl, hs, s); break;
    case 8: ok = twohop_tw<8>(lv, match, sc.prop, ctrl, hs, s); break;
    case 16: ok = twohop_tw<16>(lv, match, sc.prop, ctrl, hs, s); break;
    case 32: ok = twohop_tw<32>(lv, match, sc.prop, ctrl, hs, s); break;
    default: ok = twohop_tw<64>(lv, match, sc.prop, ctrl, hs, s); break;
  }
  if (!ok) return false;
  const int ntiles = (lv.n + kTileV - 1) / kTileV;
  const int g = grid_for(ntiles, 1, 2048);
  k_iso_count<<<g, kBlock, 0, s>>>(lv, match, ctrl, sc.tile_lead, ntiles);
  KCHECK();
  k_iso_list<<<g, kBlock, 0, s>>>(lv, match, sc.tile_lead, sc.longlist, ntiles);
  KCHECK();
  k_iso_pair<<<grid_for(lv.n / 2 + 1, kBlock * 4), kBlock, 0, s>>>(lv.b, sc.longlist, match, ctrl);
  KCHECK();
  return true;
}

bool launch_contract_a(const LevelView& lv, const int32_t* match, const int64_t* vc,
                       const int64_t* vg, Ctrl* ctrl, const Scratch& sc, int32_t* cmap,
                       int64_t* cvc, int64_t* cvg, hipStream_t s) {
  const int ntiles = (lv.n + kTileV - 1) / kTileV;
  const int g = grid_for(ntiles, 1, 2048);
  k_contract_count<<<g, kBlock, 0, s>>>(lv, match, ctrl, sc.tile_lead, sc.tile_ub, ntiles);
  KCHECK();
  k_contract_map<<<g, kBlock, 0, s>>>(lv, match, vc, vg, sc.tile_lead, sc.tile_ub, cmap, cvc, cvg,
                                      sc.cmem0, sc.cmem1, sc.toff, ntiles);
  KCHECK();
  return true;
}

// nc_max: an upper bound of the coarse vertex count (sizes the grids)
bool launch_contract_b(const LevelView& lv, const int32_t* cmap, Ctrl* ctrl, const Scratch& sc,
                       int32_t nc_max, int32_t* cxadj, int32_t* cadj, int64_t* cw,
                       hipStream_t s) {
  const int ntc = (nc_max + kTileC - 1) / kTileC;
  const int ntc1 = ntc > 0 ? ntc : 1;
  const int g = grid_for(ntc1, 1, 4096);
  k_contract_rows<<<g, kBlock, 0, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, sc.tmpk,
                                       sc.tmpv, sc.cnt, sc.tile_cnt, sc.longlist, ctrl, ntc1);
  KCHECK();
  const size_t dyn = (size_t)kWin * (sizeof(int64_t) + sizeof(int32_t));
  k_contract_long<<<64, kBlock, dyn, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, sc.tmpk,
                                          sc.tmpv, sc.cnt, sc.tile_cnt, sc.longlist, ntc1);
  KCHECK();
  k_contract_compact<<<g, kBlock, 0, s>>>(ctrl, sc.toff, sc.cnt, sc.tile_cnt, sc.tmpk, sc.tmpv,
                                          cxadj, cadj, cw, ntc1);
  KCHECK();
  return true;
}

template <int TW>
static bool gain_tw(const LevelView& lv, const int8_t* part, RefCtl* rc, Cand* list,
                    hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * TW, kBlock * 2);
  k_refine_gain<TW><<<grid, kBlock, 0, s>>>(lv, part, rc, list);
  KCHECK();
  return true;
}

bool launch_refine_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list, int tw,
                        hipStream_t s) {
  bool ok;
  switch (tw) {
    case 4: ok = gain_tw<4>(lv, part, rc, list, s); break;
    case 8: ok = gain_tw<8>(lv, part, rc, list, s); break;
    case 16: ok = gain_tw<16>(lv, part, rc, list, s); break;
    case 32: ok = gain_tw<32>(lv, part, rc, list, s); break;
    default: ok = gain_tw<64>(lv, part, rc, list, s); break;
  }
  if (!ok) return false;
  k_refine_apply<<<grid_for(lv.n, kBlock * 8, 1024), kBlock, 0, s>>>(part, rc, list);
  KCHECK();
  return true;
}

bool launch_project(int32_t n, const int32_t* cmap, const int8_t* cpart, int8_t* part, RefCtl* rc,
                    int npass, hipStream_t s) {
  k_project<<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, cmap, cpart, part, rc, npass);
  KCHECK();
  return true;
}

bool launch_start_level(RefCtl* rc, int npass, hipStream_t s) {
  k_start_level<<<1, 64, 0, s>>>(rc, npass);
  KCHECK();
  return true;
}

bool launch_final_stats(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const int8_t* part, Ctrl* ctrl, int tw, hipStream_t s) {
  k_clear_stats<<<1, 64, 0, s>>>(ctrl);
  KCHECK();
  const int grid = grid_for((int64_t)lv.n * tw, kBlock * 2);
  switch (tw) {
    case 4: k_final_stats<4><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl); break;
    case 8: k_final_stats<8><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl); break;
    case 16: k_final_stats<16><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl); break;
    case 32: k_final_stats<32><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl); break;
    default: k_final_stats<64><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl); break;
  }
  KCHECK();
  return true;
}

bool launch_init(const LevelView& lv, int K, int gs, int npass, Ctrl* ctrl, const InitScratch& is,
                 int8_t* out_part, hipStream_t s) {
  k_init_tot<<<grid_for(lv.n, kBlock), kBlock, 0, s>>>(lv, is.tot);
  KCHECK();
  k_init_trials<kInitBlock><<<K, kInitBlock, 0, s>>>(lv, is.tot, K, gs, npass, ctrl, is.ctl,
                                                     is.part, is.conn, is.adjc, is.list, is.res,
                                                     out_part);
  KCHECK();
  return true;
}

bool launch_validate(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                     const int64_t* vc, const int64_t* vg, Ctrl* ctrl, int stage,
                     hipStream_t s) {
  const int g = grid_for(n, kBlock);
  if (stage == 0) {
    k_val_xadj<<<g, kBlock, 0, s>>>(n, xadj, ctrl);
  } else if (stage == 1) {
    k_val_rows<<<grid_for((int64_t)n * 16, kBlock * 2), kBlock, 0, s>>>(n, xadj, adj, w, vc, vg,
                                                                         ctrl);
  } else {
    k_val_sym<<<grid_for((int64_t)n * 16, kBlock * 2), kBlock, 0, s>>>(n, xadj, adj, w, ctrl);
  }
  KCHECK();
  return true;
}

bool launch_sort_rows(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                      int32_t* oadj, int64_t* ow, Ctrl* ctrl, hipStream_t s) {
  k_sort_rows<<<grid_for((n + kTileC - 1) / kTileC, 1, 4096), kBlock, 0, s>>>(n, xadj, adj, w,
                                                                                oadj, ow, ctrl);
  KCHECK();
  const size_t dyn = (size_t)kWin * (sizeof(int64_t) + sizeof(int32_t));
  k_sort_long<<<64, kBlock, dyn, s>>>(n, xadj, adj, w, oadj, ow, ctrl);
  KCHECK();
  return true;
}

bool launch_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg, hipStream_t s) {
  k_split_vwgt<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, vwgt, vc, vg);
  KCHECK();
  return true;
}

}  // namespace gpk
