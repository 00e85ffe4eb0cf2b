// gp_phases.h - device bodies of every phase of the partition pipeline.
//
// Each body b_X(..., bid, nblk) does the work of block bid out of nblk
// blocks.  The single-graph path launches each body as its own kernel over
// many blocks (gp_kernels.hip); the batched path calls the same bodies with
// (0, 1) from inside one persistent kernel, one workgroup per graph
// (gp_batch.hip).  A phase with a single-block tail runs it in the last
// block to finish (tail_gate).  Large LDS buffers are passed in by the
// caller so that one kernel can run several phases.
#pragma once

#include <stdlib.h>

#include "gp_dev.h"

namespace gpk {


// ------------------------------------------------------------------ helpers
// clears the per-level coarsening counters; on levels below the input graph
// the largest balance weight measured by the previous contraction becomes
// the current one
__device__ __forceinline__ void b_level_reset(Ctrl* ctrl, int promote, int bid_, int nblk_) {
  for (int i = threadIdx.x; i < kMaxRounds; i += blockDim.x) ctrl->made[i] = 0;
  if (threadIdx.x == 0) {
    if (promote) ctrl->maxb = ctrl->maxb_next;
    ctrl->nc = 0;
    ctrl->nnz_c = 0;
    ctrl->nlong = 0;
    ctrl->ubtot = 0;
    ctrl->long_in = 0;
    ctrl->long_out = 0;
    ctrl->nhuge = 0;
    ctrl->huge_in = 0;
    ctrl->huge_out = 0;
    ctrl->short_in = 0;
    ctrl->short_out = 0;
    ctrl->deferred = 0;
    ctrl->maxb_next = 0;
  }
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

// Matching rounds.  Round r >= 1 runs in two steps (two kernels in the
// single-graph path, one segment of one workgroup in the batched path):
// b_match_free settles the mutual proposals of round r - 1 and
// lists the vertices still free (fr[v] = 1 when match[v] is -1 afterwards),
// then b_match_round proposes for the listed vertices only, among their free
// neighbours, so the test of a neighbour is one byte gathered from an
// n-byte array and a late round costs what its few free vertices cost.
// Both kernels run one block per segment: segment k is vertex range
// [kS, kS + S) (S = ceil(n / blocks)); its list of round r holds the free
// vertices of that range in ascending id at slots [kS, kS + cnt[k]), so no
// global counter is needed.  Round r's settle only visits list r - 1 (round
// 0: every vertex), since a vertex matched before stays matched.  Proposals
// are double-buffered (prop_prev, prop_cur); an entry of a vertex that is no
// longer listed goes stale, which no one reads: a listed vertex proposes to
// a listed one.  b_match_settle settles the last round.
//
// When settling round r - 1 matched nothing, round r proposes exactly what
// round r - 1 did (same free vertices, same rule), so it has no mutual pair
// either and every later round repeats it: those rounds return at once.
// Both proposal buffers then hold the same proposals of the listed
// vertices, so the final settle reads either.  made[r] = 1 records that
// round r's settle matched.
__device__ __forceinline__ void b_match_free(int32_t n, int32_t* match, const int32_t* prop_prev,
                                             uint8_t* fr, const int32_t* lin,
                                             const int32_t* cin, int32_t* lout, int32_t* cout,
                                             Ctrl* ctrl, int round, int seg, int nseg) {
  if (round >= 2 && ctrl->made[round - 1] == 0) return;
  __shared__ int32_t smi[kBlock / 64];
  const int64_t S = ((int64_t)n + nseg - 1) / nseg;
  const int64_t lo = (int64_t)seg * S;
  const int64_t hi = lo + S < n ? lo + S : n;
  const int32_t cnt = round == 1 ? (int32_t)(hi > lo ? hi - lo : 0) : cin[seg];
  bool settled = false;
  int32_t kept = 0;
  for (int32_t i0 = 0; i0 < cnt; i0 += kBlock) {
    const int32_t i = i0 + (int32_t)threadIdx.x;
    bool keep = false;
    int32_t u = 0;
    if (i < cnt) {
      u = round == 1 ? (int32_t)(lo + i) : lin[lo + i];
      int32_t m = match[u];
      const int32_t p = prop_prev[u];
      if (m == -1 && p >= 0 && prop_prev[p] == u) {
        m = p;
        match[u] = p;
        settled = true;
      }
      keep = m == -1;
      fr[u] = keep ? 1 : 0;
    }
    int32_t tot;
    const int32_t ex = block_exscan<kBlock, int32_t>(keep ? 1 : 0, smi, &tot);
    if (keep) lout[lo + kept + ex] = u;
    kept += tot;
  }
  if (threadIdx.x == 0) cout[seg] = kept;
  if (__syncthreads_or(settled) && threadIdx.x == 0) ctrl->made[round] = 1;
}

template <int TW>
__device__ __forceinline__ void b_match_round(LevelView lv, int32_t* match, const uint8_t* fr,
                                              const int32_t* list, const int32_t* lcnt,
                                              const int32_t* prop_prev, int32_t* prop_cur,
                                              Ctrl* ctrl, int round, uint64_t hs, int seg,
                                              int nseg) {
  if (round >= 2 && ctrl->made[round - 1] == 0) return;
  const int64_t cap = ctrl->cap, maxb = ctrl->maxb;
  const int lane = threadIdx.x & (TW - 1);
  const int64_t S = ((int64_t)lv.n + nseg - 1) / nseg;
  const int64_t lo = (int64_t)seg * S;
  const int64_t hi = lo + S < lv.n ? lo + S : lv.n;
  const int32_t cnt = round == 0 ? (int32_t)(hi > lo ? hi - lo : 0) : lcnt[seg];
  for (int32_t ii = (int32_t)threadIdx.x / TW; ii < cnt; ii += kBlock / TW) {
    const int32_t u = round == 0 ? (int32_t)(lo + ii) : list[lo + ii];
    // loads that do not depend on each other are issued together, before
    // any test, so that each chain costs as few global round trips as it can
    const int64_t bu = lv.b[u];
    const int32_t e0 = lv.xadj[u], e1 = lv.xend[u];
    if (round > 0) {
      // The neighbours free at this round's start are a subset of those free
      // at the previous round's start, and the weight cap does not change:
      // if u's previous choice t is still free, t is still the best, and if
      // u had no choice it still has none.  Only the others rescan the row.
      const int32_t t = prop_prev[u];
      if (t < 0 || fr[t] != 0) {
        if (lane == 0) prop_cur[u] = t;
        continue;
      }
    } else if (lane == 0) {
      match[u] = -1;
    }
    const bool capcheck = bu + maxb > cap;
    int64_t bw = -1;
    int32_t bv = -1;
    // U entries per lane in flight on long rows (wide teams): the entry
    // loads, then the gathers they feed, then the tests (the maximum does not
    // depend on the order); short rows keep one, for fewer registers
    constexpr int U = TW >= 32 ? 4 : (TW == 16 ? 2 : 1);
    for (int32_t e = e0 + lane; e < e1; e += TW * U) {
      int32_t vk[U];
      int64_t wk[U];
#pragma unroll
      for (int k = 0; k < U; k++) {
        const int32_t q = e + TW * k;
        vk[k] = q < e1 ? lv.adj[q] : 0;
        wk[k] = q < e1 ? lv.w[q] : 0;
      }
      bool ok[U];
      int64_t bk[U];
#pragma unroll
      for (int k = 0; k < U; k++) {
        const bool in = e + TW * k < e1;
        ok[k] = in && (round == 0 || fr[vk[k]] != 0);
        bk[k] = in && capcheck ? lv.b[vk[k]] : 0;
      }
#pragma unroll
      for (int k = 0; k < U; k++) {
        if (!ok[k] || (capcheck && bu + bk[k] > cap)) continue;
        if (match_better(wk[k], vk[k], bw, bv, hs, u)) {
          bw = wk[k];
          bv = vk[k];
        }
      }
    }
    butterfly<TW>([&](auto o) {
      const int64_t ow = xor_lane<decltype(o)::value>(bw);
      const int32_t ov = xor_lane<decltype(o)::value>(bv);
      if (match_better(ow, ov, bw, bv, hs, u)) {
        bw = ow;
        bv = ov;
      }
    });
    if (lane == 0) prop_cur[u] = bv;
  }
}

// settles the mutual proposals of the last round; clears the hub flags of
// the two-hop pass that follows (when given)
__device__ __forceinline__ void b_match_settle(int32_t n, int32_t* match, const int32_t* prop,
                                               int bid_, int nblk_, uint8_t* hflag = nullptr) {
  for (int64_t u = (int64_t)bid_ * kBlock + threadIdx.x; u < n;
       u += (int64_t)nblk_ * kBlock) {
    if (hflag) hflag[u] = 0;
    if (match[u] != -1) continue;
    const int32_t p = prop[u];
    if (p >= 0 && prop[p] == (int32_t)u) match[u] = p;
  }
}

// --------------------------------------------------------------- two-hop pass
// hub[u] = first neighbour of an unmatched u under the edge order (-1: none);
// matched vertices get -2.  hflag[h] = 1 marks every vertex that is some
// vertex's hub (the flags were cleared by the settle before).
template <int TW>
__device__ __forceinline__ void b_hub(LevelView lv, const int32_t* match, int32_t* hub,
                                      uint64_t hs, int bid_, int nblk_,
                                      uint8_t* hflag = nullptr) {
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t uu = team; uu < lv.n; uu += nteams) {
    const int32_t u = (int32_t)uu;
    if (match[u] != -1) {
      if (lane == 0) hub[u] = -2;
      continue;
    }
    int64_t bw = -1;
    int32_t bv = -1;
    const int32_t e1 = lv.xend[u];
    for (int32_t e = lv.xadj[u] + lane; e < e1; e += TW) {
      const int32_t v = lv.adj[e];
      const int64_t w = lv.w[e];
      if (match_better(w, v, bw, bv, hs, u)) {
        bw = w;
        bv = v;
      }
    }
    butterfly<TW>([&](auto o) {
      const int64_t ow = xor_lane<decltype(o)::value>(bw);
      const int32_t ov = xor_lane<decltype(o)::value>(bv);
      if (match_better(ow, ov, bw, bv, hs, u)) {
        bw = ow;
        bv = ov;
      }
    });
    if (lane == 0) {
      hub[u] = bv;
      if (hflag && bv >= 0) hflag[bv] = 1;
    }
  }
}

// The members of h's group are the x in row h with hub[x] == h; the sorted
// row lists them in ascending id.  They are paired first-second,
// third-fourth, ... when the pair fits under the cap.  Each unmatched vertex
// has one hub, so every match[] entry is written by one team only.  A vertex
// that is nobody's hub (hflag[h] == 0) has no members and pairs nothing, so
// its row is not read.
template <int TW>
__device__ __forceinline__ void b_twohop(LevelView lv, const int32_t* hub, int32_t* match,
                                         const Ctrl* ctrl, int bid_, int nblk_,
                                         const uint8_t* hflag = nullptr) {
  const int64_t cap = ctrl->cap;
  const int lane = threadIdx.x & (TW - 1);
  const int tb = lane_id() & ~(TW - 1);
  const uint64_t tmask = TW == 64 ? ~0ull : ((1ull << TW) - 1ull);
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t hh = team; hh < lv.n; hh += nteams) {
    const int32_t h = (int32_t)hh;
    if (hflag && hflag[h] == 0) continue;  // the whole team skips together
    const int32_t e1 = lv.xend[h];
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
// exclusive scan of the isolated-vertex tile counts (one block)
__device__ __forceinline__ void b_iso_scan(Ctrl* ctrl, int32_t* tile_cnt, int ntiles) {
  __shared__ int32_t smi[kBlock / 64];
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

// Multi-block phases end without a completion count: on a multi-die GPU the
// release fence each finishing block would need writes its L2 back, which
// costs far more than a separate one-block launch for the tail.  The batched
// path (one block per graph) runs the tail inline (inline_tail).
__device__ __forceinline__ void b_iso_count(LevelView lv, const int32_t* match,
                                                      Ctrl* ctrl, int32_t* tile_cnt,
                                                      int ntiles, int bid_, int nblk_,
                                                      bool inline_tail = true) {
  __shared__ int32_t smi[kBlock / 64];
  for (int t = bid_; t < ntiles; t += nblk_) {
    int32_t c = 0;
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      if (u < lv.n && match[u] == -1 && lv.xend[u] == lv.xadj[u]) c++;
    }
    c = block_sum<kBlock, int32_t>(c, smi);
    if (threadIdx.x == 0) tile_cnt[t] = c;
  }
  if (!inline_tail) return;
  __syncthreads();
  b_iso_scan(ctrl, tile_cnt, ntiles);
}

__device__ __forceinline__ void b_iso_list(LevelView lv, const int32_t* match,
                                                     const int32_t* tile_base, int32_t* iso,
                                                     int ntiles, int bid_, int nblk_) {
  __shared__ int32_t smi[kBlock / 64];
  for (int t = bid_; t < ntiles; t += nblk_) {
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    bool f[4];
    int32_t c = 0;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      f[j] = u < lv.n && match[u] == -1 && lv.xend[u] == lv.xadj[u];
      c += f[j];
    }
    int32_t tot;
    int32_t r = tile_base[t] + block_exscan<kBlock, int32_t>(c, smi, &tot);
    for (int j = 0; j < 4; j++)
      if (f[j]) iso[r++] = (int32_t)(base + j);
  }
}

__device__ __forceinline__ void b_iso_pair(const int64_t* b, const int32_t* iso,
                                                     int32_t* match, const Ctrl* ctrl, int bid_, int nblk_) {
  const int32_t npairs = ctrl->niso / 2;
  const int64_t cap = ctrl->cap;
  for (int64_t i = (int64_t)bid_ * kBlock + threadIdx.x; i < npairs;
       i += (int64_t)nblk_ * kBlock) {
    const int32_t x = iso[2 * i], y = iso[2 * i + 1];
    if (b[x] + b[y] <= cap) {
      match[x] = y;
      match[y] = x;
    }
  }
}

// --------------------------------------------------------------- contraction
// tile t covers fine vertices [t*kTileV, (t+1)*kTileV); each thread 4 of them
__device__ __forceinline__ void b_contract_scan(Ctrl* ctrl, int32_t* tile_lead, int64_t* tile_ub,
                                                int ntiles, const int64_t* partials,
                                                int nparts);

__device__ __forceinline__ void b_contract_count(LevelView lv, const int32_t* match,
                                                           Ctrl* ctrl, int32_t* tile_lead,
                                                           int64_t* tile_ub, int ntiles, int64_t* partials, int bid_, int nblk_,
                                                           bool inline_tail = true) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ int32_t smi[kBlock / 64];
  int64_t mx = 0;
  for (int t = bid_; t < ntiles; t += nblk_) {
    int32_t lead = 0;
    int64_t ub = 0;
    const int64_t base = (int64_t)t * kTileV + threadIdx.x * 4;
    for (int j = 0; j < 4; j++) {
      const int64_t u = base + j;
      if (u >= lv.n) break;
      const int32_t m = match[u];
      if (m < 0 || u < m) {
        lead++;
        ub += lv.xend[u] - lv.xadj[u];
        int64_t bsum = lv.b[u];
        if (m >= 0) {
          ub += lv.xend[m] - lv.xadj[m];
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
  if (!inline_tail) {
    if (threadIdx.x == 0) partials[bid_] = mx;  // largest merged weight of this block
    return;
  }
  if (threadIdx.x == 0) ctrl->maxb_next = mx > ctrl->maxb_next ? mx : ctrl->maxb_next;
  __syncthreads();
  b_contract_scan(ctrl, tile_lead, tile_ub, ntiles, nullptr, 0);
}

// exclusive scans of the leader and entry-bound tile totals (one block); with
// partials, also the largest merged balance weight over nparts blocks
__device__ __forceinline__ void b_contract_scan(Ctrl* ctrl, int32_t* tile_lead, int64_t* tile_ub,
                                                int ntiles, const int64_t* partials,
                                                int nparts) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ int32_t smi[kBlock / 64];
  if (partials) {
    int64_t mx = 0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) mx = partials[i] > mx ? partials[i] : mx;
    mx = block_max<kBlock, int64_t>(mx, sml);
    if (threadIdx.x == 0) ctrl->maxb_next = mx > ctrl->maxb_next ? mx : ctrl->maxb_next;
  }
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

__device__ __forceinline__ void b_contract_map(LevelView lv, const int32_t* match,
                                                         const int64_t* vc, const int64_t* vg,
                                                         const int32_t* tile_lead,
                                                         const int64_t* tile_ub, int32_t* cmap,
                                                         int64_t* cvc, int64_t* cvg,
                                                         int32_t* cmem0, int32_t* cmem1,
                                                         int64_t* toff, int ntiles, int64_t* tile_cnt,
                                                         int ntiles_c, int bid_, int nblk_) {
  __shared__ int64_t sml[kBlock / 64];
  __shared__ int32_t smi[kBlock / 64];
  // coarse-tile entry counts, accumulated by the row sorts that follow
  for (int64_t i = (int64_t)bid_ * kBlock + threadIdx.x; i < ntiles_c;
       i += (int64_t)nblk_ * kBlock)
    tile_cnt[i] = 0;
  for (int t = bid_; t < ntiles; t += nblk_) {
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
        ub += lv.xend[u] - lv.xadj[u];
        if (m >= 0) ub += lv.xend[m] - lv.xadj[m];
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
      int64_t d = lv.xend[u] - lv.xadj[u];
      if (m >= 0) {
        cmap[m] = c;
        sc += vc[m];
        sg += vg[m];
        d += lv.xend[m] - lv.xadj[m];
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

// candidate i of a row already gathered into LDS
struct StagedLoader {
  const int32_t* k;
  const int64_t* v;
  __device__ __forceinline__ void operator()(int i, int32_t& kk, int64_t& vv) const {
    kk = k[i];
    vv = v[i];
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
  ld.d0 = lv.xend[m0] - ld.e0;
  ld.e1 = m1 >= 0 ? lv.xadj[m1] : 0;
  const int d1 = m1 >= 0 ? lv.xend[m1] - ld.e1 : 0;
  *L = ld.d0 + d1;
  return ld;
}

// returns the row's entry count (also stored to *cnt_out)
template <int T>
__device__ __forceinline__ int team_row(const CoarseRowLoader& ld, int L, int32_t* okey,
                                        int64_t* oval, int32_t* cnt_out) {
  const int lane = threadIdx.x & (T - 1);
  int32_t k = INT_MAX;
  int64_t v = 0;
  if (lane < L) ld(lane, k, v);
  team_bitonic<T>(k, v);
  bool dummy = false;
  int cnt = team_emit<T, true>(k, v, okey, oval, &dummy);
  if (lane == 0) *cnt_out = cnt;
  return cnt;
}

__device__ __forceinline__ int wave_row_packed(const LevelView& lv, const int32_t* cmap,
                                               const CoarseRowLoader& ld, int32_t c, int L,
                                               int32_t* sk, int32_t* ok, int64_t* ov);

// Rows are sorted in groups of kRowsPerBlock per block, each by a team sized
// to its candidate count: a 16-lane team for <= 16 candidates (team i takes
// row i), a 32-lane team for <= 32, a wave for <= 64 (all three in
// registers), a wave in its private LDS for <= kWaveCap; longer rows go to
// the lists of the long-row kernels.  Sixteen rows per block keep enough
// rows in flight to hide the gather latency on the large sparse levels.
constexpr int kRowsPerBlock = 16;

__device__ __forceinline__ void b_contract_rows(
    LevelView lv, const int32_t* cmap, const int32_t* cmem0, const int32_t* cmem1,
    const int64_t* toff, const Ctrl* ctrl, int32_t* tmpk, int64_t* tmpv, int32_t* cnt,
    int64_t* tile_cnt, int32_t* longlist, Ctrl* wctrl, int ntiles_c, unsigned char* lds,
    int bid_, int nblk_, int32_t* hugelist = nullptr, const int32_t* rowlist = nullptr,
    const int32_t* rowcnt = nullptr) {
  // lds: kBlock/64 wave-private regions of kWaveCap x (int64 + int32) bytes
  int64_t* sv = (int64_t*)lds;
  int32_t* sk = (int32_t*)(sv + kRowBlockCap);
  constexpr int R = kRowsPerBlock;
  __shared__ int32_t s_e0[R], s_d0[R], s_e1[R], s_len[R], s_c[R];
  // rows of each register or LDS class: [0] <= 32, [1] <= 64, [2] <= kWaveCap
  __shared__ int8_t s_list[3][R];
  __shared__ int32_t s_count[3];
  static_assert(kWaveCap * (kBlock / 64) <= kRowBlockCap, "wave regions exceed the block region");
  static_assert(R == kBlock / 16 && R <= 64, "a 16-lane team per row; the rows fit one wave");
  static_assert(kTileC % R == 0, "row groups nest in compaction tiles");
  (void)ntiles_c;
  // rowlist: block k sorts the rows b_contract_short listed in its segment
  // (rowcnt[k] of them, at rowlist[kS ...]), else every coarse row
  const int32_t nc = ctrl->nc;
  const int64_t S = rowlist ? ((int64_t)nc + nblk_ - 1) / nblk_ : 0;
  const int32_t nrow = rowlist ? rowcnt[bid_] : nc;
  if (rowlist) rowlist += bid_ * S;
  const int wave = threadIdx.x / 64;
  const int32_t ngroups = (nrow + R - 1) / R;
  int64_t li_acc = 0, hi_acc = 0;  // candidates of the rows listed (thread 0)
  for (int32_t grp = rowlist ? 0 : bid_; grp < ngroups; grp += rowlist ? 1 : nblk_) {
    const int32_t c0 = grp * R;
    const int rows = c0 + R < nrow ? R : nrow - c0;
    if (threadIdx.x < 64) {
      // wave 0 reads the rows' members and sorts the rows into classes
      int L = 0;
      int32_t c = 0;
      if ((int)threadIdx.x < rows) {
        c = rowlist ? rowlist[c0 + threadIdx.x] : c0 + (int32_t)threadIdx.x;
        s_c[threadIdx.x] = c;
        const int32_t m0 = cmem0[c], m1 = cmem1[c];
        const int32_t e0 = lv.xadj[m0], d0 = lv.xend[m0] - e0;
        const int32_t e1 = m1 >= 0 ? lv.xadj[m1] : 0;
        const int32_t d1 = m1 >= 0 ? lv.xend[m1] - e1 : 0;
        L = d0 + d1;
        s_e0[threadIdx.x] = e0;
        s_d0[threadIdx.x] = d0;
        s_e1[threadIdx.x] = e1;
        s_len[threadIdx.x] = L;
      }
      const bool in_rows = (int)threadIdx.x < rows;
      // rows beyond kWaveCap: one wave per row when the packed keys fit,
      // else one block per row; listed with one counter update per group
      const bool is_long =
          in_rows && L > kWaveCap && (!hugelist || (L <= kLongWave && nc < kPackMaxNc));
      const bool is_huge = in_rows && L > kWaveCap && !is_long;
      const uint64_t ml = __ballot(is_long), mh = __ballot(is_huge);
      if (ml | mh) {
        int bl = 0, bh = 0;
        if (threadIdx.x == 0) {
          if (ml) bl = atomicAdd(&wctrl->nlong, (int)__popcll(ml));
          if (mh) bh = atomicAdd(&wctrl->nhuge, (int)__popcll(mh));
        }
        bl = __shfl(bl, 0, 64);
        bh = __shfl(bh, 0, 64);
        const uint64_t lt = lanemask_lt();
        if (is_long) longlist[bl + __popcll(ml & lt)] = c;
        if (is_huge) hugelist[bh + __popcll(mh & lt)] = c;
        if (is_long || is_huge) cnt[c] = 0;
        const int64_t sl = team_sum<64, int64_t>(is_long ? (int64_t)L : 0);
        const int64_t sh = team_sum<64, int64_t>(is_huge ? (int64_t)L : 0);
        li_acc += sl;
        hi_acc += sh;
      }
      const bool cls[3] = {in_rows && L > 16 && L <= 32, in_rows && L > 32 && L <= 64,
                           in_rows && L > 64 && L <= kWaveCap};
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const uint64_t m = __ballot(cls[q]);
        if (cls[q]) s_list[q][__popcll(m & lanemask_lt())] = (int8_t)threadIdx.x;
        if (threadIdx.x == 0) s_count[q] = __popcll(m);
      }
    }
    __syncthreads();
    auto loader = [&](int i) {
      CoarseRowLoader ld;
      ld.xadj = lv.xadj;
      ld.adj = lv.adj;
      ld.w = lv.w;
      ld.cmap = cmap;
      ld.c = s_c[i];
      ld.e0 = s_e0[i];
      ld.d0 = s_d0[i];
      ld.e1 = s_e1[i];
      return ld;
    };
    {
      const int i = (int)threadIdx.x / 16;
      if (i < rows && s_len[i] <= 16) {
        const int32_t c = s_c[i];
        team_row<16>(loader(i), s_len[i], tmpk + toff[c], tmpv + toff[c], &cnt[c]);
      }
    }
    for (int q = (int)threadIdx.x / 32; q < s_count[0]; q += kBlock / 32) {
      const int i = s_list[0][q];
      const int32_t c = s_c[i];
      team_row<32>(loader(i), s_len[i], tmpk + toff[c], tmpv + toff[c], &cnt[c]);
    }
    for (int q = wave; q < s_count[1]; q += kBlock / 64) {
      const int i = s_list[1][q];
      const int32_t c = s_c[i];
      team_row<64>(loader(i), s_len[i], tmpk + toff[c], tmpv + toff[c], &cnt[c]);
    }
    for (int q = wave; q < s_count[2]; q += kBlock / 64) {
      const int i = s_list[2][q];
      const int32_t c = s_c[i];
      int k;
      if (nc < kPackMaxNc) {
        // packed keys in the wave's region (kWaveCap keys)
        k = wave_row_packed(lv, cmap, loader(i), c, s_len[i], sk + wave * kWaveCap,
                            tmpk + toff[c], tmpv + toff[c]);
      } else {
        bool dummy = false;
        k = wave_sort_emit<true>(s_len[i], loader(i), sk + wave * kWaveCap, sv + wave * kWaveCap,
                                 tmpk + toff[c], tmpv + toff[c], &dummy);
      }
      if (lane_id() == 0) cnt[c] = k;
    }
    __syncthreads();
    if (!rowlist && threadIdx.x < 64) {
      int64_t sum = (int)threadIdx.x < rows ? cnt[c0 + threadIdx.x] : 0;
      sum = team_sum<64, int64_t>(sum);
      if (threadIdx.x == 0 && sum)
        atomicAdd((unsigned long long*)&tile_cnt[c0 / kTileC], (unsigned long long)sum);
    }
  }
  if (threadIdx.x == 0) {
    if (li_acc) atomicAdd((unsigned long long*)&wctrl->long_in, (unsigned long long)li_acc);
    if (hi_acc) atomicAdd((unsigned long long*)&wctrl->huge_in, (unsigned long long)hi_acc);
  }
}

// Rows of at most T candidates, one T-lane team each (T = 32 in the
// single-graph path; 16 in the batched path, whose one workgroup per graph
// needs more rows in flight): the team reads its row's members, gathers and sorts the candidates in registers and writes
// the merged row.  Block k takes the rows [kS, kS + S) (S = ceil(nc /
// blocks)) and lists its longer rows at defer[kS ...], dcnt[k] of them,
// for b_contract_rows (no global counter).  With few registers and no
// barrier in the row loop, many rows' gather chains are in flight at once on
// the large sparse levels.
template <int T = 32>
__device__ __forceinline__ void b_contract_short(LevelView lv, const int32_t* cmap,
                                                 const int32_t* cmem0, const int32_t* cmem1,
                                                 const int64_t* toff, const Ctrl* ctrl,
                                                 int32_t* okey, int64_t* oval, int32_t* cnt,
                                                 int32_t* defer, int32_t* dcnt, int64_t* sio,
                                                 int seg, int nseg) {
  __shared__ int32_t s_nd;
  __shared__ int64_t sml[kBlock / 64];
  int64_t rin = 0, rout = 0;  // candidates read and entries written (lane 0 of each team)
  if (threadIdx.x == 0) s_nd = 0;
  __syncthreads();
  const int lane = threadIdx.x & (T - 1);
  const int32_t nc = ctrl->nc;
  const int64_t S = ((int64_t)nc + nseg - 1) / nseg;
  const int64_t lo = (int64_t)seg * S;
  const int64_t hi = lo + S < nc ? lo + S : nc;
  for (int64_t cc = lo + threadIdx.x / T; cc < hi; cc += kBlock / T) {
    const int32_t c = (int32_t)cc;
    const int32_t m0 = cmem0[c], m1 = cmem1[c];
    const int64_t o = toff[c];
    const int32_t e0 = lv.xadj[m0], x0 = lv.xend[m0];
    const int32_t e1 = m1 >= 0 ? lv.xadj[m1] : 0, x1 = m1 >= 0 ? lv.xend[m1] : 0;
    const int L = (x0 - e0) + (x1 - e1);
    if (L > T) {
      if (lane == 0) defer[lo + atomicAdd(&s_nd, 1)] = c;
      continue;
    }
    CoarseRowLoader ld;
    ld.xadj = lv.xadj;
    ld.adj = lv.adj;
    ld.w = lv.w;
    ld.cmap = cmap;
    ld.c = c;
    ld.e0 = e0;
    ld.d0 = x0 - e0;
    ld.e1 = e1;
    const int k = team_row<T>(ld, L, okey + o, oval + o, &cnt[c]);
    if (lane == 0) {
      rin += L;
      rout += k;
    }
  }
  // per-block totals (no shared counter: device-wide atomics from every
  // block would serialize); summed only for the profiler (b_contract_sums)
  rin = block_sum<kBlock, int64_t>(rin, sml);
  rout = block_sum<kBlock, int64_t>(rout, sml);
  if (threadIdx.x == 0) {
    dcnt[seg] = s_nd;
    sio[2 * seg] = rin;
    sio[2 * seg + 1] = rout;
  }
}

// the short-row kernel's per-block totals into the control block (one block)
__device__ __forceinline__ void b_contract_sums(Ctrl* ctrl, const int32_t* dcnt,
                                                const int64_t* sio, int nseg) {
  __shared__ int64_t sml[kBlock / 64];
  int64_t d = 0, a = 0, b = 0;
  for (int i = threadIdx.x; i < nseg; i += kBlock) {
    d += dcnt[i];
    a += sio[2 * i];
    b += sio[2 * i + 1];
  }
  d = block_sum<kBlock, int64_t>(d, sml);
  a = block_sum<kBlock, int64_t>(a, sml);
  b = block_sum<kBlock, int64_t>(b, sml);
  if (threadIdx.x == 0) {
    ctrl->deferred = d;
    ctrl->short_in = a;
    ctrl->short_out = b;
  }
}

// exclusive scan of the coarse-tile entry counts; their total is 2m of the
// coarse level (one block)
// per-tile entry counts of the coarse rows from their final counts (one
// wave per tile of kTileC rows)
__device__ __forceinline__ void b_tile_count(const Ctrl* ctrl, const int32_t* cnt,
                                             int64_t* tile_cnt, int ntiles_c, int bid_,
                                             int nblk_) {
  static_assert(kTileC == 64, "one lane per row of a tile");
  const int32_t nc = ctrl->nc;
  for (int t = bid_ * (kBlock / 64) + (int)threadIdx.x / 64; t < ntiles_c;
       t += nblk_ * (kBlock / 64)) {
    const int32_t c = t * kTileC + lane_id();
    int64_t k = c < nc ? cnt[c] : 0;
    k = team_sum<64, int64_t>(k);
    if (lane_id() == 0) tile_cnt[t] = k;
  }
}

__device__ __forceinline__ void b_tile_scan(Ctrl* ctrl, int64_t* tile_cnt, int ntiles_c) {
  __shared__ int64_t sml[kBlock / 64];
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

__device__ __forceinline__ void b_contract_long(LevelView lv, const int32_t* cmap,
                                                          const int32_t* cmem0,
                                                          const int32_t* cmem1,
                                                          const int64_t* toff, Ctrl* ctrl,
                                                          int32_t* tmpk, int64_t* tmpv,
                                                          int32_t* cnt, int64_t* tile_cnt,
                                                          const int32_t* longlist,
                                                          int ntiles_c, unsigned char* lds,
                                                          bool staged, int bid_, int nblk_,
                                                          bool inline_tail = true,
                                                          bool huge = false) {
  // lds: kWin x (int64 + int32) bytes, and with `staged` another
  // kSortCap x (int64 + int32) bytes that hold a whole row
  int64_t* acc = (int64_t*)lds;
  int32_t* cc = (int32_t*)(acc + kWin);
  int64_t* stv = (int64_t*)(cc + kWin);
  int32_t* stk = (int32_t*)(stv + kSortCap);
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  // huge: the rows that the row kernel listed for one block each
  const int32_t nlong = huge ? ctrl->nhuge : ctrl->nlong;
  int64_t out_acc = 0;  // entries written (thread 0), one counter update per block
  for (int32_t i = bid_; i < nlong; i += nblk_) {
    const int32_t c = longlist[i];
    int L;
    CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
    bool dummy = false;
    int k;
    if (staged && L <= kSortCap) {
      // Gather the row into LDS once; when its coarse ids span few windows
      // the dense merge runs over the staged copy (one LDS pass per window),
      // otherwise the staged copy is sorted in place.
      int32_t kmin = INT_MAX, kmax = -1;
      for (int j = threadIdx.x; j < L; j += kBlock) {
        int32_t kk;
        int64_t vv;
        ld(j, kk, vv);
        stk[j] = kk;
        stv[j] = vv;
        if (kk != INT_MAX) {
          kmin = kk < kmin ? kk : kmin;
          kmax = kk > kmax ? kk : kmax;
        }
      }
      kmin = block_min<kBlock, int32_t>(kmin, smi);
      kmax = block_max<kBlock, int32_t>(kmax, smi);
      const StagedLoader sl{stk, stv};
      const int64_t nwin = kmax < 0 ? 0 : ((int64_t)kmax - kmin) / kWin + 1;
      if (nwin <= 16) {
        k = block_dense_emit<kBlock, true>(L, sl, acc, cc, smi, sml, tmpk + toff[c],
                                           tmpv + toff[c], &dummy);
      } else {
        k = block_sort_emit<kBlock, true>(L, sl, cc, acc, tmpk + toff[c], tmpv + toff[c],
                                          &dummy, smi);
      }
    } else if (L <= kSortCap) {
      // the LDS window doubles as the block sort's buffers
      k = block_sort_emit<kBlock, true>(L, ld, cc, acc, tmpk + toff[c], tmpv + toff[c], &dummy,
                                        smi);
    } else {
      k = block_dense_emit<kBlock, true>(L, ld, acc, cc, smi, sml, tmpk + toff[c],
                                         tmpv + toff[c], &dummy);
    }
    if (threadIdx.x == 0) {
      cnt[c] = k;
      if (tile_cnt) atomicAdd((unsigned long long*)&tile_cnt[c / kTileC], (unsigned long long)k);
      out_acc += k;
    }
  }
  if (threadIdx.x == 0 && out_acc)
    atomicAdd((unsigned long long*)(huge ? &ctrl->huge_out : &ctrl->long_out),
              (unsigned long long)out_acc);
  if (!inline_tail) return;
  __syncthreads();
  b_tile_scan(ctrl, tile_cnt, ntiles_c);
}

// One coarse row of 64 < L <= kLongCap candidates on a level with fewer
// than kPackMaxNc coarse vertices, by one wave.  Candidate j (a position in
// the concatenated member rows) becomes the key (coarse id << kPackIdBits) | j,
// unique within the row, or INT_MAX for the internal edge; the keys are
// sorted in the wave's LDS (sk: next_pow2(L) keys, at least 512 slots), and
// each run of one coarse id is summed by the lane that holds its head,
// reading the weights at the runs' positions.  Writes the row's distinct
// coarse neighbours to ok / ov and returns their count (in every lane).
__device__ __forceinline__ int wave_row_packed(const LevelView& lv, const int32_t* cmap,
                                               const CoarseRowLoader& ld, int32_t c, int L,
                                               int32_t* sk, int32_t* ok, int64_t* ov) {
  const int lane = lane_id();
  constexpr int32_t kPos = (1 << kPackIdBits) - 1;
  const int P2 = next_pow2(L);  // >= 128: L > 64
  const int32_t ebase = ld.d0 > 0 ? ld.e0 : ld.e1;  // an entry of the row (L > 0)
  // keys, eight candidates per lane in flight; every load is made, at a
  // valid index (slots past the row read an entry of it and are dropped), so
  // that none waits behind a branch
  for (int j0 = 0; j0 < P2; j0 += 512) {
    int32_t e[8], y[8], x[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int j = j0 + u * 64 + lane;
      e[u] = j < L ? (j < ld.d0 ? ld.e0 + j : ld.e1 + (j - ld.d0)) : ebase;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) y[u] = lv.adj[e[u]];
#pragma unroll
    for (int u = 0; u < 8; u++) x[u] = cmap[y[u]];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int j = j0 + u * 64 + lane;
      sk[j] = (j < L && x[u] != c) ? ((x[u] << kPackIdBits) | j) : INT_MAX;
    }
  }
  wave_sync();
  wave_sort_keys(sk, P2);
  // lane t owns the sorted slots [t * per, (t + 1) * per)
  const int per = P2 >> 6;
  const int s0 = lane * per;
  int heads = 0;
  for (int j = s0; j < s0 + per; j++) {
    const int32_t k = sk[j];
    if (k == INT_MAX) break;
    if (j == 0 || (sk[j - 1] >> kPackIdBits) != (k >> kPackIdBits)) heads++;
  }
  int incl = heads;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  int pos = incl - heads;  // output slot of this lane's first head
  // weights of the own slots, eight loads in flight; the sum of the slots
  // before the first head continues the run of an earlier lane
  int64_t lead = 0, acc = 0;
  int32_t cur = -1;
  bool seen_head = false;
  for (int j = s0; j < s0 + per; j += 8) {
    int32_t kk[8];
    int64_t ww[8];
#pragma unroll
    for (int u = 0; u < 8; u++) kk[u] = j + u < s0 + per ? sk[j + u] : INT_MAX;
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int32_t q = kk[u] != INT_MAX ? (kk[u] & kPos) : 0;
      const int32_t e = q < ld.d0 ? ld.e0 + q : ld.e1 + (q - ld.d0);
      ww[u] = lv.w[e];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      if (kk[u] == INT_MAX) continue;
      const int32_t cid = kk[u] >> kPackIdBits;
      const bool head = (j + u == 0) || (sk[j + u - 1] >> kPackIdBits) != cid;
      if (head) {
        if (seen_head) {
          ok[pos] = cur;
          ov[pos] = acc;
          pos++;
        }
        seen_head = true;
        cur = cid;
        acc = ww[u];
      } else if (seen_head) {
        acc += ww[u];
      } else {
        lead += ww[u];
      }
    }
  }
  // the last run of a lane may continue into the next lanes: add their lead
  // sums up to and including the first lane that holds a head
  const bool open = seen_head;
  const int empty = s0 >= L || sk[s0] == INT_MAX;  // holds no candidate
  bool more = true;
  for (int o = 1; o < 64; o++) {
    const int64_t l2 = __shfl_down(lead, o, 64);
    const int h2 = __shfl_down(heads, o, 64);
    const int e2 = __shfl_down(empty, o, 64);
    if (open && more && lane + o < 64 && !e2) {
      acc += l2;
      if (h2 > 0) more = false;
    } else {
      more = false;
    }
    if (!__any(open && more)) break;
  }
  if (seen_head) {
    ok[pos] = cur;
    ov[pos] = acc;
  }
  wave_sync();  // the keys are reused by the next row
  return total;
}

// Rows of kWaveCap < L <= kLongWave candidates on a level with fewer than
// kPackMaxNc coarse vertices: one wave per row (sk: the wave's kLongWave keys
// of LDS).
__device__ __forceinline__ void b_contract_longw(LevelView lv, const int32_t* cmap,
                                                 const int32_t* cmem0, const int32_t* cmem1,
                                                 const int64_t* toff, Ctrl* ctrl, int32_t* tmpk,
                                                 int64_t* tmpv, int32_t* cnt, int64_t* tile_cnt,
                                                 const int32_t* longlist, int32_t* sk, int wid,
                                                 int nw) {
  const int32_t nlong = ctrl->nlong;
  int64_t out_acc = 0;  // entries written (lane 0), one counter update per wave
  for (int32_t i = wid; i < nlong; i += nw) {
    const int32_t c = longlist[i];
    int L;
    const CoarseRowLoader ld = coarse_loader(lv, cmap, cmem0, cmem1, c, &L);
    const int total = wave_row_packed(lv, cmap, ld, c, L, sk, tmpk + toff[c], tmpv + toff[c]);
    if (lane_id() == 0) {
      cnt[c] = total;
      if (tile_cnt)
        atomicAdd((unsigned long long*)&tile_cnt[c / kTileC], (unsigned long long)total);
      out_acc += total;
    }
  }
  if (lane_id() == 0 && out_acc)
    atomicAdd((unsigned long long*)&ctrl->long_out, (unsigned long long)out_acc);
}

__device__ __forceinline__ void b_contract_compact(const Ctrl* ctrl,
                                                             const int64_t* toff,
                                                             const int32_t* cnt,
                                                             const int64_t* tile_base,
                                                             const int32_t* tmpk,
                                                             const int64_t* tmpv, int32_t* cxadj,
                                                             int32_t* cadj, int64_t* cw,
                                                             int ntiles_c, int bid_, int nblk_) {
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int32_t srow[kTileC + 1];
  const int32_t nc = ctrl->nc;
  for (int t = bid_; t < ntiles_c; t += nblk_) {
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
    // only the thread that owns row nc - 1 in this tile writes the end offset
    if (threadIdx.x < kTileC && c == nc - 1) cxadj[nc] = (int32_t)(base + ex + k);
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
  if (nc == 0 && bid_ == 0 && threadIdx.x == 0) cxadj[0] = 0;
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
  rc->moved_bs = 0;
}

// Called by every thread of one block once the pass totals are known.
template <int BS, class Items>
__device__ void decide_admission(RefCtl* rc, const Items& items, uint32_t ncand, int64_t cand_b,
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
    // ncand is the exact candidate count: small counts take the rank form
    if (mode == 0) {
      thr = select_prefix<BS>(items, gmin, idbits, tbits, 0, budget, sh, ncand);
    } else {
      const int64_t excess = rc->pw[s] - rc->maxw[s];
      // the covering prefix counts what the candidates take off side s
      const SrcItems<Items> src{items};
      u128 t1 = select_prefix<BS>(src, gmin, idbits, tbits, 1, excess, sh, ncand);
      u128 t2 = 0;
      if (cand_b > budget) t2 = select_prefix<BS>(items, gmin, idbits, tbits, 0, budget, sh, ncand);
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

// moved_bs: weight the pass took off side s, moved_b: weight it added to d
__device__ __forceinline__ void finish_pass(RefCtl* rc, int64_t moved_bs, int64_t moved_b,
                                            int64_t moved_n) {
  const int s = rc->s, d = 1 - s;
  rc->last_ncand = rc->ncand;
  rc->last_d = d;
  rc->last_moved_n = moved_n;
  rc->pw[s] -= moved_bs;
  rc->pw[d] += moved_b;
  rc->total_moves += moved_n;
  rc->last_cut = rc->ext_sum / 2;
  if (rc->mode == 1) rc->z = 0;
  else rc->z = moved_n == 0 ? rc->z + 1 : 0;
  rc->pass++;
  rc->done = (rc->z >= 2 || rc->pass >= rc->npass) ? 1 : 0;
  clear_pass_acc(rc);
}

__device__ __forceinline__ void refine_decide_common(int32_t n, RefCtl* rc, const Cand* list,
                                                     SelShared* sel, int mode, int s,
                                                     int64_t ext_acc, int64_t cb, int64_t gmn,
                                                     int64_t gmx);

template <int TW>
__device__ __forceinline__ void b_refine_gain(LevelView lv, const int8_t* part,
                                                        RefCtl* rc, Cand* list, SelShared* sel,
                                                        int64_t* partials, int bid_, int nblk_,
                                                        bool inline_tail = true,
                                                        int64_t* sext = nullptr,
                                                        int64_t* stot = nullptr,
                                                        const int64_t* b1 = nullptr) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  int mode, s;
  plan_pass(*rc, &mode, &s);
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
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
      const int32_t e1 = lv.xend[v];
      int32_t e = lv.xadj[v] + lane;
      // four entries per lane in flight: their neighbour and side loads
      // overlap instead of forming one dependent chain per entry
      for (; e + 3 * TW < e1; e += 4 * TW) {
        int32_t a[4];
        int64_t ww[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          a[q] = lv.adj[e + q * TW];
          ww[q] = lv.w[e + q * TW];
        }
        int8_t pq[4];
#pragma unroll
        for (int q = 0; q < 4; q++) pq[q] = part[a[q]];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          if (pq[q] != pv) ext += ww[q];
          else in += ww[q];
        }
      }
      for (; e < e1; e += TW) {
        const int64_t w = lv.w[e];
        if (part[lv.adj[e]] != pv) ext += w;
        else in += w;
      }
      ext = team_sum<TW>(ext);
      in = team_sum<TW>(in);
      if (lane == 0) {
        const int64_t gain = ext - in;
        ext_acc += ext;
        if (sext) {
          sext[v] = ext;
          stot[v] = ext + in;
        }
        cand = pv == s && (mode == 1 || gain > 0);
        if (cand) {
          // side 1 is measured in column b1 when one is given (time balance)
          const int64_t w0 = lv.b[v], w1 = b1 ? b1[v] : w0;
          c.gain = gain;
          c.b = s ? w0 : w1;
          c.bs = s ? w1 : w0;
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
  if (!inline_tail) {
    // per-block partials (4 x nblk int64), reduced by the decision launch
    if (threadIdx.x == 0) {
      partials[4 * bid_ + 0] = ext_acc;
      partials[4 * bid_ + 1] = cb;
      partials[4 * bid_ + 2] = gmn;
      partials[4 * bid_ + 3] = gmx;
    }
    return;
  }
  __syncthreads();
  refine_decide_common(lv.n, rc, list, sel, mode, s, ext_acc, cb, gmn, gmx);
}

// the pass totals are known: record them and choose the admitted prefix
__device__ __forceinline__ void refine_decide_common(int32_t n, RefCtl* rc, const Cand* list,
                                                     SelShared* sel, int mode, int s,
                                                     int64_t ext_acc, int64_t cb, int64_t gmn,
                                                     int64_t gmx) {
  if (threadIdx.x == 0) {
    rc->ext_sum = ext_acc;
    rc->cand_b = cb;
    rc->gmin_acc = gmn;
    rc->gmax_acc = gmx;
    rc->mode = mode;
    rc->s = s;
  }
  __syncthreads();
  const uint32_t ncand = rc->ncand;
  const ListItems items{list, ncand};
  decide_admission<kBlock>(rc, items, ncand, cb, gmn, gmx, n, sel);
}

// one block: reduce the gain launch's per-block partials, then decide
__device__ __forceinline__ void b_refine_decide(int32_t n, RefCtl* rc, const Cand* list,
                                                const int64_t* partials, int nparts,
                                                SelShared* sel) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  int mode, s;
  plan_pass(*rc, &mode, &s);
  int64_t ext_acc = 0, cb = 0, gmn = INT64_MAX, gmx = INT64_MIN;
  // four partials per thread in flight
  constexpr int U = 4;
  for (int i0 = threadIdx.x; i0 < nparts; i0 += U * kBlock) {
    int64_t q[U][4];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int i = i0 + u * kBlock;
#pragma unroll
      for (int k = 0; k < 4; k++) q[u][k] = i < nparts ? partials[4 * i + k] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (i0 + u * kBlock >= nparts) continue;
      ext_acc += q[u][0];
      cb += q[u][1];
      gmn = q[u][2] < gmn ? q[u][2] : gmn;
      gmx = q[u][3] > gmx ? q[u][3] : gmx;
    }
  }
  ext_acc = block_sum<kBlock, int64_t>(ext_acc, sml);
  cb = block_sum<kBlock, int64_t>(cb, sml);
  gmn = block_min<kBlock, int64_t>(gmn, sml);
  gmx = block_max<kBlock, int64_t>(gmx, sml);
  refine_decide_common(n, rc, list, sel, mode, s, ext_acc, cb, gmn, gmx);
}

// One block for a level of at most kSettleMax vertices: reduce the gain
// launch's partials, decide, move the admitted candidates and close the pass,
// all in the launch that follows the gain kernel (the candidate list holds at
// most n entries, so one block walks it quickly).
constexpr int32_t kSettleMax = 65536;

__device__ __forceinline__ void b_refine_settle(int32_t n, int8_t* part, RefCtl* rc,
                                                const Cand* list, const int64_t* partials,
                                                int nparts, SelShared* sel, int32_t* pass_out,
                                                int32_t* mark = nullptr) {
  __shared__ int64_t sms[kBlock / 64];
  if (rc->done) return;
  b_refine_decide(n, rc, list, partials, nparts, sel);
  __syncthreads();
  const RefCtl r = *rc;
  const int d = 1 - r.s;
  int64_t mb = 0, mbs = 0, mn = 0;
  if (r.admit != kAdmitNone) {
    const int64_t nc = r.ncand;
    constexpr int U = 4;  // candidate loads in flight per thread
    for (int64_t i0 = threadIdx.x; i0 < nc; i0 += (int64_t)U * kBlock) {
      Cand c[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (i < nc) c[u] = list[i];
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (i < nc && admitted(r, c[u])) {
          part[c[u].v] = (int8_t)d;
          if (mark) mark[c[u].v] = r.pass + 1;
          mb += c[u].b;
          mbs += c[u].bs;
          mn++;
        }
      }
    }
  }
  mb = block_sum<kBlock, int64_t>(mb, sms);
  mbs = block_sum<kBlock, int64_t>(mbs, sms);
  mn = block_sum<kBlock, int64_t>(mn, sms);
  if (threadIdx.x == 0) {
    finish_pass(rc, mbs, mb, mn);
    *pass_out = rc->pass;
  }
}

__device__ __forceinline__ void b_refine_finish(RefCtl* rc, int32_t* pass_out) {
  if (rc->done) return;
  if (threadIdx.x == 0) {
    finish_pass(rc, rc->moved_bs, rc->moved_b, rc->moved_n);
    *pass_out = rc->pass;
  }
}

__device__ __forceinline__ void b_refine_apply(int8_t* part, RefCtl* rc,
                                                         const Cand* list, int32_t* pass_out, int bid_, int nblk_,
                                                         bool inline_tail = true,
                                                         int32_t* mark = nullptr) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  const RefCtl r = *rc;
  const int d = 1 - r.s;
  int64_t mb = 0, mbs = 0, mn = 0;
  for (int64_t i = (int64_t)bid_ * kBlock + threadIdx.x; i < r.ncand;
       i += (int64_t)nblk_ * kBlock) {
    const Cand c = list[i];
    if (admitted(r, c)) {
      part[c.v] = (int8_t)d;
      if (mark) mark[c.v] = r.pass + 1;
      mb += c.b;
      mbs += c.bs;
      mn++;
    }
  }
  mb = block_sum<kBlock, int64_t>(mb, sml);
  mbs = block_sum<kBlock, int64_t>(mbs, sml);
  mn = block_sum<kBlock, int64_t>(mn, sml);
  if (threadIdx.x == 0 && (mb || mn)) {
    atomicAdd((unsigned long long*)&rc->moved_b, (unsigned long long)mb);
    atomicAdd((unsigned long long*)&rc->moved_bs, (unsigned long long)mbs);
    atomicAdd((unsigned long long*)&rc->moved_n, (unsigned long long)mn);
  }
  if (!inline_tail) return;
  __syncthreads();
  b_refine_finish(rc, pass_out);
}

__device__ __forceinline__ void start_level(RefCtl* rc, int npass) {
  rc->pass = 0;
  rc->z = 0;
  rc->npass = npass;
  rc->done = npass <= 0 ? 1 : 0;
  rc->total_moves = 0;
  clear_pass_acc(rc);
}

__device__ __forceinline__ void b_project(int32_t n, const int32_t* cmap,
                                                    const int8_t* cpart, int8_t* part, RefCtl* rc,
                                                    int npass, int bid_, int nblk_,
                                                    int32_t* mark = nullptr) {
  for (int64_t u = (int64_t)bid_ * kBlock + threadIdx.x; u < n;
       u += (int64_t)nblk_ * kBlock) {
    part[u] = cpart[cmap[u]];
    if (mark) mark[u] = 0;
  }
  if (bid_ == 0 && threadIdx.x == 0) start_level(rc, npass);
}

__device__ __forceinline__ void b_start_level(RefCtl* rc, int npass, int bid_, int nblk_) {
  if (threadIdx.x == 0) start_level(rc, npass);
}

// Later passes of a level read the per-vertex external weight and total
// incident weight kept in sext / stot (internal = total - external) instead
// of the rows: one vertex per thread, the same candidates and per-block
// partials as the gain kernel.
__device__ __forceinline__ void b_refine_scan(int32_t n, const int8_t* part, const int64_t* b,
                                              const int64_t* b1, const int64_t* sext,
                                              const int64_t* stot, RefCtl* rc, Cand* list,
                                              int64_t* partials, int bid_, int nblk_) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  int mode, s;
  plan_pass(*rc, &mode, &s);
  int64_t ext_acc = 0, cb = 0, gmn = INT64_MAX, gmx = INT64_MIN;
  const int64_t stride = (int64_t)nblk_ * kBlock;
  // every thread runs the same number of iterations for the wave ballot
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t v = (int64_t)bid_ * kBlock + threadIdx.x + it * stride;
    bool cand = false;
    Cand c;
    c.pad = 0;
    if (v < n) {
      const int8_t pv = part[v];
      const int64_t ext = sext[v], in = stot[v] - ext, w0 = b[v], w1 = b1 ? b1[v] : w0;
      const int64_t gain = ext - in;
      ext_acc += ext;
      cand = pv == s && (mode == 1 || gain > 0);
      if (cand) {
        c.gain = gain;
        c.b = s ? w0 : w1;
        c.bs = s ? w1 : w0;
        c.v = (int32_t)v;
        cb += c.b;
        gmn = gain < gmn ? gain : gmn;
        gmx = gain > gmx ? gain : gmx;
      }
    }
    append_cand(cand, c, list, &rc->ncand);
  }
  ext_acc = block_sum<kBlock, int64_t>(ext_acc, sml);
  cb = block_sum<kBlock, int64_t>(cb, sml);
  gmn = block_min<kBlock, int64_t>(gmn, sml);
  gmx = block_max<kBlock, int64_t>(gmx, sml);
  if (threadIdx.x == 0) {
    partials[4 * bid_ + 0] = ext_acc;
    partials[4 * bid_ + 1] = cb;
    partials[4 * bid_ + 2] = gmn;
    partials[4 * bid_ + 3] = gmx;
  }
}

// After pass p moved the vertices marked p + 1 (all from one side to d):
// every unmoved neighbour x of a moved vertex u sees the edge change sides
// (internal <-> external: one exact integer atomic on its external weight,
// so the order does not matter; its total does not change); a moved u
// swaps its external and internal weights, except for the edges to other
// moved vertices, which stay internal.  One team per listed candidate;
// unmoved candidates are skipped.
template <int TW>
__device__ __forceinline__ void b_refine_delta(LevelView lv, const int8_t* part,
                                               const int32_t* mark, int64_t* sext,
                                               const int64_t* stot, const RefCtl* rc,
                                               const Cand* list, int p, int bid_, int nblk_) {
  // pass p did not run, moved nothing, or was the level's last
  if (rc->pass != p + 1 || rc->last_moved_n == 0 || rc->done) return;
  const uint32_t nlist = rc->last_ncand;
  const int d = rc->last_d;
  const int32_t stamp = p + 1;
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t i = team; i < nlist; i += nteams) {
    const int32_t u = list[i].v;
    if (mark[u] != stamp) continue;  // the whole team skips together
    int64_t corr = 0;
    const int32_t e1 = lv.xend[u];
    for (int32_t e = lv.xadj[u] + lane; e < e1; e += TW) {
      const int32_t x = lv.adj[e];
      const int64_t w = lv.w[e];
      if (mark[x] == stamp) {
        corr += w;
      } else {
        atomicAdd((unsigned long long*)&sext[x], (unsigned long long)(part[x] == d ? -w : w));
      }
    }
    corr = team_sum<TW>(corr);
    if (lane == 0) {
      sext[u] = stot[u] - sext[u] - corr;  // the old internal weight, less corr
    }
  }
}

// ------------------------------------------------------ communication volume
// The ids of the input graph are a topological order, so the successors of
// v are its neighbours with larger ids.  v's output is as large as its
// largest edge to a successor, out(v), and crosses to the other side once
// when any successor lies there; the volume is the sum of the outputs that
// cross.

// out(v) for every vertex (one team per row)
template <int TW>
__device__ __forceinline__ void b_vol_out(LevelView lv, int64_t* out, int bid_, int nblk_) {
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t vv = team; vv < lv.n; vv += nteams) {
    const int32_t v = (int32_t)vv;
    int64_t m = 0;
    for (int32_t e = lv.xadj[v] + lane; e < lv.xend[v]; e += TW)
      if (lv.adj[e] > v && lv.w[e] > m) m = lv.w[e];
    m = team_max<TW, int64_t>(m);
    if (lane == 0) out[v] = m;
  }
}

// successors of v on the other side of v
template <int TW>
__device__ __forceinline__ void b_vol_count(LevelView lv, const int8_t* part, int32_t* cnt,
                                            int bid_, int nblk_) {
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t vv = team; vv < lv.n; vv += nteams) {
    const int32_t v = (int32_t)vv;
    const int8_t pv = part[v];
    int32_t c = 0;
    for (int32_t e = lv.xadj[v] + lane; e < lv.xend[v]; e += TW) {
      const int32_t x = lv.adj[e];
      c += x > v && part[x] != pv;
    }
    c = team_sum<TW, int32_t>(c);
    if (lane == 0) cnt[v] = c;
  }
}

// A volume pass's candidates: the gain of moving v from its side s to d at
// the pass's start is out(v) ([a successor on d] - [a successor on s]), plus
// out(u) for each predecessor u on d whose only successor on the other side
// is v, minus out(u) for each predecessor u on s with no successor on the
// other side.  Same list, partials and pass plan as the gain kernel.
template <int TW>
__device__ __forceinline__ void b_vol_gain(LevelView lv, const int8_t* part, const int64_t* out,
                                           const int32_t* cnt, RefCtl* rc, Cand* list,
                                           int64_t* partials, int bid_, int nblk_) {
  __shared__ int64_t sml[kBlock / 64];
  if (rc->done) return;
  int mode, s;
  plan_pass(*rc, &mode, &s);
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  int64_t ext_acc = 0, cb = 0, gmn = INT64_MAX, gmx = INT64_MIN;
  const int64_t iters = (lv.n + nteams - 1) / nteams;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t uu = team + it * nteams;
    bool cand = false;
    Cand c;
    c.pad = 0;
    if (uu < lv.n) {
      const int32_t v = (int32_t)uu;
      const int8_t pv = part[v];
      int64_t ext = 0, pred = 0;
      int32_t succ_s = 0, succ_d = 0;
      for (int32_t e = lv.xadj[v] + lane; e < lv.xend[v]; e += TW) {
        const int32_t x = lv.adj[e];
        const int8_t px = part[x];
        if (px != pv) ext += lv.w[e];
        if (x > v) {
          if (px == pv) succ_s++;
          else succ_d++;
        } else {
          const int32_t cx = cnt[x];
          if (px != pv && cx == 1) pred += out[x];
          if (px == pv && cx == 0) pred -= out[x];
        }
      }
      ext = team_sum<TW>(ext);
      pred = team_sum<TW>(pred);
      succ_s = team_sum<TW, int32_t>(succ_s);
      succ_d = team_sum<TW, int32_t>(succ_d);
      if (lane == 0) {
        const int64_t gain = pred + out[v] * ((succ_d > 0 ? 1 : 0) - (succ_s > 0 ? 1 : 0));
        ext_acc += ext;
        cand = pv == s && (mode == 1 || gain > 0);
        if (cand) {
          c.gain = gain;
          c.b = lv.b[v];
          c.bs = c.b;
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
    partials[4 * bid_ + 0] = ext_acc;
    partials[4 * bid_ + 1] = cb;
    partials[4 * bid_ + 2] = gmn;
    partials[4 * bid_ + 3] = gmx;
  }
}

// the volume of the current assignment, added to *vol (integer atomics)
template <int TW>
__device__ __forceinline__ void b_vol_total(LevelView lv, const int8_t* part, const int64_t* out,
                                            int64_t* vol, int bid_, int nblk_) {
  __shared__ int64_t sml[kBlock / 64];
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  int64_t acc = 0;
  const int64_t iters = (lv.n + nteams - 1) / nteams;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t vv = team + it * nteams;
    int32_t c = 0;
    if (vv < lv.n) {
      const int32_t v = (int32_t)vv;
      const int8_t pv = part[v];
      for (int32_t e = lv.xadj[v] + lane; e < lv.xend[v]; e += TW) {
        const int32_t x = lv.adj[e];
        c += x > v && part[x] != pv;
      }
    }
    c = team_sum<TW, int32_t>(c);
    if (lane == 0 && vv < lv.n && c > 0) acc += out[vv];
  }
  acc = block_sum<kBlock, int64_t>(acc, sml);
  if (threadIdx.x == 0 && acc) atomicAdd((unsigned long long*)vol, (unsigned long long)acc);
}

// cut (as sum of ext), loads and times of the final assignment
template <int TW>
__device__ __forceinline__ void b_final_stats(LevelView lv, const int64_t* vc,
                                                        const int64_t* vg, const int8_t* part,
                                                        Ctrl* ctrl, int bid_, int nblk_,
                                                        int64_t* partials = nullptr) {
  __shared__ int64_t sml[kBlock / 64];
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  int64_t ext_acc = 0, l0 = 0, l1 = 0, t0 = 0, t1 = 0;
  for (int64_t uu = team; uu < lv.n; uu += nteams) {
    const int32_t v = (int32_t)uu;
    const int8_t pv = part[v];
    int64_t ext = 0;
    for (int32_t e = lv.xadj[v] + lane; e < lv.xend[v]; e += TW)
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
    if (partials) {  // per-block partials, summed by b_final_reduce
      partials[5 * bid_ + 0] = ext_acc;
      partials[5 * bid_ + 1] = l0;
      partials[5 * bid_ + 2] = l1;
      partials[5 * bid_ + 3] = t0;
      partials[5 * bid_ + 4] = t1;
    } else {
      atomicAdd((unsigned long long*)&ctrl->res_ext, (unsigned long long)ext_acc);
      atomicAdd((unsigned long long*)&ctrl->res_load[0], (unsigned long long)l0);
      atomicAdd((unsigned long long*)&ctrl->res_load[1], (unsigned long long)l1);
      atomicAdd((unsigned long long*)&ctrl->res_time[0], (unsigned long long)t0);
      atomicAdd((unsigned long long*)&ctrl->res_time[1], (unsigned long long)t1);
    }
  }
}

// one block: totals of b_final_stats' per-block partials
__device__ __forceinline__ void b_final_reduce(Ctrl* ctrl, const int64_t* partials, int nparts) {
  __shared__ int64_t sml[kBlock / 64];
  int64_t v[5] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nparts; i += kBlock)
    for (int q = 0; q < 5; q++) v[q] += partials[5 * i + q];
  for (int q = 0; q < 5; q++) v[q] = block_sum<kBlock, int64_t>(v[q], sml);
  if (threadIdx.x == 0) {
    ctrl->res_ext = v[0];
    ctrl->res_load[0] = v[1];
    ctrl->res_load[1] = v[2];
    ctrl->res_time[0] = v[3];
    ctrl->res_time[1] = v[4];
  }
}

__device__ __forceinline__ void b_clear_stats(Ctrl* ctrl, int bid_, int nblk_) {
  if (threadIdx.x == 0) {
    ctrl->res_ext = 0;
    ctrl->res_load[0] = ctrl->res_load[1] = 0;
    ctrl->res_time[0] = ctrl->res_time[1] = 0;
  }
}

// ------------------------------------------------------- initial bisection
// tot[v] = sum of v's incident weights; one kInitTotTeam-lane team per row
constexpr int kInitTotTeam = 16;

__device__ __forceinline__ void b_init_tot(LevelView lv, int64_t* tot, int bid_, int nblk_) {
  constexpr int TW = kInitTotTeam;
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)nblk_ * kBlock / TW;
  for (int64_t v = team; v < lv.n; v += nteams) {
    int64_t s = 0;
    const int32_t e1 = lv.xend[v];
    for (int32_t e = lv.xadj[v] + lane; e < e1; e += TW) s += lv.w[e];
    s = team_sum<TW>(s);
    if (lane == 0) tot[v] = s;
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
  butterfly<64>([&](auto o) {
    GrowBest o2;
    o2.a = xor_lane<decltype(o)::value>(b.a);
    o2.g = xor_lane<decltype(o)::value>(b.g);
    o2.v = xor_lane<decltype(o)::value>(b.v);
    if (grow_better(o2, b)) b = o2;
  });
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
        for (int32_t e = lv.xadj[v]; e < lv.xend[v]; e++) {
          if (part[lv.adj[e]] != pv) ext += lv.w[e];
          else in += lv.w[e];
        }
        const int64_t gain = ext - in;
        ext_acc += ext;
        cand = pv == s && (mode == 1 || gain > 0);
        if (cand) {
          c.gain = gain;
          c.b = lv.b[v];
          c.bs = c.b;
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
    const ListItems items{list, ncand};
    decide_admission<BS>(rc, items, ncand, cb, gmn, gmx, lv.n, sel);
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
    if (threadIdx.x == 0) finish_pass(rc, mb, mb, mn);
  }
}

// One block per trial: greedy growing, then refinement, then its cut.  The
// last block to finish keeps the first trial minimal in (infeasible, cut).
// keeps the first trial minimal in (infeasible, cut): its loads go to
// ctrl->ref, its assignment to out_part
template <int BS>
__device__ void b_trial_pick(int K, int32_t n, Ctrl* ctrl, const RefCtl* tctl,
                             const int8_t* tpart, const int64_t* tres, int8_t* out_part) {
  __shared__ int s_best;
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < K; i++) {
      const int64_t ci = tres[2 * i], ii = tres[2 * i + 1];
      const int64_t cbst = tres[2 * best], ib = tres[2 * best + 1];
      if (ii < ib || (ii == ib && ci < cbst)) best = i;
    }
    s_best = best;
    ctrl->ref.pw[0] = tctl[best].pw[0];
    ctrl->ref.pw[1] = tctl[best].pw[1];
    ctrl->ref.last_cut = tres[2 * best];
  }
  __syncthreads();
  const int8_t* bp = tpart + (int64_t)s_best * n;
  for (int32_t v = threadIdx.x; v < n; v += BS) out_part[v] = bp[v];
  __syncthreads();
}

template <int BS>
// Trial t of K with its state in global memory (coarsest graphs too large
// for LDS); writes cut, infeasibility, loads and assignment of the trial.
__device__ void b_trial_global(LevelView lv, const int64_t* tot, int K, int t, int gs, int npass,
                               const Ctrl* ctrl, RefCtl* tctl, int8_t* tpart, int64_t* tconn,
                               int32_t* tadj, Cand* tlist, int64_t* tres, SelShared* selp) {
  __shared__ int64_t sml[BS / 64];
  __shared__ GrowBest sgb[BS / 64];
  __shared__ uint32_t s_ncand;
  SelShared& sel = *selp;
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
    for (int32_t e = lv.xadj[pick] + threadIdx.x; e < lv.xend[pick]; e += BS) {
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
    for (int32_t e = lv.xadj[v]; e < lv.xend[v]; e++)
      if (part[lv.adj[e]] != pv) ext += lv.w[e];
  }
  ext = block_sum<BS, int64_t>(ext, sml);
  if (threadIdx.x == 0) {
    tres[2 * t] = ext / 2;
    tres[2 * t + 1] = (rc->pw[0] > rc->maxw[0] || rc->pw[1] > rc->maxw[1]) ? 1 : 0;
  }
  __syncthreads();
}

// LDS-resident trials (coarsest graphs of at most kTrialLdsMax vertices):
// one block of BS threads per trial.  Gains are kept up to date instead of
// recomputed: when a set M of vertices changes side (all from one side to
// the other), gain(x) flips sign for x in M, and every neighbour y of a moved
// vertex gains -2w when it ends on the mover's new side, +2w otherwise.  This
// yields the same integers as recomputing ext - int from scratch.
constexpr int kTrialBlock = 256;
constexpr int kTrialLdsMax = 3072;
constexpr int kTrialLongDeg = 128;  // mean row length above which picks read rows block-wide

// gain, b (int64), xadj (int32, n + 1), side, adjacency, move flag (int8),
// plus one dirty flag per thread of the block
__host__ __device__ constexpr size_t trial_lds_bytes(int32_t n, int bs) {
  return (size_t)n * 23 + 4 + (size_t)bs + 16;
}

// Refinement passes on an LDS-resident state (gain, balance weight, side,
// move flag per vertex); gains are updated incrementally (see above).
template <int BS>
__device__ void lds_refine(const LevelView& lv, int64_t* s_gain, const int64_t* s_b,
                           int8_t* s_part, int8_t* s_mv, RefCtl& srf, SelShared& sel) {
  const int32_t n = lv.n;
  __shared__ int64_t sm4[4 * (BS / 64)];
  constexpr int kChunk = 16, kChunkCap = 512;
  __shared__ int32_t s_chunk_v[kChunkCap], s_chunk_e[kChunkCap];
  __shared__ int s_nchunk;
  for (;;) {
    if (srf.done) break;
    if (threadIdx.x == 0) s_nchunk = 0;
    int mode, s;
    plan_pass(srf, &mode, &s);
    const LdsItems items{s_gain, s_b, s_part, n, s, mode};
    int64_t cb = 0, cnt = 0, gmn = INT64_MAX, gmx = INT64_MIN;
    for (int32_t v = threadIdx.x; v < n; v += BS) {
      Cand c;
      if (!items.get(v, c)) continue;
      cb += c.b;
      cnt++;
      gmn = c.gain < gmn ? c.gain : gmn;
      gmx = c.gain > gmx ? c.gain : gmx;
    }
    block_sum_sum_min_max<BS>(cb, cnt, gmn, gmx, sm4);
    if (threadIdx.x == 0) {
      srf.mode = mode;
      srf.s = s;
    }
    __syncthreads();
    decide_admission<BS>(&srf, items, (uint32_t)cnt, cb, gmn, gmx, n, &sel);
    __syncthreads();
    // admitted vertices change side (each thread only touches its own) and
    // queue their rows as chunks of kChunk entries
    const int d = 1 - s;
    int64_t mb = 0, mn = 0;
    for (int32_t v = threadIdx.x; v < n; v += BS) {
      Cand c;
      if (items.get(v, c) && admitted(srf, c)) {
        s_mv[v] = 1;
        s_part[v] = (int8_t)d;
        s_gain[v] = -c.gain;
        mb += c.b;
        mn++;
        const int32_t a = lv.xadj[v], nc = (lv.xend[v] - a + kChunk - 1) / kChunk;
        const int slot = atomicAdd(&s_nchunk, nc);
        for (int k = 0; k < nc && slot + k < kChunkCap; k++) {
          s_chunk_v[slot + k] = v;
          s_chunk_e[slot + k] = a + k * kChunk;
        }
      }
    }
    __syncthreads();
    const int nchunk = s_nchunk;
    if (nchunk <= kChunkCap) {
      // every thread takes whole chunks, kChunk loads in flight: the rows of
      // all moved vertices cost about one global round trip together
      for (int c = threadIdx.x; c < nchunk; c += BS) {
        const int32_t v = s_chunk_v[c], e = s_chunk_e[c];
        const int32_t e1 = lv.xend[v];
        int32_t y[kChunk];
        int64_t w[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; u++) {
          y[u] = e + u < e1 ? lv.adj[e + u] : 0;
          w[u] = e + u < e1 ? lv.w[e + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < kChunk; u++)
          if (e + u < e1)
            atomicAdd((unsigned long long*)&s_gain[y[u]],
                      (unsigned long long)(s_part[y[u]] == d ? -2 * w[u] : 2 * w[u]));
        if (e == lv.xadj[v]) s_mv[v] = 0;
      }
    }
    // otherwise (a long queue): wave k takes the moved vertices among ids
    // [64 j, 64 j + 64) for j = k mod (BS / 64) and walks each of their rows
    // with all 64 lanes, U entries per lane in flight (long rows of dense
    // coarse graphs cost a few round trips each, not one per U entries)
    if (nchunk > kChunkCap) {
      constexpr int U = 8;
      for (int32_t b0 = (int32_t)(threadIdx.x & ~63u); b0 < n; b0 += BS) {
        const int32_t v = b0 + lane_id();
        const bool mine = v < n && s_mv[v] != 0;
        uint64_t m = __ballot(mine);
        while (m) {
          const int32_t u = b0 + __builtin_ctzll(m);
          m &= m - 1;
          const int32_t e1 = lv.xend[u];
          for (int32_t e = lv.xadj[u] + lane_id(); e < e1; e += 64 * U) {
            int32_t y[U];
            int64_t w[U];
#pragma unroll
            for (int k = 0; k < U; k++) {
              const int32_t q = e + 64 * k;
              y[k] = q < e1 ? lv.adj[q] : 0;
              w[k] = q < e1 ? lv.w[q] : 0;
            }
#pragma unroll
            for (int k = 0; k < U; k++)
              if (e + 64 * k < e1)
                atomicAdd((unsigned long long*)&s_gain[y[k]],
                          (unsigned long long)(s_part[y[k]] == d ? -2 * w[k] : 2 * w[k]));
          }
        }
        if (mine) s_mv[v] = 0;
      }
    }
    int64_t unused_min = 0, unused_max = 0;
    block_sum_sum_min_max<BS>(mb, mn, unused_min, unused_max, sm4);
    if (threadIdx.x == 0) finish_pass(&srf, mb, mb, mn);
    __syncthreads();
  }
}

// Trial t of K on an LDS-resident copy of the coarsest graph; writes its
// cut, infeasibility, loads and assignment to tres / tctl / tpart.
// lds: trial_lds_bytes(n) bytes; sel, srf: block-shared scratch.
template <int BS, bool kLongRows = false>
__device__ void b_trial_lds(LevelView lv, const int64_t* tot, int K, int t, int gs, int npass,
                            const Ctrl* ctrl, RefCtl* tctl, int8_t* tpart, int64_t* tres,
                            unsigned char* lds, SelShared* selp, RefCtl* srfp) {
  const int32_t n = lv.n;
  int64_t* s_gain = (int64_t*)lds;
  int64_t* s_b = s_gain + n;
  int32_t* s_xadj = (int32_t*)(s_b + n);
  int8_t* s_part = (int8_t*)(s_xadj + n + 1);
  int8_t* s_adj = s_part + n;
  int8_t* s_mv = s_adj + n;
  uint8_t* s_dirty = (uint8_t*)(s_mv + n);  // BS flags: thread's own vertices changed
  __shared__ int64_t sml[BS / 64];
  __shared__ GrowBest sgb[BS / 64];
  SelShared& sel = *selp;
  RefCtl& srf = *srfp;
  const int gb = 1 - gs;
  int64_t W = 0;
  for (int32_t v = threadIdx.x; v < n; v += BS) {
    s_gain[v] = -tot[v];
    const int64_t bv = lv.b[v];
    s_b[v] = bv;
    s_part[v] = (int8_t)gb;
    s_adj[v] = 0;
    s_mv[v] = 0;
    W += bv;
  }
  // the coarsest level is compact: n + 1 offsets
  for (int32_t v = threadIdx.x; v <= n; v += BS) s_xadj[v] = lv.xadj[v];
  s_dirty[threadIdx.x] = 0;
  W = block_sum<BS, int64_t>(W, sml);
  const int64_t tg = ctrl->tgt[gs], mg = ctrl->ref.maxw[gs];
  const int32_t seedv = (int32_t)(((int64_t)t * n) / K);
  // Greedy growing of side gs, one vertex at a time.  Thread t owns the
  // vertices v = t mod BS and keeps the best of those that can still be
  // added; it rescans them only when one of them changed (the pick or a
  // neighbour of it) or its best stopped fitting.  The room mg - pg only
  // shrinks, so a vertex that does not fit never fits again, and a best that
  // still fits stays the best of the owner's fitting vertices.
  //
  // Fast form: |gain(v)| <= tot(v), so when every tot is below 2^61 the pair
  // (adjacent, gain) packs into one ordered 63-bit key (adjacent << 62) |
  // (gain + 2^61), held in s_gain while growing, and the order (adjacent
  // desc, gain desc, id asc) becomes one unsigned compare plus the id.
  int64_t tmax = 0;
  for (int32_t v = threadIdx.x; v < n; v += BS) tmax = tot[v] > tmax ? tot[v] : tmax;
  tmax = block_max<BS, int64_t>(tmax, sml);
  const bool packed = tmax < ((int64_t)1 << 61);
  const uint64_t kBias = 1ull << 61, kAdj = 1ull << 62, kField = (1ull << 62) - 1;
  const uint64_t kSide = 1ull << 63;
  int64_t pg = 0;
  // Compact form (incident weights below 2^49, at most 4,096 vertices): the
  // whole order fits one 63-bit key, (adjacent << 62) | ((gain + 2^49) << 12)
  // | (4095 - id), so the best is a plain unsigned maximum.  While a vertex of
  // side gb is not picked its key only grows (a picked neighbour adds 2w to
  // its gain and sets the adjacency bit), so each update is offered to the
  // owner's best with an LDS atomicMax, and an owner rescans only when its
  // best was picked or stopped fitting.
  const bool compact = tmax < ((int64_t)1 << 49) && n <= 4096;
  if (compact) {
    uint64_t* s_key = (uint64_t*)s_gain;
    __shared__ uint64_t s_best[BS];
    __shared__ uint64_t s_wmax[BS / 64];
    const uint64_t cBias = 1ull << 49, cAdj = 1ull << 62, cSide = 1ull << 63;
    const uint64_t cField = ((1ull << 50) - 1) << 12;
    for (int32_t v = threadIdx.x; v < n; v += BS)
      s_key[v] = ((uint64_t)(s_gain[v] + (int64_t)cBias) << 12) | (uint64_t)(4095 - v);
    __syncthreads();
    auto vid = [](uint64_t k) { return (int32_t)(4095 - (int32_t)(k & 4095)); };
    // Best fitting key among the vertices of owner thread `own` (v = own mod
    // BS), leaving out `skip`.  All slot loads are issued before any test,
    // and the tests combine with bitwise operators, so a rescan costs one
    // LDS round trip rather than a dependent load-and-branch per slot.
    auto rescan_slots = [&](auto slots, int own, int64_t room, int32_t skip) {
      constexpr int S = decltype(slots)::value;
      uint64_t kv[S];
      int64_t bw[S];
#pragma unroll
      for (int q = 0; q < S; q++) {
        const int32_t v = own + q * BS;
        const int32_t vv = v < n ? v : 0;
        kv[q] = s_key[vv];
        bw[q] = s_b[vv];
      }
      uint64_t bk = 0;
#pragma unroll
      for (int q = 0; q < S; q++) {
        const int32_t v = own + q * BS;
        const bool ok = (v < n) & (v != skip) & ((kv[q] >> 63) == 0) & (bw[q] <= room);
        const uint64_t k = ok ? kv[q] : 0;
        bk = k > bk ? k : bk;
      }
      return bk;
    };
    static_assert(kTrialLdsMax <= 12 * BS, "slot classes cover the LDS-resident sizes");
    auto rescan = [&](int own, int64_t room, int32_t skip) {
      if (n <= 4 * BS) return rescan_slots(LaneXor<4>{}, own, room, skip);
      if (n <= 8 * BS) return rescan_slots(LaneXor<8>{}, own, room, skip);
      return rescan_slots(LaneXor<12>{}, own, room, skip);
    };
    // s_best[t]: thread t's best, written by t at the loop top or, for the
    // owner of the pick, by a rescanning lane of another wave while the
    // update runs.  s_raise[t]: keys raised by the update (LDS atomicMax),
    // folded into the best and cleared by t at the loop top.
    __shared__ uint64_t s_raise[BS];
    s_best[threadIdx.x] = rescan((int)threadIdx.x, mg, -1);
    s_raise[threadIdx.x] = 0;
    __syncthreads();
    bool first = true;
    const bool seed_fits = s_b[seedv] <= mg;  // the first pick is the seed when it fits
    const int seed_wave = (seedv % BS) / 64;
    uint64_t seen = 0;     // the best as of its last fit check
    int64_t seen_b = 0;    // and that vertex's balance weight
    // this thread's best fitting key after the last update (raises folded in)
    auto own_best = [&](int64_t room) {
      uint64_t bk = s_best[threadIdx.x];
      const uint64_t rz = s_raise[threadIdx.x];
      if (rz) {
        s_raise[threadIdx.x] = 0;
        bk = rz > bk ? rz : bk;
      }
      if (bk != 0) {
        // keys of unpicked vertices only grow and the room only shrinks, so
        // the best needs a rescan only when its own weight stops fitting
        if (bk != seen) {
          seen = bk;
          seen_b = s_b[vid(bk)];
        }
        if (seen_b > room) {
          bk = rescan((int)threadIdx.x, room, -1);
          seen = bk;
          seen_b = bk ? s_b[vid(bk)] : 0;
        }
      }
      s_best[threadIdx.x] = bk;
      butterfly<64>([&](auto o) {
        const uint64_t k2 = xor_lane<decltype(o)::value>(bk);
        bk = k2 > bk ? k2 : bk;
      });
      return bk;  // the wave's best
    };
    // the block's pick from the waves' bests (after the barrier that
    // publishes them); -1 when nothing fits
    auto block_pick = [&]() {
      uint64_t gk = s_wmax[0];
#pragma unroll
      for (int w = 1; w < BS / 64; w++) gk = s_wmax[w] > gk ? s_wmax[w] : gk;
      int32_t pick = gk ? vid(gk) : -1;
      if (first && seed_fits) pick = seedv;
      first = false;
      return pick;
    };
    // the pick's owner gets a new best from 16 lanes of the next wave (one
    // slot each, then a 16-lane maximum), in parallel with the update; a key
    // read before the update raised it reaches s_raise as well
    auto rescan_owner = [&](int32_t pick, int64_t room_next) {
      const int wave = (int)threadIdx.x / 64;
      const int own = pick % BS;
      static_assert(kTrialLdsMax <= 16 * BS, "one rescanning lane per slot");
      if (wave == ((own + 64) % BS) / 64 && lane_id() < 16) {
        const int32_t v = own + lane_id() * BS;
        uint64_t k = 0;
        if (v < n && v != pick) {
          const uint64_t kv = s_key[v];
          const int64_t bv = s_b[v];
          k = ((kv >> 63) == 0 && bv <= room_next) ? kv : 0;
        }
        k = team_max<16>(k);
        if (lane_id() == 0) s_best[own] = k;
      }
    };
    // the pick changes side: its gain field negated, the adjacency bit kept
    auto move_pick = [&](int32_t pick, uint64_t kp) {
      s_part[pick] = (int8_t)gs;
      const int64_t f = (int64_t)((kp & cField) >> 12);  // gain + 2^49
      s_key[pick] =
          cSide | (kp & cAdj) | ((uint64_t)(2 * (int64_t)cBias - f) << 12) | (kp & 4095);
    };
    // neighbour y of the pick: key updated, raise offered to its owner
    auto raise = [&](int32_t y, uint64_t ky, int64_t by, int64_t w, int64_t room_next) {
      const bool side = (ky >> 63) != 0;
      const uint64_t nk = (ky + ((uint64_t)(side ? -2 * w : 2 * w) << 12)) | cAdj;
      s_key[y] = nk;
      if (!side && by <= room_next) atomicMax((unsigned long long*)&s_raise[y % BS], nk);
    };
    if constexpr (kLongRows) {
      // Long rows (dense coarsest graphs): after the pick is known, the whole
      // block reads its row, U entries per thread in flight, and updates the
      // neighbours; one row read per pick instead of one per wave.
      constexpr int U = 8;
      while (pg < tg) {
        const int64_t room = mg - pg;
        const uint64_t wk = own_best(room);
        if (lane_id() == 0) s_wmax[threadIdx.x / 64] = wk;
        __syncthreads();
        const int32_t pick = block_pick();
        if (pick < 0) break;
        const int64_t bp = s_b[pick];
        const int64_t room_next = room - bp;
        rescan_owner(pick, room_next);
        const int32_t p0 = s_xadj[pick], p1 = s_xadj[pick + 1];
        if (threadIdx.x == 0) move_pick(pick, s_key[pick]);
        for (int32_t e = p0 + (int32_t)threadIdx.x; e < p1; e += BS * U) {
          int32_t y[U];
          int64_t w[U];
#pragma unroll
          for (int k = 0; k < U; k++) {
            const int32_t q = e + BS * k;
            y[k] = q < p1 ? lv.adj[q] : 0;
            w[k] = q < p1 ? lv.w[q] : 0;
          }
          uint64_t ky[U];
          int64_t by[U];
#pragma unroll
          for (int k = 0; k < U; k++) {
            const bool act = e + BS * k < p1;
            ky[k] = act ? s_key[y[k]] : 0;
            by[k] = act ? s_b[y[k]] : 0;
          }
#pragma unroll
          for (int k = 0; k < U; k++)
            if (e + BS * k < p1) raise(y[k], ky[k], by[k], w[k], room_next);
        }
        pg += bp;
        __syncthreads();
      }
    } else {
      constexpr int kPre = 2;  // row entries per lane fetched ahead
      while (pg < tg) {
        const int64_t room = mg - pg;
        const uint64_t wk = own_best(room);
        // The pick is always one wave's best (or, first, the seed), so each
        // wave fetches the row of its own candidate now and the global
        // latency runs under the barrier; the wave whose candidate is picked
        // applies the update from registers.  Candidates of different waves
        // are different vertices (every vertex has one owner thread).
        const int wave = (int)threadIdx.x / 64;
        const int32_t pre =
            (first && seed_fits && wave == seed_wave) ? seedv : (wk ? vid(wk) : -1);
        int32_t p0 = 0, p1 = 0;
        int32_t py[kPre];
        int64_t pw[kPre];
        if (pre >= 0) {
          p0 = s_xadj[pre];
          p1 = s_xadj[pre + 1];
#pragma unroll
          for (int j = 0; j < kPre; j++) {
            const int32_t e = p0 + lane_id() + 64 * j;
            py[j] = e < p1 ? lv.adj[e] : 0;
            pw[j] = e < p1 ? lv.w[e] : 0;
          }
        }
        if (lane_id() == 0) s_wmax[wave] = wk;
        __syncthreads();
        const int32_t pick = block_pick();
        if (pick < 0) break;
        const int64_t bp = s_b[pick];
        const int64_t room_next = room - bp;
        rescan_owner(pick, room_next);
        if (pre == pick) {
          // lane 0 moves the pick itself while the lanes update its
          // neighbours (never the pick: no self loops); every LDS read is
          // issued before any write, so the update is one round trip
          uint64_t ky[kPre];
          int64_t by[kPre];
#pragma unroll
          for (int j = 0; j < kPre; j++) {
            const bool act = p0 + lane_id() + 64 * j < p1;
            ky[j] = act ? s_key[py[j]] : 0;
            by[j] = act ? s_b[py[j]] : 0;
          }
          const uint64_t kp = lane_id() == 0 ? s_key[pick] : 0;
#pragma unroll
          for (int j = 0; j < kPre; j++)
            if (p0 + lane_id() + 64 * j < p1) raise(py[j], ky[j], by[j], pw[j], room_next);
          if (lane_id() == 0) move_pick(pick, kp);
          for (int32_t e = p0 + lane_id() + 64 * kPre; e < p1; e += 64) {
            const int32_t y = lv.adj[e];
            raise(y, s_key[y], s_b[y], lv.w[e], room_next);
          }
        }
        pg += bp;
        __syncthreads();
      }
    }
    __syncthreads();
    for (int32_t v = threadIdx.x; v < n; v += BS) {
      const uint64_t k = s_key[v];
      s_adj[v] = (int8_t)((k >> 62) & 1);
      s_gain[v] = (int64_t)((k & cField) >> 12) - (int64_t)cBias;
    }
  } else if (packed) {
    uint64_t* s_key = (uint64_t*)s_gain;
    for (int32_t v = threadIdx.x; v < n; v += BS) s_key[v] = (uint64_t)s_gain[v] + kBias;
    __syncthreads();
    // (key, id) of the best fitting vertex of this thread; key 0 = none.
    // Bit 63 of a key marks a vertex already on side gs.  The slot count is
    // fixed per size class so that the loads of all slots are in flight at
    // once (slots past n read vertex 0 and are discarded).
    auto rescan_slots = [&](auto slots, int64_t room, uint64_t& bk, int32_t& bv) {
      constexpr int S = decltype(slots)::value;
      uint64_t kv[S];
      int64_t bw[S];
#pragma unroll
      for (int q = 0; q < S; q++) {
        const int32_t v = (int32_t)threadIdx.x + q * BS;
        const int32_t vv = v < n ? v : 0;
        kv[q] = s_key[vv];
        bw[q] = s_b[vv];
      }
      bk = 0;
      bv = -1;
#pragma unroll
      for (int q = 0; q < S; q++) {
        const int32_t v = (int32_t)threadIdx.x + q * BS;
        const bool ok = (v < n) & ((kv[q] >> 63) == 0) & (bw[q] <= room);
        const uint64_t k = ok ? kv[q] : 0;
        const bool take = k > bk;  // ascending ids: ties keep the smaller id
        bk = take ? k : bk;
        bv = take ? v : bv;
      }
    };
    static_assert(kTrialLdsMax <= 12 * BS, "slot classes cover the LDS-resident sizes");
    auto rescan = [&](int64_t room, uint64_t& bk, int32_t& bv) {
      if (n <= 4 * BS) rescan_slots(LaneXor<4>{}, room, bk, bv);
      else if (n <= 8 * BS) rescan_slots(LaneXor<8>{}, room, bk, bv);
      else rescan_slots(LaneXor<12>{}, room, bk, bv);
    };
    auto better = [](uint64_t k2, int32_t v2, uint64_t k, int32_t v) {
      return k2 > k || (k2 == k && v2 < v);
    };
    __shared__ uint64_t s_bk[BS / 64];
    __shared__ int32_t s_bv[BS / 64];
    uint64_t bk;
    int32_t bv;
    rescan(mg, bk, bv);
    bool first = true;
    while (pg < tg) {
      uint64_t wk = bk;
      int32_t wv = bv;
      butterfly<64>([&](auto o) {
        const uint64_t k2 = xor_lane<decltype(o)::value>(wk);
        const int32_t v2 = xor_lane<decltype(o)::value>(wv);
        const bool t2 = better(k2, v2, wk, wv);
        wk = t2 ? k2 : wk;
        wv = t2 ? v2 : wv;
      });
      if (lane_id() == 0) {
        s_bk[threadIdx.x / 64] = wk;
        s_bv[threadIdx.x / 64] = wv;
      }
      __syncthreads();
      uint64_t gk = s_bk[0];
      int32_t gv = s_bv[0];
#pragma unroll
      for (int w = 1; w < BS / 64; w++) {
        const bool t2 = better(s_bk[w], s_bv[w], gk, gv);
        gk = t2 ? s_bk[w] : gk;
        gv = t2 ? s_bv[w] : gv;
      }
      int32_t pick = gk ? gv : -1;
      if (first && pg + s_b[seedv] <= mg) pick = seedv;
      first = false;
      if (pick < 0) break;
      if (threadIdx.x == 0) {
        s_part[pick] = (int8_t)gs;
        // gain -> -gain in the biased field; the adjacency bit is kept and
        // bit 63 marks the side
        const uint64_t k = s_key[pick];
        s_key[pick] = kSide | (k & kAdj) |
                      (uint64_t)(2 * (int64_t)kBias - (int64_t)(k & kField));
        s_dirty[pick % BS] = 1;
      }
      __syncthreads();
      const int32_t e1 = s_xadj[pick + 1];
      for (int32_t e = s_xadj[pick] + threadIdx.x; e < e1; e += BS) {
        const int32_t y = lv.adj[e];
        const int64_t w = lv.w[e];
        const uint64_t ky = s_key[y];
        s_key[y] = (ky + (uint64_t)((ky >> 63) ? -2 * w : 2 * w)) | kAdj;
        s_dirty[y % BS] = 1;
      }
      pg += s_b[pick];
      __syncthreads();
      const int64_t room = mg - pg;
      if (s_dirty[threadIdx.x] || (bv >= 0 && s_b[bv] > room)) {
        s_dirty[threadIdx.x] = 0;
        rescan(room, bk, bv);
      }
    }
    __syncthreads();
    for (int32_t v = threadIdx.x; v < n; v += BS) {
      const uint64_t k = s_key[v];
      s_adj[v] = (int8_t)((k >> 62) & 1);
      s_gain[v] = (int64_t)(k & kField) - (int64_t)kBias;
    }
  } else {
    auto rescan = [&](int64_t room) {
      GrowBest lb;
      lb.v = -1;
      lb.a = 0;
      lb.g = 0;
      for (int32_t v = threadIdx.x; v < n; v += BS) {
        if (s_part[v] != gb || s_b[v] > room) continue;
        GrowBest x;
        x.a = s_adj[v];
        x.g = s_gain[v];
        x.v = v;
        if (grow_better(x, lb)) lb = x;
      }
      return lb;
    };
    GrowBest lb = rescan(mg);
    bool first = true;
    while (pg < tg) {
      const GrowBest best = block_grow_argmax<BS>(lb, sgb);
      int32_t pick = best.v;
      if (first && pg + s_b[seedv] <= mg) pick = seedv;
      first = false;
      if (pick < 0) break;
      if (threadIdx.x == 0) {
        s_part[pick] = (int8_t)gs;
        s_gain[pick] = -s_gain[pick];
        s_dirty[pick % BS] = 1;
      }
      __syncthreads();
      // the neighbours of the pick are distinct (canonical rows): plain updates
      const int32_t e1 = s_xadj[pick + 1];
      for (int32_t e = s_xadj[pick] + threadIdx.x; e < e1; e += BS) {
        const int32_t y = lv.adj[e];
        const int64_t w = lv.w[e];
        s_adj[y] = 1;
        s_gain[y] += s_part[y] == gs ? -2 * w : 2 * w;
        s_dirty[y % BS] = 1;
      }
      pg += s_b[pick];
      __syncthreads();
      const int64_t room = mg - pg;
      if (s_dirty[threadIdx.x] || (lb.v >= 0 && s_b[lb.v] > room)) {
        s_dirty[threadIdx.x] = 0;
        lb = rescan(room);
      }
    }
  }
  if (threadIdx.x == 0) {
    srf.maxw[0] = ctrl->ref.maxw[0];
    srf.maxw[1] = ctrl->ref.maxw[1];
    srf.pw[gs] = pg;
    srf.pw[gb] = W - pg;
    start_level(&srf, npass);
  }
  __syncthreads();
  LevelView lvl = lv;
  lvl.xadj = s_xadj;
  lvl.xend = s_xadj + 1;
  lds_refine<BS>(lvl, s_gain, s_b, s_part, s_mv, srf, sel);
  // cut = sum over v of (gain + tot) / 4
  int64_t q = 0;
  for (int32_t v = threadIdx.x; v < n; v += BS) q += s_gain[v] + tot[v];
  q = block_sum<BS, int64_t>(q, sml);
  int8_t* part = tpart + (int64_t)t * n;
  for (int32_t v = threadIdx.x; v < n; v += BS) part[v] = s_part[v];
  if (threadIdx.x == 0) {
    tres[2 * t] = q / 4;
    tres[2 * t + 1] = (srf.pw[0] > srf.maxw[0] || srf.pw[1] > srf.maxw[1]) ? 1 : 0;
    tctl[t].pw[0] = srf.pw[0];
    tctl[t].pw[1] = srf.pw[1];
  }
  __syncthreads();
}

// -------------------------------------------------------------- gp_create
__device__ __forceinline__ void b_val_xadj(int32_t n, const int32_t* xadj, Ctrl* ctrl, int bid_, int nblk_) {
  for (int64_t v = (int64_t)bid_ * kBlock + threadIdx.x; v < n;
       v += (int64_t)nblk_ * kBlock) {
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
  butterfly<64>([&](auto o) { v = sat62(v, xor_lane<decltype(o)::value>(v)); });
  if (lane_id() == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  uint64_t r = 0;
  for (int i = 0; i < BS / 64; i++) r = sat62(r, sm[i]);
  __syncthreads();
  return r;
}

// ranges, self loops, sortedness, weight sums; one 16-lane team per row
__device__ __forceinline__ void b_val_rows(int32_t n, const int32_t* xadj,
                                                     const int32_t* adj, const int64_t* w,
                                                     const int64_t* vc, const int64_t* vg,
                                                     Ctrl* ctrl, int bid_, int nblk_) {
  __shared__ uint64_t smu[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  const uint64_t lim = 1ull << 62;
  uint32_t err = 0, unsorted = 0;
  uint64_t sw = 0, sc = 0, sg = 0;
  int64_t mc = 0, mg = 0;
  const int lane = threadIdx.x & 15;
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / 16;
  const int64_t nteams = (int64_t)nblk_ * kBlock / 16;
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

__device__ __forceinline__ void b_sort_rows(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl,
                                                      unsigned char* lds, int bid_, int nblk_) {
  // lds: kSortCap x (int64 + int32) bytes
  int64_t* sv = (int64_t*)lds;
  int32_t* sk = (int32_t*)(sv + kSortCap);
  __shared__ int32_t smi[kBlock / 64];
  bool dup = false;
  for (int64_t u0 = (int64_t)bid_ * kTileC; u0 < n; u0 += (int64_t)nblk_ * kTileC) {
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
__device__ __forceinline__ void b_sort_long(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl,
                                                      unsigned char* lds, int bid_, int nblk_) {
  int64_t* acc = (int64_t*)lds;
  int32_t* cc = (int32_t*)(acc + kWin);
  __shared__ int32_t smi[kBlock / 64];
  __shared__ int64_t sml[kBlock / 64];
  bool dup = false;
  for (int64_t u = bid_; u < n; u += nblk_) {
    const int32_t e0 = xadj[u], L = xadj[u + 1] - e0;
    if (L <= kSortCap) continue;
    PlainRowLoader ld{adj, w, e0};
    block_dense_emit<kBlock, false>(L, ld, acc, cc, smi, sml, oadj + e0, ow + e0, &dup);
  }
  if (dup) atomicOr(&ctrl->verr, kVDup);
}

// every entry u->v must have v->u with the same weight (rows sorted)
__device__ __forceinline__ void b_val_sym(int32_t n, const int32_t* xadj,
                                                    const int32_t* adj, const int64_t* w,
                                                    Ctrl* ctrl, int bid_, int nblk_) {
  const int lane = threadIdx.x & 15;
  const int64_t team = ((int64_t)bid_ * kBlock + threadIdx.x) / 16;
  const int64_t nteams = (int64_t)nblk_ * kBlock / 16;
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

__device__ __forceinline__ void b_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg, int bid_, int nblk_) {
  for (int64_t v = (int64_t)bid_ * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)nblk_ * blockDim.x) {
    vc[v] = vwgt[2 * v];
    vg[v] = vwgt[2 * v + 1];
  }
}


}  // namespace gpk
