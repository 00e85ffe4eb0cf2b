// gp_dev.h - device building blocks for gfx950 (wave64).
//
// Teams: a team is TW consecutive lanes of one wave (TW in 1..64) that work
// on one CSR row; reductions inside a team use cross-lane shuffles.  Block
// reductions combine per-wave results through LDS.  Everything here is
// integer arithmetic, so results do not depend on the order in which lanes,
// waves or blocks combine.
#pragma once

#include <limits.h>

#include "gp_internal.h"

namespace gpk {

typedef unsigned __int128 u128;

// SplitMix64 output finaliser (Steele, Lea, Flood 2014; constants by Vigna).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// ------------------------------------------------------ lane exchange
// The value of lane (lane ^ O), O in {1, 2, 4, 8, 16, 32}, moved in registers:
// DPP within 16-lane rows (xor 1 and 2 are quad permutations; xor 4 is the
// half-row mirror (x ^ 7) followed by the quad reversal (x ^ 3); xor 8 is the
// row mirror (x ^ 15) followed by the half-row mirror), and the gfx950
// permlane swaps across rows (16) and wave halves (32).  An LDS permute
// (ds_bpermute) costs an LDS round trip per step instead.  Every lane of the
// aligned group of 2 O lanes holding the pair must be active.  O is a
// template argument so that no step is ever dispatched at run time.
template <int CTRL>
__device__ __forceinline__ int32_t dpp(int32_t v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int O>
__device__ __forceinline__ int32_t xor_lane32(int32_t v) {
  static_assert(O == 1 || O == 2 || O == 4 || O == 8 || O == 16 || O == 32, "lane xor");
  if constexpr (O == 1) {
    return dpp<0xB1>(v);  // quad_perm(1,0,3,2)
  } else if constexpr (O == 2) {
    return dpp<0x4E>(v);  // quad_perm(2,3,0,1)
  } else if constexpr (O == 4) {
    return dpp<0x1B>(dpp<0x141>(v));  // half-row mirror, then quad_perm(3,2,1,0)
  } else if constexpr (O == 8) {
    return dpp<0x141>(dpp<0x140>(v));  // row mirror, then half-row mirror
  } else if constexpr (O == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    return (int32_t)((lane_id() & 16) ? p[0] : p[1]);
  } else {
    const auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int32_t)((lane_id() & 32) ? p[0] : p[1]);
  }
}

template <int O, class T>
__device__ __forceinline__ T xor_lane(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lane values");
  if constexpr (sizeof(T) == 4) {
    int32_t x;
    __builtin_memcpy(&x, &v, 4);
    x = xor_lane32<O>(x);
    T r;
    __builtin_memcpy(&r, &x, 4);
    return r;
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    const uint32_t lo = (uint32_t)xor_lane32<O>((int32_t)(uint32_t)u);
    const uint32_t hi = (uint32_t)xor_lane32<O>((int32_t)(uint32_t)(u >> 32));
    u = ((uint64_t)hi << 32) | lo;
    T r;
    __builtin_memcpy(&r, &u, 8);
    return r;
  }
}

// Butterfly over a team of TW lanes: step(integral O) for O = TW/2, ..., 1.
template <int O>
struct LaneXor {
  static constexpr int value = O;
};

template <int TW, class F>
__device__ __forceinline__ void butterfly(F&& step) {
  if constexpr (TW > 32) step(LaneXor<32>{});
  if constexpr (TW > 16) step(LaneXor<16>{});
  if constexpr (TW > 8) step(LaneXor<8>{});
  if constexpr (TW > 4) step(LaneXor<4>{});
  if constexpr (TW > 2) step(LaneXor<2>{});
  if constexpr (TW > 1) step(LaneXor<1>{});
}

// ----------------------------------------------------------------- teams
template <int TW, class T>
__device__ __forceinline__ T team_sum(T v) {
  butterfly<TW>([&](auto o) { v += xor_lane<decltype(o)::value>(v); });
  return v;
}

template <int TW, class T>
__device__ __forceinline__ T team_max(T v) {
  butterfly<TW>([&](auto o) {
    const T u = xor_lane<decltype(o)::value>(v);
    v = u > v ? u : v;
  });
  return v;
}

template <int TW, class T>
__device__ __forceinline__ T team_min(T v) {
  butterfly<TW>([&](auto o) {
    const T u = xor_lane<decltype(o)::value>(v);
    v = u < v ? u : v;
  });
  return v;
}

// --------------------------------------------------------------- blocks
// sm must hold BS/64 elements; every thread gets the result
template <int BS, class T>
__device__ __forceinline__ T block_sum(T v, T* sm) {
  v = team_sum<64>(v);
  if (lane_id() == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  T r = 0;
#pragma unroll
  for (int i = 0; i < BS / 64; i++) r += sm[i];
  __syncthreads();
  return r;
}

template <int BS, class T>
__device__ __forceinline__ T block_max(T v, T* sm) {
  v = team_max<64>(v);
  if (lane_id() == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  T r = sm[0];
#pragma unroll
  for (int i = 1; i < BS / 64; i++) r = sm[i] > r ? sm[i] : r;
  __syncthreads();
  return r;
}

template <int BS, class T>
__device__ __forceinline__ T block_min(T v, T* sm) {
  v = team_min<64>(v);
  if (lane_id() == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  T r = sm[0];
#pragma unroll
  for (int i = 1; i < BS / 64; i++) r = sm[i] < r ? sm[i] : r;
  __syncthreads();
  return r;
}

// (sum a, sum b, min c, max d) over the block with one LDS exchange; sm
// holds 4 * BS/64 elements; every thread gets the results
template <int BS>
__device__ __forceinline__ void block_sum_sum_min_max(int64_t& a, int64_t& b, int64_t& c,
                                                      int64_t& d, int64_t* sm) {
  butterfly<64>([&](auto o) {
    a += xor_lane<decltype(o)::value>(a);
    b += xor_lane<decltype(o)::value>(b);
    const int64_t c2 = xor_lane<decltype(o)::value>(c);
    const int64_t d2 = xor_lane<decltype(o)::value>(d);
    c = c2 < c ? c2 : c;
    d = d2 > d ? d2 : d;
  });
  constexpr int W = BS / 64;
  const int w = threadIdx.x / 64;
  if (lane_id() == 0) {
    sm[w] = a;
    sm[W + w] = b;
    sm[2 * W + w] = c;
    sm[3 * W + w] = d;
  }
  __syncthreads();
  a = sm[0];
  b = sm[W];
  c = sm[2 * W];
  d = sm[3 * W];
#pragma unroll
  for (int i = 1; i < W; i++) {
    a += sm[i];
    b += sm[W + i];
    c = sm[2 * W + i] < c ? sm[2 * W + i] : c;
    d = sm[3 * W + i] > d ? sm[3 * W + i] : d;
  }
  __syncthreads();
}

// exclusive prefix over the block in thread order; *total = block sum.
template <int BS, class T>
__device__ __forceinline__ T block_exscan(T v, T* sm, T* total) {
  const int l = lane_id();
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (l >= o) x += y;
  }
  if (l == 63) sm[threadIdx.x / 64] = x;
  __syncthreads();
  T base = 0, tot = 0;
  const int w = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < BS / 64; i++) {
    if (i < w) base += sm[i];
    tot += sm[i];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Returns true in every thread of the block that finished last among
// nblocks blocks sharing *ctr (which it also resets to 0).  Global writes
// made by any block before the call are visible to the last block after it.
__device__ __forceinline__ bool last_block(uint32_t* ctr, uint32_t nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t prev = atomicAdd(ctr, 1u);
    s_last = (prev == nblocks - 1);
    if (s_last) *ctr = 0;
  }
  __syncthreads();
  int last = s_last;
  if (last) __threadfence();
  return last;
}

// Tail of a phase that runs on nblk blocks: true in the block that runs the
// phase's single-block tail.  With one block it is that block, after a
// barrier; otherwise the last block to finish (see last_block).
__device__ __forceinline__ bool tail_gate(uint32_t* ctr, int nblk) {
  if (nblk == 1) {
    __syncthreads();
    return true;
  }
  return last_block(ctr, (uint32_t)nblk);
}

// Appends c to list when flag is set, one atomic per wave.  The order of
// the list is unspecified; every consumer of it is order-independent.
__device__ __forceinline__ void append_cand(bool flag, const Cand& c, Cand* list,
                                            uint32_t* counter) {
  uint64_t m = __ballot(flag);
  if (m == 0) return;
  int leader = __builtin_ctzll(m);
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (flag) list[base + (uint32_t)__popcll(m & lanemask_lt())] = c;
}

// ------------------------------------------------------ admission threshold
// Candidates are admitted in order of the key (gain desc, id asc), encoded as
// key = ((gain - gmin) << idbits) | (2^idbits - 1 - v), larger key first.
__device__ __forceinline__ u128 cand_key(const Cand& c, int64_t gmin, int idbits) {
  uint64_t g = (uint64_t)(c.gain - gmin);
  uint64_t idpart = ((1ull << idbits) - 1ull) - (uint64_t)(uint32_t)c.v;
  return ((u128)g << idbits) | (u128)idpart;
}

constexpr int kSelSmall = 256;

// block-shared state of the threshold search; the small-list buffers live
// here (one copy per block, whatever the candidate source)
struct SelShared {
  int64_t hist[256];
  u128 prefix;
  int64_t above;
  int done;
  int scnt;
  u128 result;
  alignas(16) uint64_t skey[2 * kSelSmall];  // key words interleaved
  int64_t sw[kSelSmall];
};

// Candidate sources for the threshold search: a compacted list, or every
// vertex of an LDS-resident graph filtered by the pass predicate.
struct ListItems {
  const Cand* list;
  uint32_t n;
  __device__ __forceinline__ uint32_t count() const { return n; }
  __device__ __forceinline__ bool get(uint32_t i, Cand& c) const {
    c = list[i];
    return true;
  }
};

// the same candidates weighted by what they take from their side
template <class Items>
struct SrcItems {
  Items it;
  __device__ __forceinline__ uint32_t count() const { return it.count(); }
  __device__ __forceinline__ bool get(uint32_t i, Cand& c) const {
    if (!it.get(i, c)) return false;
    c.b = c.bs;
    return true;
  }
};

struct LdsItems {
  const int64_t* gain;
  const int64_t* b;
  const int8_t* part;
  int32_t n;
  int s, mode;
  __device__ __forceinline__ uint32_t count() const { return (uint32_t)n; }
  __device__ __forceinline__ bool get(uint32_t i, Cand& c) const {
    if (part[i] != s) return false;
    const int64_t g = gain[i];
    if (mode == 0 && g <= 0) return false;
    c.gain = g;
    c.b = b[i];
    c.bs = c.b;
    c.v = (int32_t)i;
    c.pad = 0;
    return true;
  }
};

// Radix descent over the candidates (8-bit digits from the top).
//   want_ge = 0: threshold of the longest prefix with weight <= bound
//   want_ge = 1: threshold of the shortest prefix with weight >= bound (> 0)
// Returns thr with the prefix = { key >= thr }.  Every thread of the block
// must call it; BS is the block size.
//
// Per digit: a weighted 256-bin histogram of the candidates that share the
// prefix chosen so far (a wave whose hitting lanes all fall in one bin adds
// their sum with one atomic, which keeps skewed digits from serialising on
// one bin), then a block-wide scan over the bins from the top picks the bin
// where the bound is crossed.
// Exact threshold of select_prefix (below) for at most kSelSmall
// candidates.  They are gathered into LDS; thread i takes candidate i and
// sums the weights of the candidates whose keys are larger (keys are
// distinct), which gives its running sum in the order key desc; the one
// candidate whose running sum first reaches the bound is the crossing one.
// The result equals the radix descent's:
//   want_ge: bound <= 0 -> the all-ones key of the digit width; total < bound
//            -> 0; else the key at which the running sum first reaches bound;
//   else:    bound < 0 -> that all-ones key + 1; total <= bound -> 0; else the
//            key at which the running sum first exceeds bound, + 1.
template <int BS, class Items>
__device__ u128 select_small(const Items& items, int64_t gmin, int idbits, int tbits, int want_ge,
                             int64_t bound, SelShared* sh) {
  // key words interleaved (one 16-byte read per key), padded to a multiple
  // of 8 with key 0 and weight 0, which change no running sum
  uint64_t* s_key = sh->skey;
  int64_t* s_w = sh->sw;
  int& s_cnt = sh->scnt;
  const int ndig = (tbits + 7) / 8;
  const u128 ones = (((u128)1) << (8 * ndig)) - 1;
  if (want_ge ? bound <= 0 : bound < 0) return want_ge ? ones : ones + 1;
  if (threadIdx.x == 0) {
    s_cnt = 0;
    sh->result = 0;  // the running sums never reach the bound
  }
  for (int i = threadIdx.x; i < kSelSmall; i += BS) {
    s_key[2 * i] = 0;
    s_key[2 * i + 1] = 0;
    s_w[i] = 0;
  }
  __syncthreads();
  const uint32_t cnt = items.count();
  for (uint32_t i = threadIdx.x; i < cnt; i += BS) {
    Cand c;
    if (!items.get(i, c)) continue;
    const int slot = atomicAdd(&s_cnt, 1);
    if (slot < kSelSmall) {
      const u128 k = cand_key(c, gmin, idbits);
      s_key[2 * slot] = (uint64_t)(k >> 64);
      s_key[2 * slot + 1] = (uint64_t)k;
      s_w[slot] = c.b;
    }
  }
  __syncthreads();
  const int m = s_cnt < kSelSmall ? s_cnt : kSelSmall;
  const int m8 = (m + 7) & ~7;
  for (int i = threadIdx.x; i < m; i += BS) {
    const uint64_t hi = s_key[2 * i], lo = s_key[2 * i + 1];
    const int64_t wi = s_w[i];
    int64_t above = 0;  // weights of the larger keys
    for (int j0 = 0; j0 < m8; j0 += 8) {
      uint64_t hj[8], lj[8];
      int64_t wj[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        hj[u] = s_key[2 * (j0 + u)];
        lj[u] = s_key[2 * (j0 + u) + 1];
        wj[u] = s_w[j0 + u];
      }
#pragma unroll
      for (int u = 0; u < 8; u++)
        above += (hj[u] > hi || (hj[u] == hi && lj[u] > lo)) ? wj[u] : 0;
    }
    const int64_t incl = above + wi;
    const bool cross = want_ge ? (incl >= bound && above < bound) : (incl > bound && above <= bound);
    if (cross) {
      const u128 k = ((u128)hi << 64) | (u128)lo;
      sh->result = want_ge ? k : k + 1;
    }
  }
  __syncthreads();
  const u128 r = sh->result;
  __syncthreads();
  return r;
}

template <int BS, class Items>
__device__ u128 select_prefix(const Items& items, int64_t gmin, int idbits, int tbits,
                              int want_ge, int64_t bound, SelShared* sh,
                              uint32_t ncand_hint = 0xffffffffu) {
  static_assert(BS % 64 == 0 && (BS >= 256 || 256 % BS == 0), "block of whole waves");
  if (ncand_hint <= (uint32_t)kSelSmall)
    return select_small<BS>(items, gmin, idbits, tbits, want_ge, bound, sh);
  constexpr int PER = BS >= 256 ? 1 : 256 / BS;  // histogram bins per thread
  __shared__ int64_t sm_scan[BS / 64];
  __shared__ int32_t sm_min[BS / 64];
  const int ndig = (tbits + 7) / 8;
  const uint32_t cnt = items.count();
  const int lane = lane_id();
  if (threadIdx.x == 0) {
    sh->prefix = 0;
    sh->above = 0;
    sh->done = 0;
    sh->result = 0;
  }
  // U candidates per thread are loaded before any is used, so that the
  // loads of one round overlap instead of paying a round trip each; up to
  // BS * U candidates stay in registers for all digits
  constexpr int U = 4;
  const bool cached = cnt <= (uint32_t)(BS * U);
  Cand cc[U];
  bool cg[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const uint32_t i = (uint32_t)(u * BS) + threadIdx.x;
    cc[u].b = 0;
    cg[u] = cached && i < cnt && items.get(i, cc[u]);
  }
  __syncthreads();
  for (int d = ndig - 1; d >= 0; d--) {
    const int shf = 8 * d;
    for (int q = threadIdx.x; q < 256; q += BS) sh->hist[q] = 0;
    __syncthreads();
    const u128 P = sh->prefix;
    // uniform trip count: every lane of a wave takes part in the ballots
    for (uint32_t base = 0; base < cnt; base += BS * U) {
      Cand cs[U];
      bool got[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (cached) {
          cs[u] = cc[u];
          got[u] = cg[u];
        } else {
          const uint32_t i = base + (uint32_t)(u * BS) + threadIdx.x;
          cs[u].b = 0;
          got[u] = i < cnt && items.get(i, cs[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        int bkt = -1;
        if (got[u]) {
          const u128 k = cand_key(cs[u], gmin, idbits);
          if ((k >> (shf + 8)) == P) bkt = (int)((k >> shf) & 255);
        }
        const uint64_t hits = __ballot(bkt >= 0);
        if (hits == 0) continue;
        const int lead = __builtin_ctzll(hits);
        const int b0 = __shfl(bkt, lead, 64);
        if (__ballot(bkt >= 0 && bkt != b0) == 0) {
          const int64_t sum = team_sum<64, int64_t>(bkt >= 0 ? cs[u].b : 0);
          if (lane == lead)
            atomicAdd((unsigned long long*)&sh->hist[b0], (unsigned long long)sum);
        } else if (bkt >= 0) {
          atomicAdd((unsigned long long*)&sh->hist[bkt], (unsigned long long)cs[u].b);
        }
      }
    }
    __syncthreads();
    // thread t looks at bins 255 - j for j in [t*PER, t*PER + PER): the bins
    // from the top, with running sums
    const int j0 = (int)threadIdx.x * PER;
    int64_t hv[PER];
    int64_t local = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
      hv[q] = j0 + q < 256 ? sh->hist[255 - (j0 + q)] : 0;
      local += hv[q];
    }
    int64_t tot;
    const int64_t ex = block_exscan<BS, int64_t>(local, sm_scan, &tot);
    const int64_t above0 = sh->above;
    int64_t run = above0 + ex, at = 0;
    int first = 1 << 30;
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const bool cross = j0 + q < 256 &&
                         (want_ge ? (run + hv[q] >= bound) : (run + hv[q] > bound));
      if (cross && first == (1 << 30)) {
        first = j0 + q;
        at = run;
      }
      run += hv[q];
    }
    const int mine = first;
    first = block_min<BS, int32_t>(first, sm_min);
    if (first < 256 && mine == first) {
      sh->above = at;
      sh->prefix = (P << 8) | (u128)(unsigned)(255 - first);
    }
    if (first >= 256 && threadIdx.x == 0) {
      // only for want_ge = 0: every candidate with this prefix fits
      sh->above = above0 + tot;
      sh->result = P << (shf + 8);
      sh->done = 1;
    }
    __syncthreads();
    if (sh->done) break;
  }
  u128 r;
  if (sh->done) r = sh->result;
  else r = want_ge ? sh->prefix : sh->prefix + 1;
  __syncthreads();
  return r;
}

__device__ __forceinline__ int bitlen64(uint64_t x) { return x == 0 ? 0 : 64 - __clzll(x); }

// ------------------------------------------------------------ row sorting
// A row of L candidates (key, val) is reduced to its distinct keys in
// ascending order with the vals of equal keys summed (MERGE) or with a flag
// raised on a repeated key (!MERGE).  Key INT_MAX means "drop".

// one element per lane, T lanes, L <= T
template <int T, int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_step(int32_t& k, int64_t& v) {
  const int lane = threadIdx.x & (T - 1);
  const int32_t k2 = xor_lane<STRIDE>(k);
  const int64_t v2 = xor_lane<STRIDE>(v);
  const bool up = (lane & SIZE) == 0;
  const bool lower = (lane & STRIDE) == 0;
  const bool take = (lower == up) ? (k2 < k) : (k2 > k);
  if (take) {
    k = k2;
    v = v2;
  }
  if constexpr (STRIDE > 1) bitonic_step<T, SIZE, STRIDE / 2>(k, v);
}

template <int T, int SIZE>
__device__ __forceinline__ void bitonic_stage(int32_t& k, int64_t& v) {
  bitonic_step<T, SIZE, SIZE / 2>(k, v);
  if constexpr (SIZE < T) bitonic_stage<T, SIZE * 2>(k, v);
}

// one element per lane, T lanes, L <= T; ascending keys
template <int T>
__device__ __forceinline__ void team_bitonic(int32_t& k, int64_t& v) {
  bitonic_stage<T, 2>(k, v);
}

// after team_bitonic: writes the distinct keys, returns their count
template <int T, bool MERGE>
__device__ __forceinline__ int team_emit(int32_t k, int64_t v, int32_t* okey, int64_t* oval,
                                         bool* dup) {
  const int lane = threadIdx.x & (T - 1);
  if (MERGE) {
#pragma unroll
    for (int o = 1; o < T; o <<= 1) {
      int32_t ko = __shfl_up(k, o, T);
      int64_t vo = __shfl_up(v, o, T);
      if (lane >= o && ko == k) v += vo;
    }
  }
  int32_t knext = __shfl_down(k, 1, T);
  const bool valid = k != INT_MAX;
  const bool last = (lane == T - 1) || (knext != k);
  if (!MERGE && valid && !last) *dup = true;
  const bool emit = valid && (MERGE ? last : true);
  uint64_t m = __ballot(emit);
  const int tb = lane_id() & ~(T - 1);
  uint64_t tm = (T == 64) ? m : ((m >> tb) & ((1ull << T) - 1ull));
  int pos = __popcll(tm & ((1ull << lane) - 1ull));
  if (emit) {
    okey[pos] = k;
    oval[pos] = v;
  }
  return __popcll(tm);
}

__device__ __forceinline__ int next_pow2(int x) {
  int p = 2;
  while (p < x) p <<= 1;
  return p;
}

// L <= kSortCap, whole block, LDS arrays sk/sv of kSortCap entries
template <int BS, bool MERGE, class Loader>
__device__ int block_sort_emit(int L, const Loader& ld, int32_t* sk, int64_t* sv, int32_t* okey,
                               int64_t* oval, bool* dup, int32_t* smi) {
  const int P2 = next_pow2(L);
  for (int i = threadIdx.x; i < P2; i += BS) {
    int32_t k = INT_MAX;
    int64_t v = 0;
    if (i < L) ld(i, k, v);
    sk[i] = k;
    sv[i] = v;
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P2 / 2; i += BS) {
        int lo = (i / stride) * stride * 2 + (i % stride);
        int hi = lo + stride;
        bool up = (lo & size) == 0;
        int32_t a = sk[lo], b = sk[hi];
        if ((a > b) == up && a != b) {
          sk[lo] = b;
          sk[hi] = a;
          int64_t t = sv[lo];
          sv[lo] = sv[hi];
          sv[hi] = t;
        }
      }
      __syncthreads();
    }
  }
  // distinct keys: thread t owns a chunk of consecutive slots
  const int per = (P2 + BS - 1) / BS;
  const int s0 = threadIdx.x * per;
  int heads = 0;
  for (int i = s0; i < s0 + per && i < P2; i++) {
    if (sk[i] == INT_MAX) break;
    if (i == 0 || sk[i - 1] != sk[i]) heads++;
    else if (!MERGE) *dup = true;
  }
  int total;
  int base = block_exscan<BS, int>(heads, smi, &total);
  for (int i = s0; i < s0 + per && i < P2; i++) {
    int32_t k = sk[i];
    if (k == INT_MAX) break;
    if (i == 0 || sk[i - 1] != k) {
      int64_t s = sv[i];
      if (MERGE)
        for (int j = i + 1; j < P2 && sk[j] == k; j++) s += sv[j];
      okey[base] = k;
      oval[base] = s;
      base++;
    }
  }
  __syncthreads();
  return total;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 64 < L <= kWaveCap, one wave, LDS arrays sk/sv private to the wave
template <bool MERGE, class Loader>
__device__ int wave_sort_emit(int L, const Loader& ld, int32_t* sk, int64_t* sv, int32_t* okey,
                              int64_t* oval, bool* dup) {
  const int lane = lane_id();
  const int P2 = next_pow2(L);
  for (int i = lane; i < P2; i += 64) {
    int32_t k = INT_MAX;
    int64_t v = 0;
    if (i < L) ld(i, k, v);
    sk[i] = k;
    sv[i] = v;
  }
  wave_sync();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < P2 / 2; i += 64) {
        const int lo = (i / stride) * stride * 2 + (i % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int32_t a = sk[lo], b = sk[hi];
        if ((a > b) == up && a != b) {
          sk[lo] = b;
          sk[hi] = a;
          const int64_t t = sv[lo];
          sv[lo] = sv[hi];
          sv[hi] = t;
        }
      }
      wave_sync();
    }
  }
  const int per = P2 / 64;  // P2 >= 128 here
  const int s0 = lane * per;
  int heads = 0;
  for (int i = s0; i < s0 + per; i++) {
    if (sk[i] == INT_MAX) break;
    if (i == 0 || sk[i - 1] != sk[i]) heads++;
    else if (!MERGE) *dup = true;
  }
  int x = heads;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  const int total = __shfl(x, 63, 64);
  int base = x - heads;
  for (int i = s0; i < s0 + per; i++) {
    const int32_t k = sk[i];
    if (k == INT_MAX) break;
    if (i == 0 || sk[i - 1] != k) {
      int64_t sum = sv[i];
      if (MERGE)
        for (int j = i + 1; j < P2 && sk[j] == k; j++) sum += sv[j];
      okey[base] = k;
      oval[base] = sum;
      base++;
    }
  }
  wave_sync();
  return total;
}

// ------------------------------------------------- key-only wave sorts
// Bitonic network on one int32 key per lane, 64 lanes, ascending; N
// independent columns at once (one key each per lane) so that the lane
// exchanges of one column overlap the compares of the others.
template <int N, int SIZE, int STRIDE>
__device__ __forceinline__ void kbitonic_step(int32_t (&k)[N]) {
  const int lane = lane_id();
  const bool up = (lane & SIZE) == 0;
  const bool lower = (lane & STRIDE) == 0;
  int32_t k2[N];
#pragma unroll
  for (int c = 0; c < N; c++) k2[c] = xor_lane<STRIDE>(k[c]);
#pragma unroll
  for (int c = 0; c < N; c++)
    k[c] = (lower == up) ? (k2[c] < k[c] ? k2[c] : k[c]) : (k2[c] > k[c] ? k2[c] : k[c]);
  if constexpr (STRIDE > 1) kbitonic_step<N, SIZE, STRIDE / 2>(k);
}

template <int N, int SIZE>
__device__ __forceinline__ void kbitonic_stage(int32_t (&k)[N]) {
  kbitonic_step<N, SIZE, SIZE / 2>(k);
  if constexpr (SIZE < 64) kbitonic_stage<N, SIZE * 2>(k);
}

// half-cleaners with strides 32, 16, ..., 1, all ascending: sorts bitonic
// 64-lane sequences whose halves are already split (lower <= upper)
template <int N, int STRIDE>
__device__ __forceinline__ void khalf_clean(int32_t (&k)[N]) {
  const bool lower = (lane_id() & STRIDE) == 0;
  int32_t k2[N];
#pragma unroll
  for (int c = 0; c < N; c++) k2[c] = xor_lane<STRIDE>(k[c]);
#pragma unroll
  for (int c = 0; c < N; c++)
    k[c] = lower ? (k2[c] < k[c] ? k2[c] : k[c]) : (k2[c] > k[c] ? k2[c] : k[c]);
  if constexpr (STRIDE > 1) khalf_clean<N, STRIDE / 2>(k);
}

// one compare-exchange step over the wave's LDS keys: pair t joins slots
// lo(t) and hi(t); U pairs per lane per iteration, all loads first (the
// pairs of one step are disjoint)
template <int U, class Pair>
__device__ __forceinline__ void kstep_lds(int32_t* sk, int npairs, const Pair& pair) {
  const int lane = lane_id();
  for (int t0 = 0; t0 < npairs; t0 += 64 * U) {
    int lo[U], hi[U];
    int32_t a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) pair(t0 + u * 64 + lane, lo[u], hi[u]);
#pragma unroll
    for (int u = 0; u < U; u++) {
      a[u] = sk[lo[u]];
      b[u] = sk[hi[u]];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      sk[lo[u]] = a[u] < b[u] ? a[u] : b[u];
      sk[hi[u]] = a[u] < b[u] ? b[u] : a[u];
    }
  }
}

template <class Pair>
__device__ __forceinline__ void kstep(int32_t* sk, int npairs, const Pair& pair) {
  if (npairs >= 256) kstep_lds<4>(sk, npairs, pair);
  else if (npairs >= 128) kstep_lds<2>(sk, npairs, pair);
  else kstep_lds<1>(sk, npairs, pair);
}

// the 64-key columns [r, r + N) of the wave's LDS keys through f, in registers
template <int N, class F>
__device__ __forceinline__ void kcolumns(int32_t* sk, int r, const F& f) {
  const int lane = lane_id();
  int32_t k[N];
#pragma unroll
  for (int c = 0; c < N; c++) k[c] = sk[(r + c) * 64 + lane];
  f(k);
#pragma unroll
  for (int c = 0; c < N; c++) sk[(r + c) * 64 + lane] = k[c];
}

// Ascending sort of P2 distinct int32 keys (INT_MAX padding allowed), P2 a
// power of two in [128, 64 * 64], in LDS private to one wave.  Columns of 64
// consecutive keys are sorted in registers, up to four at a time; each merge
// of two sorted blocks of `size` / 2 keys compares key j with its mirror
// j ^ (size - 1), which leaves both halves bitonic and split, then runs
// half-cleaners from stride size / 4 down: strides of 64 and more in LDS,
// the last six in registers.  Every step is a fixed compare-exchange
// network, so the result does not depend on timing.
__device__ __forceinline__ void wave_sort_keys(int32_t* sk, int P2) {
  const int cols = P2 >> 6;  // 2, or a multiple of 4
  auto sort_cols = [&](auto& k) { kbitonic_stage<sizeof(k) / sizeof(k[0]), 2>(k); };
  auto clean_cols = [&](auto& k) { khalf_clean<sizeof(k) / sizeof(k[0]), 32>(k); };
  if (cols >= 4) {
    for (int r = 0; r < cols; r += 4) kcolumns<4>(sk, r, sort_cols);
  } else {
    kcolumns<2>(sk, 0, sort_cols);
  }
  wave_sync();
  for (int size = 128; size <= P2; size <<= 1) {
    const int half = size >> 1;
    kstep(sk, P2 >> 1, [&](int t, int& lo, int& hi) {
      lo = (t & ~(half - 1)) * 2 + (t & (half - 1));
      hi = lo ^ (size - 1);
    });
    wave_sync();
    for (int stride = half >> 1; stride >= 64; stride >>= 1) {
      kstep(sk, P2 >> 1, [&](int t, int& lo, int& hi) {
        lo = (t & ~(stride - 1)) * 2 + (t & (stride - 1));
        hi = lo + stride;
      });
      wave_sync();
    }
    if (cols >= 4) {
      for (int r = 0; r < cols; r += 4) kcolumns<4>(sk, r, clean_cols);
    } else {
      kcolumns<2>(sk, 0, clean_cols);
    }
    wave_sync();
  }
}

// any L: dense accumulation over windows of kWin ids (LDS acc/cnt/pres)
template <int BS, bool MERGE, class Loader>
__device__ int block_dense_emit(int L, const Loader& ld, int64_t* acc, int32_t* cnt,
                                int32_t* smi, int64_t* sml, int32_t* okey, int64_t* oval,
                                bool* dup) {
  int32_t kmin = INT_MAX, kmax = -1;
  for (int i = threadIdx.x; i < L; i += BS) {
    int32_t k;
    int64_t v;
    ld(i, k, v);
    if (k != INT_MAX) {
      kmin = k < kmin ? k : kmin;
      kmax = k > kmax ? k : kmax;
    }
  }
  kmin = block_min<BS, int32_t>(kmin, smi);
  kmax = block_max<BS, int32_t>(kmax, smi);
  int out = 0;
  if (kmax < 0) return 0;
  for (int64_t lo = kmin; lo <= kmax; lo += kWin) {
    for (int i = threadIdx.x; i < kWin; i += BS) {
      acc[i] = 0;
      cnt[i] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += BS) {
      int32_t k;
      int64_t v;
      ld(i, k, v);
      if (k != INT_MAX && k >= lo && k < lo + kWin) {
        atomicAdd((unsigned long long*)&acc[k - lo], (unsigned long long)v);
        atomicAdd(&cnt[k - lo], 1);
      }
    }
    __syncthreads();
    constexpr int per = kWin / BS;
    const int s0 = threadIdx.x * per;
    int present = 0;
    for (int j = s0; j < s0 + per; j++) {
      present += cnt[j] > 0;
      if (!MERGE && cnt[j] > 1) *dup = true;
    }
    int total;
    int base = block_exscan<BS, int>(present, smi, &total);
    for (int j = s0; j < s0 + per; j++)
      if (cnt[j] > 0) {
        okey[out + base] = (int32_t)(lo + j);
        oval[out + base] = acc[j];
        base++;
      }
    out += total;
    __syncthreads();
  }
  (void)sml;
  return out;
}

}  // namespace gpk
