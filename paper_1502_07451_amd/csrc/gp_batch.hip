// gp_batch.hip - batched partition: thousands of independent DAGs in one
// persistent kernel, one workgroup per graph, captured in a hipGraph.
//
// Each workgroup pops graphs from an atomic queue (largest first) and runs
// the whole pipeline of gp_create + gp_partition for it with the phase
// bodies of gp_phases.h called at workgroup scope (bid 0 of 1 block).  The
// coarse levels of a graph are bump-allocated from a device arena; a graph
// that does not fit reports GP_ENOMEM and the host reruns it with a larger
// arena.  Results are independent of the queue order, of the number of
// workgroups and of the arena layout: each graph's computation reads and
// writes only its own data, with integer arithmetic.
#include <string.h>

#include <mutex>

#include <algorithm>
#include <chrono>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/gp.h"
#include "gp_launch.h"
#include "gp_phases.h"

namespace gpk {

constexpr int kBatchLevels = kMaxLevels + 1;

// dynamic LDS of the persistent kernel: the dense window of the long-row
// merge (kWin x 12 bytes) and, in the same bytes, an LDS-resident trial of up
// to kBatchTrialMax vertices (2,570).  58 KB plus the kernel's 19 KB of
// static LDS stay under half of a compute unit's 160 KB, so two workgroups
// share each unit, and the coarsest graphs of stalled coarsenings (tiled
// Cholesky DAGs of 2,600 and 2,925 tasks stop at 2,150 and 2,432 vertices)
// still fit; larger coarsest graphs take the global-memory trial form, which
// rescans every vertex per pick (about ten times slower).
constexpr size_t kBatchLds = 58 * 1024;
constexpr int kBatchTrialMax =
    (int)((kBatchLds - trial_lds_bytes(0, kBlock)) / 23) < kTrialLdsMax
        ? (int)((kBatchLds - trial_lds_bytes(0, kBlock)) / 23)
        : kTrialLdsMax;
static_assert(trial_lds_bytes(kBatchTrialMax, kBlock) <= kBatchLds, "trial state exceeds the LDS");
static_assert((size_t)kWin * 12 <= kBatchLds && (size_t)kRowBlockCap * 12 <= kBatchLds,
              "contraction buffers exceed the LDS");

struct LevelRec {
  int32_t n;
  int32_t nnz;      // entries in the rows
  const int32_t* xadj;
  const int32_t* xend;  // row v is [xadj[v], xend[v]); coarse rows keep gaps
  const int32_t* adj;
  const int64_t* w;
  int64_t* vc;
  int64_t* vg;
  int32_t* match;
  int32_t* cmap;
  int8_t* part;
};

// optional export of every graph's coarsest level and its plain bisection
// (training data of the learned proposal).  rec[4g..4g+3] = n, 2m, vertex
// slot, entry slot (or -1 when the export buffers are full); graph g's xadj
// (n+1 local offsets), vwgt (n x 2) and part (n) sit at its vertex slot,
// adjncy and adjwgt at its entry slot.
struct ExportArgs {
  int64_t* rec;
  unsigned long long* head_v;
  unsigned long long* head_e;
  int32_t* xadj;
  int64_t* vwgt;
  int8_t* part;
  int32_t* adj;
  int64_t* w;
  uint64_t cap_v, cap_e;
};

struct BatchArgs {
  int32_t G;
  const int64_t* voff;
  const int64_t* eoff;
  const int32_t* xadj;
  const int32_t* adj;
  const int64_t* w;
  const int64_t* vwgt;
  const int32_t* order;
  int8_t* part;
  gp_result* res;
  int64_t r0, r1;
  int32_t eps, bal;
  uint64_t seed;
  int32_t C, R, P, K;
  uint32_t* head;
  unsigned char* arena;
  uint64_t arena_cap;
  unsigned long long* arena_off;
  unsigned char* wgs;
  uint64_t wgs_stride;
  int32_t nmax;
  int32_t nnzmax;
  int32_t chunk;
  ExportArgs ex;  // ex.rec == nullptr: no export
  int64_t* tline; // per graph: wall-clock ticks when its workgroup took it and finished it
  int32_t tw_shift;  // team width scale (see team_width_dev)
};

// per-workgroup scratch carved from wgs + blockIdx.x * wgs_stride
struct WgScratch {
  Ctrl* ctrl;
  LevelRec* lev;
  Scratch sc;
  int64_t* tot;
  RefCtl* tctl;
  int8_t* tpart;
  int64_t* tres;
  int32_t* pass_sink;
};

__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// offsets of the per-workgroup scratch; returns its size
__host__ __device__ inline uint64_t wg_layout(int32_t nmax, int32_t nnzmax, uint64_t* off) {
  const uint64_t n1 = (uint64_t)(nmax > 0 ? nmax : 1), m1 = (uint64_t)(nnzmax > 0 ? nnzmax : 1);
  const uint64_t sizes[] = {
      sizeof(Ctrl), sizeof(LevelRec) * kBatchLevels,
      4 * n1,                      // prop
      4 * (n1 / kTileV + 2),       // tile_lead
      8 * (n1 / kTileV + 2),       // tile_ub
      4 * n1, 4 * n1,              // cmem0, cmem1
      8 * n1,                      // toff
      4 * n1,                      // cnt
      8 * (n1 / kTileC + 2),       // tile_cnt
      4 * m1, 8 * m1,              // tmpk, tmpv
      4 * n1,                      // longlist
      sizeof(Cand) * n1,           // list
      8 * n1,                      // tot
      sizeof(RefCtl) * 64,         // tctl
      64 * (uint64_t)kTrialLdsMax, // tpart
      8 * 128,                     // tres
      64};                         // pass sink
  uint64_t o = 0;
  for (int i = 0; i < (int)(sizeof(sizes) / sizeof(sizes[0])); i++) {
    off[i] = o;
    o = align256(o + sizes[i]);
  }
  return o;
}

__device__ WgScratch wg_scratch(const BatchArgs& a) {
  uint64_t off[32];
  wg_layout(a.nmax, a.nnzmax, off);
  unsigned char* base = a.wgs + (uint64_t)blockIdx.x * a.wgs_stride;
  WgScratch s;
  s.ctrl = (Ctrl*)(base + off[0]);
  s.lev = (LevelRec*)(base + off[1]);
  s.sc.prop = (int32_t*)(base + off[2]);
  s.sc.tile_lead = (int32_t*)(base + off[3]);
  s.sc.tile_ub = (int64_t*)(base + off[4]);
  s.sc.cmem0 = (int32_t*)(base + off[5]);
  s.sc.cmem1 = (int32_t*)(base + off[6]);
  s.sc.toff = (int64_t*)(base + off[7]);
  s.sc.cnt = (int32_t*)(base + off[8]);
  s.sc.tile_cnt = (int64_t*)(base + off[9]);
  s.sc.tmpk = (int32_t*)(base + off[10]);
  s.sc.tmpv = (int64_t*)(base + off[11]);
  s.sc.longlist = (int32_t*)(base + off[12]);
  s.sc.list = (Cand*)(base + off[13]);
  s.sc.partials = nullptr;  // one workgroup per graph: no cross-block partials
  s.tot = (int64_t*)(base + off[14]);
  s.tctl = (RefCtl*)(base + off[15]);
  s.tpart = (int8_t*)(base + off[16]);
  s.tres = (int64_t*)(base + off[17]);
  s.pass_sink = (int32_t*)(base + off[18]);
  return s;
}

// bump allocation from the arena by thread 0, broadcast to the block;
// nullptr when the arena is exhausted
__device__ void* arena_alloc(const BatchArgs& a, uint64_t bytes) {
  __shared__ void* s_ptr;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t b = align256(bytes > 0 ? bytes : 1);
    const uint64_t off = atomicAdd(a.arena_off, (unsigned long long)b);
    s_ptr = (off + b <= a.arena_cap) ? (void*)(a.arena + off) : nullptr;
  }
  __syncthreads();
  return s_ptr;
}

// lanes per row: the single-graph path's choice from the average degree
// (thresholds 6, 12, 24, 48), scaled by 2^shift (a tuning knob of the batch;
// no result depends on the team width), within [4, 64]
__device__ int team_width_dev(int32_t n, int32_t nnz, int shift = 0) {
  int tw = 64;
  const int64_t m = nnz;
  if (n <= 0 || m <= 6ll * n) tw = 4;
  else if (m <= 12ll * n) tw = 8;
  else if (m <= 24ll * n) tw = 16;
  else if (m <= 48ll * n) tw = 32;
  tw = shift >= 0 ? tw << shift : tw >> -shift;
  return tw < 4 ? 4 : (tw > 64 ? 64 : tw);
}

#define TW_DISPATCH(tw, CALL)        \
  switch (tw) {                      \
    case 4: { constexpr int TWv = 4; CALL; } break;   \
    case 8: { constexpr int TWv = 8; CALL; } break;   \
    case 16: { constexpr int TWv = 16; CALL; } break; \
    case 32: { constexpr int TWv = 32; CALL; } break; \
    default: { constexpr int TWv = 64; CALL; } break; \
  }

__device__ void write_status(const BatchArgs& a, int g, int32_t st) {
  if (threadIdx.x == 0) {
    gp_result r;
    memset(&r, 0, sizeof(r));
    r.status = st;
    a.res[g] = r;
  }
}

__device__ void zero_ctrl(Ctrl* c) {
  uint64_t* p = (uint64_t*)c;
  for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) p[i] = 0;
  __syncthreads();
}

// one graph, the whole workgroup; returns nothing, writes res[g] and part
__device__ void batch_graph(const BatchArgs& a, int g, const WgScratch& ws, unsigned char* lds,
                            SelShared* sel, RefCtl* srf) {
  Ctrl* ctrl = ws.ctrl;
  LevelRec* lev = ws.lev;
  const Scratch& sc = ws.sc;
  const int64_t v0 = a.voff[g], e0 = a.eoff[g];
  const int32_t n = (int32_t)(a.voff[g + 1] - v0);
  const int32_t nnz = (int32_t)(a.eoff[g + 1] - e0);
  const int32_t* xadj = a.xadj + v0 + g;
  const int32_t* adj = a.adj + e0;
  const int64_t* w = a.w + e0;
  const int64_t* vwgt = a.vwgt + 2 * v0;
  zero_ctrl(ctrl);
  if (n < 0 || nnz < 0 || n > a.nmax || nnz > a.nnzmax) {
    // outside the bounds the workgroup scratch was laid out for
    write_status(a, g, GP_EINVAL);
    return;
  }
  if (n == 0) {
    if (threadIdx.x == 0) {
      gp_result r;
      memset(&r, 0, sizeof(r));
      r.feasible = 1;
      a.res[g] = r;
    }
    return;
  }
  // ---- checks and canonical form (gp_create)
  b_val_xadj(n, xadj, ctrl, 0, 1);
  __syncthreads();
  if (ctrl->verr & kVInval || xadj[n] != nnz) {
    write_status(a, g, GP_EINVAL);
    return;
  }
  int64_t* vc0 = (int64_t*)arena_alloc(a, 8ull * n);
  int64_t* vg0 = (int64_t*)arena_alloc(a, 8ull * n);
  if (!vc0 || !vg0) {
    write_status(a, g, GP_ENOMEM);
    return;
  }
  b_split_vwgt(n, vwgt, vc0, vg0, 0, 1);
  __syncthreads();
  b_val_rows(n, xadj, adj, w, vc0, vg0, ctrl, 0, 1);
  __syncthreads();
  uint32_t e = ctrl->verr;
  if (e & kVRange) { write_status(a, g, GP_ERANGE); return; }
  if (e & kVSelf) { write_status(a, g, GP_ESELF); return; }
  const int32_t* adj0 = adj;
  const int64_t* w0 = w;
  if (ctrl->vunsorted) {
    int32_t* na = (int32_t*)arena_alloc(a, 4ull * nnz);
    int64_t* nw = (int64_t*)arena_alloc(a, 8ull * nnz);
    if (!na || !nw) { write_status(a, g, GP_ENOMEM); return; }
    b_sort_rows(n, xadj, adj, w, na, nw, ctrl, lds, 0, 1);
    __syncthreads();
    b_sort_long(n, xadj, adj, w, na, nw, ctrl, lds, 0, 1);
    __syncthreads();
    if (ctrl->verr & kVDup) { write_status(a, g, GP_EDUP); return; }
    adj0 = na;
    w0 = nw;
  }
  b_val_sym(n, xadj, adj0, w0, ctrl, 0, 1);
  __syncthreads();
  e = ctrl->verr;
  if (e & kVAsym) { write_status(a, g, GP_EASYM); return; }
  if (e & kVOverflow) { write_status(a, g, GP_EOVERFLOW); return; }
  const int64_t W = (int64_t)(a.bal ? ctrl->vsum_g : ctrl->vsum_c);
  const int64_t maxb0 = a.bal ? ctrl->vmax_g : ctrl->vmax_c;
  __syncthreads();
  // ---- balance bounds, Eq. (1)-(2) in integers
  if (threadIdx.x == 0) {
    const __int128 Rr = (__int128)a.r0 + a.r1;
    const int64_t r[2] = {a.r0, a.r1};
    for (int p = 0; p < 2; p++) {
      ctrl->tgt[p] = (int64_t)(((__int128)W * r[p]) / Rr);
      const __int128 num = (__int128)W * r[p] * (1000000 + a.eps);
      const __int128 den = Rr * 1000000;
      ctrl->ref.maxw[p] = (int64_t)((num + den - 1) / den);
    }
    ctrl->cap = (int64_t)(((__int128)3 * W + 2 * (__int128)a.C - 1) / (2 * (__int128)a.C));
    ctrl->maxb = maxb0;
    lev[0].n = n;
    lev[0].nnz = nnz;
    lev[0].xadj = xadj;
    lev[0].xend = xadj + 1;
    lev[0].adj = adj0;
    lev[0].w = w0;
    lev[0].vc = vc0;
    lev[0].vg = vg0;
  }
  __syncthreads();
  // ---- coarsening
  int L = 0;
  bool oom = false;
  while (lev[L].n > a.C) {
    const LevelRec f = lev[L];
    int32_t* match = (int32_t*)arena_alloc(a, 4ull * f.n);
    int32_t* cmap = (int32_t*)arena_alloc(a, 4ull * f.n);
    int32_t* cxadj = (int32_t*)arena_alloc(a, 4ull * (f.n + 1));
    int32_t* cxend = (int32_t*)arena_alloc(a, 4ull * f.n);
    int32_t* cadj = (int32_t*)arena_alloc(a, 4ull * f.nnz);
    int64_t* cw = (int64_t*)arena_alloc(a, 8ull * f.nnz);
    int64_t* cvc = (int64_t*)arena_alloc(a, 8ull * f.n);
    int64_t* cvg = (int64_t*)arena_alloc(a, 8ull * f.n);
    if (!match || !cmap || !cxadj || !cxend || !cadj || !cw || !cvc || !cvg) {
      oom = true;
      break;
    }
    LevelView fv;
    fv.n = f.n;
    fv.nnz = f.nnz;
    fv.xadj = f.xadj;
    fv.xend = f.xend;
    fv.adj = f.adj;
    fv.w = f.w;
    fv.b = a.bal ? f.vg : f.vc;
    b_level_reset(ctrl, L > 0, 0, 1);
    __syncthreads();
    const int tw = team_width_dev(f.n, f.nnz, a.tw_shift);
    uint64_t hs = mix64(a.seed ^ (uint64_t)(uint32_t)L);
    {
      // Rounds as in the single-graph path, with one segment: round r >= 1
      // first settles round r - 1 and lists the vertices still free, then
      // only those propose.  Scratch idle during matching holds the free
      // flags (the contraction's row offsets), the two lists and the second
      // proposal buffer (its member arrays and row counts).
      uint8_t* const fr = (uint8_t*)sc.toff;
      int32_t* const lists[2] = {sc.cmem1, sc.cnt};
      int32_t* const pa = sc.prop;
      int32_t* const pb = sc.cmem0;
      __shared__ int32_t s_lcnt[2];
      for (int rr = 0; rr < a.R; rr++) {
        int32_t* const cur = (rr & 1) ? pb : pa;
        const int32_t* const prev = (rr & 1) ? pa : pb;
        if (rr > 0) {
          b_match_free(f.n, match, prev, fr, lists[(rr - 1) & 1], &s_lcnt[(rr - 1) & 1],
                       lists[rr & 1], &s_lcnt[rr & 1], ctrl, rr, 0, 1);
          __syncthreads();
        }
        TW_DISPATCH(tw, (b_match_round<TWv>(fv, match, fr, lists[rr & 1], &s_lcnt[rr & 1], prev,
                                            cur, ctrl, rr, hs, 0, 1)));
        __syncthreads();
      }
      if (a.R > 0) {
        b_match_settle(f.n, match, ((a.R - 1) & 1) ? pb : pa, 0, 1, fr);
        __syncthreads();
      }
    }
    if (a.R == 0) {
      for (int32_t u = threadIdx.x; u < f.n; u += blockDim.x) match[u] = -1;
      __syncthreads();
    }
    // hub flags: the free flags, cleared by the settle (read every row
    // without matching rounds)
    uint8_t* const hflag = a.R > 0 ? (uint8_t*)sc.toff : nullptr;
    TW_DISPATCH(tw, (b_hub<TWv>(fv, match, sc.prop, hs, 0, 1, hflag)));
    __syncthreads();
    TW_DISPATCH(tw, (b_twohop<TWv>(fv, sc.prop, match, ctrl, 0, 1, hflag)));
    __syncthreads();
    const int ntiles = (f.n + kTileV - 1) / kTileV;
    b_iso_count(fv, match, ctrl, sc.tile_lead, ntiles, 0, 1);
    __syncthreads();
    b_iso_list(fv, match, sc.tile_lead, sc.longlist, ntiles, 0, 1);
    __syncthreads();
    b_iso_pair(fv.b, sc.longlist, match, ctrl, 0, 1);
    __syncthreads();
    b_contract_count(fv, match, ctrl, sc.tile_lead, sc.tile_ub, ntiles, nullptr, 0, 1);
    __syncthreads();
    const int ntc = (f.n + kTileC - 1) / kTileC;
    b_contract_map(fv, match, f.vc, f.vg, sc.tile_lead, sc.tile_ub, cmap, cvc, cvg, sc.cmem0,
                   sc.cmem1, sc.toff, ntiles, sc.tile_cnt, ntc, 0, 1);
    __syncthreads();
    // Every coarse row goes straight to its upper-bound offset toff[c] in
    // the coarse arrays and keeps the gap after it (row c is [cxadj[c],
    // cxend[c])).  Rows of at most 16 candidates are merged by 16-lane teams
    // with no barrier between rows; the longer ones are listed (in sc.prop,
    // free after the two-hop pass) for the row sorts, then the longest for
    // the block form.
    {
      __shared__ int32_t s_ndefer;
      __shared__ int64_t s_sio[2];
      b_contract_short<16>(fv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj, cw, sc.cnt,
                           sc.prop, &s_ndefer, s_sio, 0, 1);
      __syncthreads();
      b_contract_rows(fv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj, cw, sc.cnt, sc.tile_cnt,
                      sc.longlist, ctrl, ntc, lds, 0, 1, nullptr, sc.prop, &s_ndefer);
      __syncthreads();
    }
    b_contract_long(fv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj, cw, sc.cnt, nullptr,
                    sc.longlist, ntc, lds, false, 0, 1, false);
    __syncthreads();
    {
      __shared__ int64_t s_tot[kBlock / 64];
      const int32_t nc = ctrl->nc;
      int64_t tot = 0;
      for (int32_t c = threadIdx.x; c < nc; c += kBlock) {
        const int64_t o = sc.toff[c];
        const int32_t k = sc.cnt[c];
        cxadj[c] = (int32_t)o;
        cxend[c] = (int32_t)(o + k);
        tot += k;
      }
      tot = block_sum<kBlock, int64_t>(tot, s_tot);
      if (threadIdx.x == 0) ctrl->nnz_c = (int32_t)tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      lev[L].match = match;
      lev[L].cmap = cmap;
      LevelRec c;
      c.n = ctrl->nc;
      c.nnz = ctrl->nnz_c;
      c.xadj = cxadj;
      c.xend = cxend;
      c.adj = cadj;
      c.w = cw;
      c.vc = cvc;
      c.vg = cvg;
      lev[L + 1] = c;
    }
    __syncthreads();
    L++;
    if (20 * (int64_t)lev[L].n > 19 * (int64_t)lev[L - 1].n || L == kMaxLevels) break;
  }
  // The coarsest level is made compact (n + 1 offsets) for the initial
  // bisection: tile counts, their scan, the rows packed into sc.tmpk/tmpv
  // from the offsets and counts the last contraction left in the scratch,
  // then copied back.
  if (L > 0 && !oom) {
    const int ntc = (lev[L - 1].n + kTileC - 1) / kTileC;
    LevelRec& cl = lev[L];
    b_tile_count(ctrl, sc.cnt, sc.tile_cnt, ntc, 0, 1);
    __syncthreads();
    b_tile_scan(ctrl, sc.tile_cnt, ntc);
    __syncthreads();
    int32_t* cx = const_cast<int32_t*>(cl.xadj);
    int32_t* ca = const_cast<int32_t*>(cl.adj);
    int64_t* cw = const_cast<int64_t*>(cl.w);
    b_contract_compact(ctrl, sc.toff, sc.cnt, sc.tile_cnt, ca, cw, cx, sc.tmpk, sc.tmpv, ntc, 0,
                       1);
    __syncthreads();
    for (int32_t q = threadIdx.x; q < cl.nnz; q += kBlock) {
      ca[q] = sc.tmpk[q];
      cw[q] = sc.tmpv[q];
    }
    if (threadIdx.x == 0) cl.xend = cl.xadj + 1;
    __syncthreads();
  }
  // assignment arrays of every level
  for (int l = 0; l <= L && !oom; l++) {
    int8_t* p = (int8_t*)arena_alloc(a, (uint64_t)lev[l].n);
    if (!p) oom = true;
    else if (threadIdx.x == 0) lev[l].part = p;
    __syncthreads();
  }
  if (oom) {
    write_status(a, g, GP_ENOMEM);
    return;
  }
  // ---- initial bisection on the coarsest level
  {
    const LevelRec cl = lev[L];
    LevelView cv;
    cv.n = cl.n;
    cv.nnz = cl.nnz;
    cv.xadj = cl.xadj;
    cv.xend = cl.xadj + 1;
    cv.adj = cl.adj;
    cv.w = cl.w;
    cv.b = a.bal ? cl.vg : cl.vc;
    const int K = a.K < cl.n ? a.K : cl.n;
    const int gs = a.r0 <= a.r1 ? 0 : 1;
    b_init_tot(cv, ws.tot, 0, 1);
    __syncthreads();
    if (cl.n <= kBatchTrialMax) {
      for (int t = 0; t < K; t++)
        b_trial_lds<kBlock>(cv, ws.tot, K, t, gs, a.P, ctrl, ws.tctl, ws.tpart, ws.tres, lds, sel,
                            srf);
    } else {
      const uint64_t kn = (uint64_t)K * cl.n;
      int8_t* tp = (int8_t*)arena_alloc(a, kn);
      int64_t* tc = (int64_t*)arena_alloc(a, 8 * kn);
      int32_t* ta = (int32_t*)arena_alloc(a, 4 * kn);
      Cand* tl = (Cand*)arena_alloc(a, sizeof(Cand) * kn);
      if (!tp || !tc || !ta || !tl) {
        write_status(a, g, GP_ENOMEM);
        return;
      }
      for (int t = 0; t < K; t++)
        b_trial_global<kBlock>(cv, ws.tot, K, t, gs, a.P, ctrl, ws.tctl, tp, tc, ta, tl, ws.tres,
                               sel);
      b_trial_pick<kBlock>(K, cl.n, ctrl, ws.tctl, tp, ws.tres, cl.part);
    }
    if (cl.n <= kBatchTrialMax) b_trial_pick<kBlock>(K, cl.n, ctrl, ws.tctl, ws.tpart, ws.tres, cl.part);
    __syncthreads();
    if (a.ex.rec) {
      __shared__ long long s_vs, s_es;
      if (threadIdx.x == 0) {
        const uint64_t vs = atomicAdd(a.ex.head_v, (unsigned long long)(cl.n + 1));
        const uint64_t es = atomicAdd(a.ex.head_e, (unsigned long long)cl.nnz);
        const bool ok = vs + cl.n + 1 <= a.ex.cap_v && es + cl.nnz <= a.ex.cap_e;
        s_vs = ok ? (long long)vs : -1;
        s_es = ok ? (long long)es : -1;
        a.ex.rec[4 * g + 0] = cl.n;
        a.ex.rec[4 * g + 1] = cl.nnz;
        a.ex.rec[4 * g + 2] = s_vs;
        a.ex.rec[4 * g + 3] = s_es;
      }
      __syncthreads();
      if (s_vs >= 0) {
        for (int32_t v = threadIdx.x; v <= cl.n; v += kBlock) a.ex.xadj[s_vs + v] = cl.xadj[v];
        for (int32_t v = threadIdx.x; v < cl.n; v += kBlock) {
          a.ex.vwgt[2 * (s_vs + v)] = cl.vc[v];
          a.ex.vwgt[2 * (s_vs + v) + 1] = cl.vg[v];
          a.ex.part[s_vs + v] = cl.part[v];
        }
        for (int32_t q = threadIdx.x; q < cl.nnz; q += kBlock) {
          a.ex.adj[s_es + q] = cl.adj[q];
          a.ex.w[s_es + q] = cl.w[q];
        }
      }
      __syncthreads();
    }
  }
  // ---- uncoarsening with refinement
  // The first pass of a level reads the rows and keeps every vertex's
  // external and internal weight; later passes scan those two arrays, which
  // the moved vertices' rows bring up to date after each pass.  The arrays
  // and the move marks reuse scratch that is idle by now (the contraction's
  // row offsets and counts, the trials' incident totals).
  int64_t* const sext = sc.toff;
  int64_t* const stot = ws.tot;
  int32_t* const mark = sc.cnt;
  __shared__ int64_t s_part[4];
  for (int l = L - 1; l >= 0; l--) {
    const LevelRec f = lev[l];
    b_project(f.n, f.cmap, lev[l + 1].part, f.part, &ctrl->ref, a.P, 0, 1, mark);
    __syncthreads();
    LevelView fv;
    fv.n = f.n;
    fv.nnz = f.nnz;
    fv.xadj = f.xadj;
    fv.xend = f.xend;
    fv.adj = f.adj;
    fv.w = f.w;
    fv.b = a.bal ? f.vg : f.vc;
    const int tw = team_width_dev(f.n, f.nnz, a.tw_shift);
    for (int p = 0; p < a.P; p++) {
      if (p == 0) {
        TW_DISPATCH(tw, (b_refine_gain<TWv>(fv, f.part, &ctrl->ref, sc.list, sel, nullptr, 0, 1,
                                            true, sext, stot)));
      } else {
        b_refine_scan(f.n, f.part, fv.b, nullptr, sext, stot, &ctrl->ref, sc.list, s_part, 0, 1);
        __syncthreads();
        b_refine_decide(f.n, &ctrl->ref, sc.list, s_part, 1, sel);
      }
      __syncthreads();
      b_refine_apply(f.part, &ctrl->ref, sc.list, ws.pass_sink, 0, 1, true, mark);
      __syncthreads();
      TW_DISPATCH(tw, (b_refine_delta<TWv>(fv, f.part, mark, sext, stot, &ctrl->ref, sc.list, p,
                                           0, 1)));
      __syncthreads();
    }
  }
  // ---- result
  const LevelRec l0 = lev[0];
  LevelView v0w;
  v0w.n = l0.n;
  v0w.nnz = l0.nnz;
  v0w.xadj = l0.xadj;
  v0w.xend = l0.xadj + 1;
  v0w.adj = l0.adj;
  v0w.w = l0.w;
  v0w.b = a.bal ? l0.vg : l0.vc;
  b_clear_stats(ctrl, 0, 1);
  __syncthreads();
  const int tw0 = team_width_dev(l0.n, l0.nnz, a.tw_shift);
  TW_DISPATCH(tw0, (b_final_stats<TWv>(v0w, l0.vc, l0.vg, l0.part, ctrl, 0, 1)));
  __syncthreads();
  int8_t* out = a.part + v0;
  for (int32_t v = threadIdx.x; v < n; v += blockDim.x) out[v] = l0.part[v];
  if (threadIdx.x == 0) {
    gp_result r;
    memset(&r, 0, sizeof(r));
    r.cut = ctrl->res_ext / 2;
    r.load[0] = ctrl->res_load[0];
    r.load[1] = ctrl->res_load[1];
    r.time[0] = ctrl->res_time[0];
    r.time[1] = ctrl->res_time[1];
    r.feasible = (r.load[0] <= ctrl->ref.maxw[0] && r.load[1] <= ctrl->ref.maxw[1]) ? 1 : 0;
    r.levels = L;
    r.used_learned = 0;
    r.status = GP_OK;
    a.res[g] = r;
  }
  __syncthreads();
}



// two waves per SIMD: two workgroups share each compute unit (their LDS fits)
__global__ __launch_bounds__(kBlock, 2) void k_batch(BatchArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ SelShared sel;
  __shared__ RefCtl srf;
  __shared__ int s_next;
  const WgScratch ws = wg_scratch(a);
  for (;;) {
    if (threadIdx.x == 0) s_next = (int)atomicAdd(a.head, (uint32_t)a.chunk);
    __syncthreads();
    const int first = s_next;
    __syncthreads();
    if (first >= a.G) break;
    const int last = first + a.chunk < a.G ? first + a.chunk : a.G;
    for (int i = first; i < last; i++) {
      const int g = a.order ? a.order[i] : i;
      int64_t t0 = 0;
      if (a.tline && threadIdx.x == 0) t0 = (int64_t)wall_clock64();
      batch_graph(a, g, ws, lds, &sel, &srf);  // ends with a barrier
      if (a.tline && threadIdx.x == 0) {
        a.tline[2 * g] = t0;
        a.tline[2 * g + 1] = (int64_t)wall_clock64();
      }
    }
  }
}

__global__ void k_batch_reset(uint32_t* head, unsigned long long* arena_off, ExportArgs ex) {
  if (threadIdx.x == 0) {
    *head = 0;
    *arena_off = 0;
    if (ex.rec) {
      *ex.head_v = 0;
      *ex.head_e = 0;
    }
  }
}

}  // namespace gpk

// ===================================================================== host
using namespace gpk;

namespace {

template <class T>
struct HBuf {  // device buffer
  T* p = nullptr;
  size_t cap = 0;
  bool ensure(size_t n) {
    if (n == 0) n = 1;
    if (p && n <= cap) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc((void**)&p, n * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    cap = n;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

struct gp_batch {
  hipStream_t stream = nullptr;
  int nwg = 0;          // persistent workgroups (0: 2 per compute unit)
  int chunk = 1;        // graphs per queue pop
  int order_mode = 0;   // 0: largest first, 1: input order, 2: previous call's longest first
  int tw_shift = 0;     // team width scale, -4 to 1
  HBuf<unsigned char> wgs, arena;
  HBuf<int32_t> order;
  HBuf<int64_t> tline;  // per-graph start / end ticks of the last call
  int32_t tline_g = 0;  // graphs they cover
  HBuf<gp_result> res;
  HBuf<uint32_t> head;
  HBuf<unsigned long long> arena_off;
  gp_result* hres = nullptr;  // pinned
  size_t hres_cap = 0;
  int64_t* hoff = nullptr;    // pinned voff | eoff
  size_t hoff_cap = 0;
  double arena_factor = 3.0;
  ExportArgs ex;        // export of coarsest levels (rec == nullptr: off)
  HBuf<unsigned long long> ex_heads;
  // captured launch
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchArgs cached;
  int cached_nwg = 0;
  bool have_exec = false;
  int cus = 0;
  ~gp_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    wgs.release(); arena.release(); order.release(); tline.release(); res.release();
    head.release();
    arena_off.release();
    ex_heads.release();
    if (hres) (void)hipHostFree(hres);
    if (hoff) (void)hipHostFree(hoff);
  }
};

static gp_status batch_options(const gp_options* o) {
  if (!o) return GP_EINVAL;
  const int64_t lim = (int64_t)1 << 40;
  if (o->ratio[0] < 0 || o->ratio[1] < 0 || o->ratio[0] >= lim || o->ratio[1] >= lim ||
      o->ratio[0] + o->ratio[1] == 0)
    return GP_EINVAL;
  if (o->eps_ppm < 0 || o->eps_ppm > 1000000 || (o->balance_on != 0 && o->balance_on != 1))
    return GP_EINVAL;
  if (o->coarsen_to < 1 || o->match_rounds < 0 || o->match_rounds > kMaxRounds ||
      o->refine_passes < 0 || o->refine_passes > 64 || o->init_trials < 1 || o->init_trials > 64)
    return GP_EINVAL;
  if (o->flags & GP_LEARNED) return GP_EMODEL;
  if (o->flags & (GP_TIME_BALANCE | GP_VOLUME)) return GP_EINVAL;
  return GP_OK;
}

static bool same_args(const BatchArgs& x, const BatchArgs& y) {
  return memcmp(&x, &y, sizeof(BatchArgs)) == 0;
}

// runs the persistent kernel once for the graphs in a.order[0..a.G)
static gp_status batch_launch(gp_batch* b, BatchArgs a, int nwg) {
  hipStream_t s = b->stream;
  const size_t dyn = kBatchLds;
  if (!b->have_exec || !same_args(a, b->cached) || nwg != b->cached_nwg) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->have_exec = false;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return GP_EDEVICE;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      k_batch_reset<<<1, 64, 0, cs>>>(a.head, a.arena_off, a.ex);
      k_batch<<<nwg, kBlock, dyn, cs>>>(a);
      ok = hipStreamEndCapture(cs, &b->graph) == hipSuccess;
    }
    (void)hipStreamDestroy(cs);
    if (!ok || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      return GP_EDEVICE;
    }
    b->cached = a;
    b->cached_nwg = nwg;
    b->have_exec = true;
  }
  if (hipGraphLaunch(b->exec, s) != hipSuccess) {
    (void)hipGetLastError();
    return GP_EDEVICE;
  }
  return GP_OK;
}

extern "C" {

gp_status gp_batch_create(gp_batch** out, void* stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  gp_batch* b = new (std::nothrow) gp_batch();
  if (!b) return GP_ENOMEM;
  b->stream = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete b;
    return GP_EDEVICE;
  }
  if (hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kBatchLds) != hipSuccess)
    (void)hipGetLastError();
  *out = b;
  return GP_OK;
}

void gp_batch_destroy(gp_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  delete b;
}

gp_status gp_batch_export(gp_batch* b, int64_t* rec, int32_t* xadj, int64_t* vwgt, int8_t* part,
                          int64_t cap_vertices, int32_t* adjncy, int64_t* adjwgt,
                          int64_t cap_entries) {
  if (!b) return GP_EINVAL;
  memset(&b->ex, 0, sizeof(b->ex));
  b->have_exec = false;
  if (!rec) return GP_OK;
  if (!xadj || !vwgt || !part || !adjncy || !adjwgt || cap_vertices < 0 || cap_entries < 0)
    return GP_EINVAL;
  if (!b->ex_heads.ensure(2)) return GP_ENOMEM;
  b->ex.rec = rec;
  b->ex.head_v = b->ex_heads.p;
  b->ex.head_e = b->ex_heads.p + 1;
  b->ex.xadj = xadj;
  b->ex.vwgt = vwgt;
  b->ex.part = part;
  b->ex.adj = adjncy;
  b->ex.w = adjwgt;
  b->ex.cap_v = (uint64_t)cap_vertices;
  b->ex.cap_e = (uint64_t)cap_entries;
  return GP_OK;
}

gp_status gp_batch_team_width(gp_batch* b, int32_t shift) {
  if (!b || shift < -4 || shift > 1) return GP_EINVAL;
  b->tw_shift = shift;
  return GP_OK;
}

gp_status gp_batch_config(gp_batch* b, int32_t workgroups, int32_t chunk, int32_t order_mode) {
  if (!b || workgroups < 0 || chunk < 1 || chunk > 64 || order_mode < 0 || order_mode > 2)
    return GP_EINVAL;
  b->nwg = workgroups;
  b->chunk = chunk;
  b->order_mode = order_mode;
  return GP_OK;
}

gp_status gp_partition_batch(gp_batch* b, int32_t G, const int64_t* voff, const int64_t* eoff,
                             const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                             const int64_t* vwgt, const gp_options* o, int8_t* part,
                             gp_result* res) {
  if (!b || G < 0 || (G > 0 && (!voff || !eoff || !xadj || !vwgt || !part || !res)))
    return GP_EINVAL;
  gp_status st = batch_options(o);
  if (st != GP_OK) return st;
  if (G == 0) return GP_OK;
  hipStream_t s = b->stream;
  // offsets to the host
  const size_t need = 2 * ((size_t)G + 1);
  if (b->hoff_cap < need) {
    if (b->hoff) (void)hipHostFree(b->hoff);
    b->hoff = nullptr;
    b->hoff_cap = 0;
    if (hipHostMalloc((void**)&b->hoff, need * sizeof(int64_t), hipHostMallocDefault) !=
        hipSuccess)
      return GP_ENOMEM;
    b->hoff_cap = need;
  }
  int64_t* hv = b->hoff;
  int64_t* he = b->hoff + G + 1;
  if (hipMemcpyAsync(hv, voff, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(he, eoff, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GP_EDEVICE;
  if (hv[0] != 0 || he[0] != 0) return GP_EINVAL;
  int64_t nmax = 0, nnzmax = 0;
  for (int g = 0; g < G; g++) {
    const int64_t ng = hv[g + 1] - hv[g], mg = he[g + 1] - he[g];
    if (ng < 0 || mg < 0 || ng > INT32_MAX || mg > INT32_MAX) return GP_EINVAL;
    nmax = ng > nmax ? ng : nmax;
    nnzmax = mg > nnzmax ? mg : nnzmax;
  }
  const int64_t ntot = hv[G], mtot = he[G];
  if ((ntot > 0 && !adjncy && mtot > 0) || (mtot > 0 && !adjwgt)) return GP_EINVAL;
  // processing order: largest graphs first, input order, or the longest
  // graphs of the previous call on this context first (longest processing
  // time first: the timeline tells which graphs are slow, e.g. those whose
  // coarsening stalls; without a previous call of G graphs, largest first)
  std::vector<int32_t> ord(G);
  std::iota(ord.begin(), ord.end(), 0);
  if (b->order_mode == 2 && b->tline_g == G && G > 0) {
    std::vector<int64_t> t(2 * (size_t)G);
    if (hipMemcpyAsync(t.data(), b->tline.p, sizeof(int64_t) * 2 * (size_t)G,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return GP_EDEVICE;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
      return t[2 * x + 1] - t[2 * x] > t[2 * y + 1] - t[2 * y];
    });
  } else if (b->order_mode != 1) {
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
      return (he[x + 1] - he[x]) + (hv[x + 1] - hv[x]) > (he[y + 1] - he[y]) + (hv[y + 1] - hv[y]);
    });
  }
  const int nwg = b->nwg > 0 ? b->nwg : 2 * (b->cus > 0 ? b->cus : 256);
  uint64_t offs[32];
  const uint64_t stride = wg_layout((int32_t)nmax, (int32_t)nnzmax, offs);
  const uint64_t arena_bytes =
      (uint64_t)(b->arena_factor * (double)(ntot * 57 + mtot * 12)) + (uint64_t)G * 8192 + (1 << 20);
  if (!b->wgs.ensure((size_t)stride * nwg) || !b->arena.ensure(arena_bytes) ||
      !b->order.ensure(G) || !b->tline.ensure(2 * (size_t)G) || !b->res.ensure(G) ||
      !b->head.ensure(1) || !b->arena_off.ensure(1))
    return GP_ENOMEM;
  if (b->hres_cap < (size_t)G) {
    if (b->hres) (void)hipHostFree(b->hres);
    b->hres = nullptr;
    b->hres_cap = 0;
    if (hipHostMalloc((void**)&b->hres, sizeof(gp_result) * G, hipHostMallocDefault) != hipSuccess)
      return GP_ENOMEM;
    b->hres_cap = G;
  }
  if (hipMemcpyAsync(b->order.p, ord.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return GP_EDEVICE;
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.G = G;
  a.voff = voff;
  a.eoff = eoff;
  a.xadj = xadj;
  a.adj = adjncy;
  a.w = adjwgt;
  a.vwgt = vwgt;
  a.order = b->order.p;
  a.part = part;
  a.res = b->res.p;
  a.r0 = o->ratio[0];
  a.r1 = o->ratio[1];
  a.eps = o->eps_ppm;
  a.bal = o->balance_on;
  a.seed = o->seed;
  a.C = o->coarsen_to;
  a.R = o->match_rounds;
  a.P = o->refine_passes;
  a.K = o->init_trials;
  a.head = b->head.p;
  a.arena = b->arena.p;
  a.arena_cap = b->arena.cap;
  a.arena_off = b->arena_off.p;
  a.wgs = b->wgs.p;
  a.wgs_stride = stride;
  a.nmax = (int32_t)nmax;
  a.nnzmax = (int32_t)nnzmax;
  a.chunk = b->chunk;
  a.ex = b->ex;
  a.tline = b->tline.p;
  a.tw_shift = b->tw_shift;
  b->tline_g = 0;
  if ((st = batch_launch(b, a, nwg)) != GP_OK) return st;
  if (hipMemcpyAsync(b->hres, b->res.p, sizeof(gp_result) * G, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GP_EDEVICE;
  // graphs that ran out of arena: rerun them alone with a larger arena
  for (int attempt = 0; attempt < 4; attempt++) {
    std::vector<int32_t> redo;
    for (int g = 0; g < G; g++)
      if (b->hres[g].status == GP_ENOMEM) redo.push_back(g);
    if (redo.empty()) break;
    b->arena_factor *= 2.0;
    const uint64_t nb = (uint64_t)(b->arena_factor * (double)(ntot * 57 + mtot * 12)) +
                        (uint64_t)G * 8192 + (1 << 20);
    if (!b->arena.ensure(nb)) return GP_ENOMEM;
    if (hipMemcpyAsync(b->order.p, redo.data(), sizeof(int32_t) * redo.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      return GP_EDEVICE;
    BatchArgs a2 = a;
    a2.G = (int32_t)redo.size();
    a2.arena = b->arena.p;
    a2.arena_cap = b->arena.cap;
    if ((st = batch_launch(b, a2, nwg)) != GP_OK) return st;
    if (hipMemcpyAsync(b->hres, b->res.p, sizeof(gp_result) * G, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return GP_EDEVICE;
  }
  memcpy(res, b->hres, sizeof(gp_result) * G);
  b->tline_g = G;
  return GP_OK;
}

gp_status gp_batch_timeline(gp_batch* b, int32_t G, int64_t* ticks, int64_t* hz) {
  if (!b || G < 0 || G > b->tline_g || (G > 0 && !ticks)) return GP_EINVAL;
  if (hz) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
      (void)hipGetLastError();
      return GP_EDEVICE;
    }
    *hz = (int64_t)khz * 1000;
  }
  if (G > 0 && (hipMemcpyAsync(ticks, b->tline.p, sizeof(int64_t) * 2 * (size_t)G,
                               hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
                hipStreamSynchronize(b->stream) != hipSuccess)) {
    (void)hipGetLastError();
    return GP_EDEVICE;
  }
  return GP_OK;
}

gp_status gp_batch_autotune(gp_batch* b, int32_t G, const int64_t* voff, const int64_t* eoff,
                            const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                            const int64_t* vwgt, const gp_options* o, int8_t* part,
                            gp_result* res, int32_t reps, int32_t* chosen, double* ms) {
  if (!b || reps < 1 || G < 0) return GP_EINVAL;
  if (G == 0) return gp_partition_batch(b, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, o, part, res);
  if (!voff || !part || !res) return GP_EINVAL;
  const int keep[4] = {b->nwg, b->chunk, b->order_mode, b->tw_shift};
  int64_t ntot = 0;
  if (hipMemcpy(&ntot, voff + G, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return GP_EDEVICE;
  if (ntot < 0) return GP_EINVAL;
  const int cus = b->cus > 0 ? b->cus : 256;
  // persistent workgroups per compute unit (two fit by LDS and registers) x
  // graphs per queue pop x queue order (order 2 uses the timeline of the
  // configuration run just before it); then the best of these with the team
  // width divided by 16, 8, 4 and 2, and doubled
  std::vector<int> cand;
  for (int per_cu : {1, 2})
    for (int chunk : {1, 2, 4})
      for (int order : {0, 1, 2}) cand.insert(cand.end(), {per_cu * cus, chunk, order, 0});
  const size_t n1 = cand.size() / 4;
  std::vector<int8_t> ref_part((size_t)ntot), cur_part((size_t)ntot);
  std::vector<gp_result> ref_res((size_t)G), cur_res((size_t)G);
  double best = 1e300;
  size_t best_i = 0;
  gp_status st = GP_OK;
  for (size_t i = 0; i < cand.size() / 4 && st == GP_OK; i++) {
    b->nwg = cand[4 * i];
    b->chunk = cand[4 * i + 1];
    b->order_mode = cand[4 * i + 2];
    b->tw_shift = cand[4 * i + 3];
    // the first call of a configuration captures its graph; it is not timed
    st = gp_partition_batch(b, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, o, part,
                            i == 0 ? ref_res.data() : cur_res.data());
    if (st != GP_OK) break;
    if (hipMemcpy(i == 0 ? ref_part.data() : cur_part.data(), part, (size_t)ntot,
                  hipMemcpyDeviceToHost) != hipSuccess) {
      st = GP_EDEVICE;
      break;
    }
    if (i > 0 && (memcmp(ref_part.data(), cur_part.data(), (size_t)ntot) != 0 ||
                  memcmp(ref_res.data(), cur_res.data(), sizeof(gp_result) * G) != 0)) {
      st = GP_EDEVICE;  // a configuration changed a result: never expected
      break;
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps && st == GP_OK; r++)
      st = gp_partition_batch(b, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, o, part,
                              cur_res.data());
    const double t =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
        reps;
    if (st == GP_OK && t < best) {
      best = t;
      best_i = i;
    }
    if (i + 1 == n1)  // second stage: the team width of the best so far
      for (int sh : {-4, -3, -2, -1, 1})
        cand.insert(cand.end(), {cand[4 * best_i], cand[4 * best_i + 1], cand[4 * best_i + 2], sh});
  }
  if (st != GP_OK) {
    b->nwg = keep[0];
    b->chunk = keep[1];
    b->order_mode = keep[2];
    b->tw_shift = keep[3];
    return st;
  }
  b->nwg = cand[4 * best_i];
  b->chunk = cand[4 * best_i + 1];
  b->order_mode = cand[4 * best_i + 2];
  b->tw_shift = cand[4 * best_i + 3];
  if (chosen) {
    chosen[0] = b->nwg;
    chosen[1] = b->chunk;
    chosen[2] = b->order_mode;
    chosen[3] = b->tw_shift;
  }
  if (ms) *ms = best;
  // leave the caller the chosen configuration's (identical) outputs
  st = gp_partition_batch(b, G, voff, eoff, xadj, adjncy, adjwgt, vwgt, o, part, res);
  return st;
}

// ------------------------------------------------ allocation-free batch
// Device scratch of gp_partition_batch_noalloc: one fixed array per GPU
// (the code object's own copy on each device), held until the process ends.
// Host code never uses the array's name as an address: the device address
// comes from hipGetSymbolAddress, once per device.
constexpr uint64_t kNoAllocBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoAllocDevices];
int g_noalloc_cus[kNoAllocDevices];

// the current device's scratch address and compute-unit count
gp_status noalloc_setup(unsigned char** ptr, int* cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) {
    (void)hipGetLastError();
    return GP_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    int n = 0;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kBatchLds) != hipSuccess) {
      (void)hipGetLastError();
      return GP_EDEVICE;
    }
    g_noalloc_ptr[dev] = (unsigned char*)p;
    g_noalloc_cus[dev] = n > 0 ? n : 256;
  }
  *ptr = g_noalloc_ptr[dev];
  *cus = g_noalloc_cus[dev];
  return GP_OK;
}
}  // namespace

gp_status gp_partition_batch_noalloc(int32_t G, const int64_t* voff, const int64_t* eoff,
                                     const int32_t* xadj, const int32_t* adjncy,
                                     const int64_t* adjwgt, const int64_t* vwgt,
                                     const gp_options* o, int32_t nmax, int32_t nnzmax,
                                     int64_t ntot, int64_t nnztot, int8_t* part,
                                     gp_result* res, void* stream) {
  if (G < 0 || nmax < 0 || nnzmax < 0 || ntot < 0 || nnztot < 0 ||
      (G > 0 && (!voff || !eoff || !xadj || !vwgt || !part || !res)) ||
      (nnztot > 0 && (!adjncy || !adjwgt)))
    return GP_EINVAL;
  gp_status st = batch_options(o);
  if (st != GP_OK) return st;
  if (G == 0) return GP_OK;
  unsigned char* base = nullptr;
  int cus = 0;
  if ((st = noalloc_setup(&base, &cus)) != GP_OK) return st;
  // layout: queue head, arena offset, per-workgroup scratch, arena
  uint64_t offs[32];
  const uint64_t stride = wg_layout(nmax, nnzmax, offs);
  // the levels of every graph stay in the arena until the launch ends and
  // there is no rerun here, so the arena keeps twice the first estimate of
  // gp_partition_batch when it can (fewer workgroups leave it more room)
  const uint64_t arena_est =
      (uint64_t)(3.0 * (double)(ntot * 57 + nnztot * 12)) + (uint64_t)G * 8192 + (1 << 20);
  const uint64_t head_bytes = 512;
  int nwg = 2 * cus < G ? 2 * cus : G;
  while (nwg > 1 && head_bytes + (uint64_t)nwg * stride + 2 * arena_est > kNoAllocBytes) nwg--;
  if (head_bytes + (uint64_t)nwg * stride + arena_est > kNoAllocBytes) return GP_ENOMEM;
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.G = G;
  a.voff = voff;
  a.eoff = eoff;
  a.xadj = xadj;
  a.adj = adjncy;
  a.w = adjwgt;
  a.vwgt = vwgt;
  a.order = nullptr;  // input order
  a.part = part;
  a.res = res;
  a.r0 = o->ratio[0];
  a.r1 = o->ratio[1];
  a.eps = o->eps_ppm;
  a.bal = o->balance_on;
  a.seed = o->seed;
  a.C = o->coarsen_to;
  a.R = o->match_rounds;
  a.P = o->refine_passes;
  a.K = o->init_trials;
  a.head = (uint32_t*)base;
  a.arena_off = (unsigned long long*)(base + 256);
  a.wgs = base + head_bytes;
  a.wgs_stride = stride;
  a.arena = base + head_bytes + (uint64_t)nwg * stride;
  a.arena_cap = kNoAllocBytes - head_bytes - (uint64_t)nwg * stride;
  a.nmax = nmax;
  a.nnzmax = nnzmax;
  a.chunk = 1;
  hipStream_t s = (hipStream_t)stream;
  // the queue head and the arena offset start at zero: a fill kernel, no
  // memset node, so that the two launches can be captured in a graph
  k_batch_reset<<<1, 64, 0, s>>>(a.head, a.arena_off, a.ex);
  k_batch<<<nwg, kBlock, kBatchLds, s>>>(a);
  if (hipGetLastError() != hipSuccess) return GP_EDEVICE;
  return GP_OK;
}

}  // extern "C"
