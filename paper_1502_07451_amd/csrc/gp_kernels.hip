// gp_kernels.hip - gfx950 kernels of the single-graph path and their launchers.
//
// Per level of the multilevel hierarchy:
//   matching    k_match_round (R rounds; from the second on, k_match_free
//               settles the previous one first), k_match_settle, k_hub,
//               k_twohop, k_iso_count / k_iso_list /
//               k_iso_pair
//   contraction k_contract_count -> k_contract_map -> k_contract_short
//               (rows of <= 32 candidates) -> k_contract_rows
//               -> k_contract_long (one wave per row) -> k_contract_huge
//               (one block per row) -> k_contract_ends; rows stay at their
//               upper-bound offsets, and only the coarsest level is made
//               compact (k_tile_scan -> k_contract_compact)
// at the coarsest level
//   initial bisection k_init_tot -> k_init_trials_lds (one trial per block)
// per level on the way back up
//   k_project, then P x (k_refine_gain -> k_refine_settle) on levels of at
//   most 65,536 vertices, P x (k_refine_gain -> k_refine_decide ->
//   k_refine_apply -> k_refine_finish) on larger ones
// and once at level 0 k_final_stats.  gp_create's checks: k_val_*, k_sort_*.
// The kernels are thin wrappers of the bodies in gp_phases.h.
#include <stdlib.h>

#include "gp_launch.h"
#include "gp_phases.h"

namespace gpk {

static int grid_for(int64_t items, int per_block, int cap = 4096) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__global__ void k_level_reset(Ctrl* ctrl, int promote) {
  b_level_reset(ctrl, promote, (int)blockIdx.x, (int)gridDim.x);
}

// one block per segment of the vertex range (see b_match_free)
template <int TW>
__global__ __launch_bounds__(kBlock) void k_match_round(LevelView lv, int32_t* match,
                                                        const uint8_t* fr, const int32_t* list,
                                                        const int32_t* lcnt,
                                                        const int32_t* prop_prev,
                                                        int32_t* prop_cur, Ctrl* ctrl,
                                                        int round, uint64_t hs) {
  b_match_round<TW>(lv, match, fr, list, lcnt, prop_prev, prop_cur, ctrl, round, hs,
                    (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_match_free(int32_t n, int32_t* match,
                                                       const int32_t* prop_prev, uint8_t* fr,
                                                       const int32_t* lin, const int32_t* cin,
                                                       int32_t* lout, int32_t* cout, Ctrl* ctrl,
                                                       int round) {
  b_match_free(n, match, prop_prev, fr, lin, cin, lout, cout, ctrl, round, (int)blockIdx.x,
               (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_match_settle(int32_t n, int32_t* match,
                                                         const int32_t* prop, uint8_t* hflag) {
  b_match_settle(n, match, prop, (int)blockIdx.x, (int)gridDim.x, hflag);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_hub(LevelView lv, const int32_t* match, int32_t* hub,
                                                uint64_t hs, uint8_t* hflag) {
  b_hub<TW>(lv, match, hub, hs, (int)blockIdx.x, (int)gridDim.x, hflag);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_twohop(LevelView lv, const int32_t* hub,
                                                   int32_t* match, const Ctrl* ctrl,
                                                   const uint8_t* hflag) {
  b_twohop<TW>(lv, hub, match, ctrl, (int)blockIdx.x, (int)gridDim.x, hflag);
}

__global__ __launch_bounds__(kBlock) void k_iso_count(LevelView lv, const int32_t* match,
                                                      Ctrl* ctrl, int32_t* tile_cnt,
                                                      int ntiles) {
  b_iso_count(lv, match, ctrl, tile_cnt, ntiles, (int)blockIdx.x, (int)gridDim.x, false);
}

__global__ __launch_bounds__(kBlock) void k_iso_scan(Ctrl* ctrl, int32_t* tile_cnt, int ntiles) {
  b_iso_scan(ctrl, tile_cnt, ntiles);
}

__global__ __launch_bounds__(kBlock) void k_iso_list(LevelView lv, const int32_t* match,
                                                     const int32_t* tile_base, int32_t* iso,
                                                     int ntiles) {
  b_iso_list(lv, match, tile_base, iso, ntiles, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_iso_pair(const int64_t* b, const int32_t* iso,
                                                     int32_t* match, const Ctrl* ctrl) {
  b_iso_pair(b, iso, match, ctrl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_contract_count(LevelView lv, const int32_t* match,
                                                           Ctrl* ctrl, int32_t* tile_lead,
                                                           int64_t* tile_ub, int ntiles,
                                                           int64_t* partials) {
  b_contract_count(lv, match, ctrl, tile_lead, tile_ub, ntiles, partials, (int)blockIdx.x,
                   (int)gridDim.x, false);
}

__global__ __launch_bounds__(kBlock) void k_contract_scan(Ctrl* ctrl, int32_t* tile_lead,
                                                          int64_t* tile_ub, int ntiles,
                                                          const int64_t* partials, int nparts) {
  b_contract_scan(ctrl, tile_lead, tile_ub, ntiles, partials, nparts);
}

__global__ __launch_bounds__(kBlock) void k_contract_map(LevelView lv, const int32_t* match,
                                                         const int64_t* vc, const int64_t* vg,
                                                         const int32_t* tile_lead,
                                                         const int64_t* tile_ub, int32_t* cmap,
                                                         int64_t* cvc, int64_t* cvg,
                                                         int32_t* cmem0, int32_t* cmem1,
                                                         int64_t* toff, int ntiles,
                                                         int64_t* tile_cnt, int ntiles_c) {
  b_contract_map(lv, match, vc, vg, tile_lead, tile_ub, cmap, cvc, cvg, cmem0, cmem1, toff, ntiles,
                 tile_cnt, ntiles_c, (int)blockIdx.x, (int)gridDim.x);
}

// one block per segment of the coarse rows (see b_contract_short)
__global__ __launch_bounds__(kBlock) void k_contract_short(LevelView lv, const int32_t* cmap,
                                                           const int32_t* cmem0,
                                                           const int32_t* cmem1,
                                                           const int64_t* toff,
                                                           const Ctrl* ctrl, int32_t* okey,
                                                           int64_t* oval, int32_t* cnt,
                                                           int32_t* defer, int32_t* dcnt,
                                                           int64_t* sio) {
  b_contract_short(lv, cmap, cmem0, cmem1, toff, ctrl, okey, oval, cnt, defer, dcnt, sio,
                   (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_contract_sums(Ctrl* ctrl, const int32_t* dcnt,
                                                          const int64_t* sio, int nseg) {
  b_contract_sums(ctrl, dcnt, sio, nseg);
}

// the rows the short-row kernel listed, block k taking segment k's, 16 at a
// time (the same grid as k_contract_short).  Five blocks per compute unit:
// the register cap (96) that this asks for keeps five of the 25 KB LDS
// regions busy instead of four (113 registers), which hides more of the
// gather latency (3.38 -> 3.10 ms per 4M-vertex partition; six blocks, at
// 80 registers, spill).
__global__ __launch_bounds__(kBlock, 5) void k_contract_rows(
    LevelView lv, const int32_t* cmap, const int32_t* cmem0, const int32_t* cmem1,
    const int64_t* toff, const Ctrl* ctrl, int32_t* tmpk, int64_t* tmpv, int32_t* cnt,
    int64_t* tile_cnt, int32_t* longlist, Ctrl* wctrl, int ntiles_c, int32_t* hugelist,
    const int32_t* rowlist, const int32_t* rowcnt) {
  __shared__ __align__(16) unsigned char lds[kRowBlockCap * 12];
  b_contract_rows(lv, cmap, cmem0, cmem1, toff, ctrl, tmpk, tmpv, cnt, tile_cnt, longlist, wctrl,
                  ntiles_c, lds, (int)blockIdx.x, (int)gridDim.x, hugelist, rowlist, rowcnt);
}

// per-tile entry counts of the coarse rows (for the compaction's scan)
__global__ __launch_bounds__(kBlock) void k_tile_count(const Ctrl* ctrl, const int32_t* cnt,
                                                       int64_t* tile_cnt, int ntiles_c) {
  b_tile_count(ctrl, cnt, tile_cnt, ntiles_c, (int)blockIdx.x, (int)gridDim.x);
}

// one wave per long row (packed-key sort in the wave's 16 KB of LDS)
__global__ __launch_bounds__(64) void k_contract_long(LevelView lv, const int32_t* cmap,
                                                      const int32_t* cmem0, const int32_t* cmem1,
                                                      const int64_t* toff, Ctrl* ctrl,
                                                      int32_t* tmpk, int64_t* tmpv, int32_t* cnt,
                                                      int64_t* tile_cnt,
                                                      const int32_t* longlist) {
  __shared__ int32_t sk[kLongWave];
  b_contract_longw(lv, cmap, cmem0, cmem1, toff, ctrl, tmpk, tmpv, cnt, tile_cnt, longlist, sk,
                   (int)blockIdx.x, (int)gridDim.x);
}

// one block per row of more than kLongCap candidates (or on a level whose
// coarse ids do not fit a packed key)
__global__ __launch_bounds__(kBlock) void k_contract_huge(LevelView lv, const int32_t* cmap,
                                                          const int32_t* cmem0,
                                                          const int32_t* cmem1,
                                                          const int64_t* toff, Ctrl* ctrl,
                                                          int32_t* tmpk, int64_t* tmpv,
                                                          int32_t* cnt, int64_t* tile_cnt,
                                                          const int32_t* hugelist,
                                                          int ntiles_c) {
  extern __shared__ __align__(16) unsigned char dyn_long[];
  b_contract_long(lv, cmap, cmem0, cmem1, toff, ctrl, tmpk, tmpv, cnt, tile_cnt, hugelist,
                  ntiles_c, dyn_long, true, (int)blockIdx.x, (int)gridDim.x, false, true);
}

__global__ __launch_bounds__(kBlock) void k_tile_scan(Ctrl* ctrl, int64_t* tile_cnt, int ntiles_c) {
  b_tile_scan(ctrl, tile_cnt, ntiles_c);
}

// Begin and end of every coarse row (a row stays where its upper-bound
// offset put it) and the level's entry count.
__global__ __launch_bounds__(kBlock) void k_contract_ends(Ctrl* ctrl, const int64_t* toff,
                                                          const int32_t* cnt, int32_t* cxadj,
                                                          int32_t* cxend) {
  __shared__ int64_t sml[kBlock / 64];
  const int32_t nc = ctrl->nc;
  int64_t sum = 0;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * kBlock) {
    const int32_t b = (int32_t)toff[c], k = cnt[c];
    cxadj[c] = b;
    cxend[c] = b + k;
    sum += k;
  }
  sum = block_sum<kBlock, int64_t>(sum, sml);
  if (threadIdx.x == 0 && sum) atomicAdd(&ctrl->nnz_c, (int32_t)sum);
  if (blockIdx.x == 0 && threadIdx.x == 0) cxadj[nc] = (int32_t)ctrl->ubtot;
}

__global__ __launch_bounds__(kBlock) void k_contract_compact(const Ctrl* ctrl,
                                                             const int64_t* toff,
                                                             const int32_t* cnt,
                                                             const int64_t* tile_base,
                                                             const int32_t* tmpk,
                                                             const int64_t* tmpv, int32_t* cxadj,
                                                             int32_t* cadj, int64_t* cw,
                                                             int ntiles_c) {
  b_contract_compact(ctrl, toff, cnt, tile_base, tmpk, tmpv, cxadj, cadj, cw, ntiles_c, (int)blockIdx.x, (int)gridDim.x);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_refine_gain(LevelView lv, const int8_t* part,
                                                        RefCtl* rc, Cand* list,
                                                        int64_t* partials, int64_t* sext,
                                                        int64_t* stot, const int64_t* b1) {
  __shared__ SelShared sel;
  b_refine_gain<TW>(lv, part, rc, list, &sel, partials, (int)blockIdx.x, (int)gridDim.x, false,
                    sext, stot, b1);
}

__global__ __launch_bounds__(kBlock) void k_refine_scan(int32_t n, const int8_t* part,
                                                        const int64_t* b, const int64_t* b1,
                                                        const int64_t* sext, const int64_t* stot,
                                                        RefCtl* rc, Cand* list,
                                                        int64_t* partials) {
  b_refine_scan(n, part, b, b1, sext, stot, rc, list, partials, (int)blockIdx.x,
                (int)gridDim.x);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_refine_delta(LevelView lv, const int8_t* part,
                                                         const int32_t* mark, int64_t* sext,
                                                         int64_t* stot, const RefCtl* rc,
                                                         const Cand* list, int p) {
  b_refine_delta<TW>(lv, part, mark, sext, stot, rc, list, p, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_refine_decide(int32_t n, RefCtl* rc, const Cand* list,
                                                          const int64_t* partials, int nparts) {
  __shared__ SelShared sel;
  b_refine_decide(n, rc, list, partials, nparts, &sel);
}

__global__ __launch_bounds__(kBlock) void k_refine_apply(int8_t* part, RefCtl* rc,
                                                         const Cand* list, int32_t* pass_out,
                                                         int32_t* mark) {
  b_refine_apply(part, rc, list, pass_out, (int)blockIdx.x, (int)gridDim.x, false, mark);
}

__global__ void k_refine_finish(RefCtl* rc, int32_t* pass_out) { b_refine_finish(rc, pass_out); }

__global__ __launch_bounds__(kBlock) void k_refine_settle(int32_t n, int8_t* part, RefCtl* rc,
                                                          const Cand* list,
                                                          const int64_t* partials, int nparts,
                                                          int32_t* pass_out, int32_t* mark) {
  __shared__ SelShared sel;
  b_refine_settle(n, part, rc, list, partials, nparts, &sel, pass_out, mark);
}

__global__ __launch_bounds__(kBlock) void k_project(int32_t n, const int32_t* cmap,
                                                    const int8_t* cpart, int8_t* part, RefCtl* rc,
                                                    int npass, int32_t* mark) {
  b_project(n, cmap, cpart, part, rc, npass, (int)blockIdx.x, (int)gridDim.x, mark);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_vol_out(LevelView lv, int64_t* out) {
  b_vol_out<TW>(lv, out, (int)blockIdx.x, (int)gridDim.x);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_vol_count(LevelView lv, const int8_t* part,
                                                      int32_t* cnt) {
  b_vol_count<TW>(lv, part, cnt, (int)blockIdx.x, (int)gridDim.x);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_vol_gain(LevelView lv, const int8_t* part,
                                                     const int64_t* out, const int32_t* cnt,
                                                     RefCtl* rc, Cand* list, int64_t* partials) {
  b_vol_gain<TW>(lv, part, out, cnt, rc, list, partials, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_vol_reset(Ctrl* ctrl) {
  if (threadIdx.x == 0) ctrl->res_vol = 0;
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_vol_total(LevelView lv, const int8_t* part,
                                                      const int64_t* out, Ctrl* ctrl) {
  b_vol_total<TW>(lv, part, out, &ctrl->res_vol, (int)blockIdx.x, (int)gridDim.x);
}

// time balance: the loads become (CPU cost of side 0, GPU cost of side 1),
// taken from the statistics kernel, with their own bounds; a new pass sequence
__global__ void k_time_bounds(Ctrl* ctrl, int64_t maxw0, int64_t maxw1, int npass) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    RefCtl* rc = &ctrl->ref;
    rc->pw[0] = ctrl->res_time[0];
    rc->pw[1] = ctrl->res_time[1];
    rc->maxw[0] = maxw0;
    rc->maxw[1] = maxw1;
    start_level(rc, npass);
  }
}

__global__ void k_start_level(RefCtl* rc, int npass) {
  b_start_level(rc, npass, (int)blockIdx.x, (int)gridDim.x);
}

template <int TW>
__global__ __launch_bounds__(kBlock) void k_final_stats(LevelView lv, const int64_t* vc,
                                                        const int64_t* vg, const int8_t* part,
                                                        Ctrl* ctrl, int64_t* partials) {
  b_final_stats<TW>(lv, vc, vg, part, ctrl, (int)blockIdx.x, (int)gridDim.x, partials);
}

__global__ __launch_bounds__(kBlock) void k_final_reduce(Ctrl* ctrl, const int64_t* partials,
                                                         int nparts) {
  b_final_reduce(ctrl, partials, nparts);
}

__global__ void k_clear_stats(Ctrl* ctrl) {
  b_clear_stats(ctrl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_init_tot(LevelView lv, int64_t* tot) {
  b_init_tot(lv, tot, (int)blockIdx.x, (int)gridDim.x);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_init_trials(LevelView lv, const int64_t* tot, int K,
                                                    int gs, int npass, Ctrl* ctrl, RefCtl* tctl,
                                                    int8_t* tpart, int64_t* tconn,
                                                    int32_t* tadj, Cand* tlist, int64_t* tres,
                                                    int8_t* out_part) {
  __shared__ SelShared sel;
  b_trial_global<BS>(lv, tot, K, (int)blockIdx.x, gs, npass, ctrl, tctl, tpart, tconn, tadj, tlist,
                     tres, &sel);
  if (!last_block(&ctrl->ctr_init, gridDim.x)) return;
  b_trial_pick<BS>(K, lv.n, ctrl, tctl, tpart, tres, out_part);
}

template <int BS, bool kLongRows>
__global__ __launch_bounds__(BS) void k_init_trials_lds(LevelView lv, const int64_t* tot, int K,
                                                        int gs, int npass, Ctrl* ctrl,
                                                        RefCtl* tctl, int8_t* tpart,
                                                        int64_t* tres, int8_t* out_part) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ SelShared sel;
  __shared__ RefCtl srf;
  b_trial_lds<BS, kLongRows>(lv, tot, K, (int)blockIdx.x, gs, npass, ctrl, tctl, tpart, tres,
                             dyn_lds, &sel, &srf);
  if (!last_block(&ctrl->ctr_init, gridDim.x)) return;
  b_trial_pick<BS>(K, lv.n, ctrl, tctl, tpart, tres, out_part);
}

__global__ __launch_bounds__(kBlock) void k_val_xadj(int32_t n, const int32_t* xadj, Ctrl* ctrl) {
  b_val_xadj(n, xadj, ctrl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_val_rows(int32_t n, const int32_t* xadj,
                                                     const int32_t* adj, const int64_t* w,
                                                     const int64_t* vc, const int64_t* vg,
                                                     Ctrl* ctrl) {
  b_val_rows(n, xadj, adj, w, vc, vg, ctrl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_sort_rows(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl) {
  __shared__ __align__(16) unsigned char lds[kSortCap * 12];
  b_sort_rows(n, xadj, adj, w, oadj, ow, ctrl, lds, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_sort_long(int32_t n, const int32_t* xadj,
                                                      const int32_t* adj, const int64_t* w,
                                                      int32_t* oadj, int64_t* ow, Ctrl* ctrl) {
  extern __shared__ __align__(16) unsigned char dyn_sl[];
  b_sort_long(n, xadj, adj, w, oadj, ow, ctrl, dyn_sl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_val_sym(int32_t n, const int32_t* xadj,
                                                    const int32_t* adj, const int64_t* w,
                                                    Ctrl* ctrl) {
  b_val_sym(n, xadj, adj, w, ctrl, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg) {
  b_split_vwgt(n, vwgt, vc, vg, (int)blockIdx.x, (int)gridDim.x);
}

// ================================================================ profiling
const char* const kProfNames[PK_N] = {
    "k_match_round", "k_match_free", "k_match_settle", "k_hub", "k_twohop", "k_iso",
    "k_contract_count",
    "k_contract_map", "k_contract_short", "k_contract_rows", "k_contract_long", "k_contract_huge",
    "k_contract_compact", "k_init_tot",
    "k_init_trials", "k_refine_gain", "k_refine_scan", "k_refine_delta", "k_refine_settle",
    "k_refine_apply", "k_project", "k_final_stats"};

thread_local Prof* g_prof = nullptr;

static hipEvent_t prof_event(Prof* p) {
  if (p->used >= p->npool) {
    const int ncap = p->npool ? 2 * p->npool : 256;
    hipEvent_t* np = (hipEvent_t*)realloc(p->pool, sizeof(hipEvent_t) * ncap);
    if (!np) return nullptr;
    p->pool = np;
    for (int i = p->npool; i < ncap; i++)
      if (hipEventCreate(&p->pool[i]) != hipSuccess) p->pool[i] = nullptr;
    p->npool = ncap;
  }
  return p->pool[p->used++];
}

ProfScope::ProfScope(int kind, int tw, double bytes, hipStream_t st) : s(st) {
  Prof* p = g_prof;
  if (!p || p->failed) return;
  if (p->nrec >= p->cap) {
    const int ncap = p->cap ? 2 * p->cap : 256;
    ProfRec* nr = (ProfRec*)realloc(p->recs, sizeof(ProfRec) * ncap);
    if (!nr) {
      p->failed = true;
      return;
    }
    p->recs = nr;
    p->cap = ncap;
  }
  hipEvent_t a = prof_event(p), b = prof_event(p);
  if (!a || !b) {
    p->failed = true;
    return;
  }
  r = &p->recs[p->nrec++];
  r->kind = kind;
  r->tw = tw;
  r->level = p->level;
  r->idx = p->idx;
  r->bytes = bytes;
  r->a = a;
  r->b = b;
  r->executed = 1;
  (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
  if (r) (void)hipEventRecord(r->b, s);
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
static void rounds_tw(const LevelView& lv, int32_t* match, uint8_t* fr, int32_t* const* lists,
                      int32_t* const* cnts, int32_t* pa, int32_t* pb, Ctrl* ctrl, int R,
                      uint64_t hs, hipStream_t s) {
  // segments: as many blocks as the rows' teams fill, the same for both kernels
  const int nseg = grid_for((int64_t)lv.n * TW, kBlock, kMatchSegMax);
  const double n = lv.n, m2 = lv.nnz;
  for (int r = 0; r < R; r++) {
    int32_t* cur = (r & 1) ? pb : pa;
    const int32_t* prev = (r & 1) ? pa : pb;
    if (g_prof) g_prof->idx = r;
    if (r > 0) {
      ProfScope ps(PK_MATCH_FREE, 0, 0.0, s);
      k_match_free<<<nseg, kBlock, 0, s>>>(lv.n, match, prev, fr, lists[(r - 1) & 1],
                                           cnts[(r - 1) & 1], lists[r & 1], cnts[r & 1], ctrl,
                                           r);
    }
    ProfScope ps(PK_MATCH_ROUND, TW, r == 0 ? 4 * (n + 1) + 12 * m2 + 12 * n : 0.0, s);
    k_match_round<TW><<<nseg, kBlock, 0, s>>>(lv, match, fr, lists[r & 1], cnts[r & 1], prev,
                                              cur, ctrl, r, hs);
  }
}

bool launch_match_rounds(const LevelView& lv, int32_t* match, uint8_t* fr, int32_t* list_a,
                         int32_t* list_b, int32_t* seg_cnt, int32_t* prop_a, int32_t* prop_b,
                         Ctrl* ctrl, int R, uint64_t hs, int tw, hipStream_t s) {
  if (R <= 0) return true;
  int32_t* const lists[2] = {list_a, list_b};
  int32_t* const cnts[2] = {seg_cnt, seg_cnt + kMatchSegMax};
  switch (tw) {
    case 4: rounds_tw<4>(lv, match, fr, lists, cnts, prop_a, prop_b, ctrl, R, hs, s); break;
    case 8: rounds_tw<8>(lv, match, fr, lists, cnts, prop_a, prop_b, ctrl, R, hs, s); break;
    case 16: rounds_tw<16>(lv, match, fr, lists, cnts, prop_a, prop_b, ctrl, R, hs, s); break;
    case 32: rounds_tw<32>(lv, match, fr, lists, cnts, prop_a, prop_b, ctrl, R, hs, s); break;
    default: rounds_tw<64>(lv, match, fr, lists, cnts, prop_a, prop_b, ctrl, R, hs, s); break;
  }
  KCHECK();
  {
    ProfScope ps(PK_MATCH_SETTLE, 0, 0.0, s);
    // the free flags are spent: the settle clears them as the two-hop
    // pass's hub flags
    k_match_settle<<<grid_for(lv.n, kBlock * 4), kBlock, 0, s>>>(
        lv.n, match, ((R - 1) & 1) ? prop_b : prop_a, fr);
  }
  KCHECK();
  return true;
}

template <int TW>
static bool twohop_tw(const LevelView& lv, int32_t* match, int32_t* hub, const Ctrl* ctrl,
                      uint64_t hs, uint8_t* hflag, hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * TW, kBlock * 2);
  {
    ProfScope ps(PK_HUB, TW, 0.0, s);
    k_hub<TW><<<grid, kBlock, 0, s>>>(lv, match, hub, hs, hflag);
  }
  KCHECK();
  {
    // every row is read only without hub flags; with them, the rows read
    // depend on the matching (no byte count)
    ProfScope ps(PK_TWOHOP, TW, hflag ? 0.0 : 4.0 * (lv.n + 1) + 4.0 * lv.nnz + 4.0 * lv.n, s);
    k_twohop<TW><<<grid, kBlock, 0, s>>>(lv, hub, match, ctrl, hflag);
  }
  KCHECK();
  return true;
}

bool launch_twohop(const LevelView& lv, int32_t* match, Ctrl* ctrl, const Scratch& sc,
                   uint64_t hs, int tw, uint8_t* hflag, hipStream_t s) {
  bool ok;
  switch (tw) {
    case 4: ok = twohop_tw<4>(lv, match, sc.prop, ctrl, hs, hflag, s); break;
    case 8: ok = twohop_tw<8>(lv, match, sc.prop, ctrl, hs, hflag, s); break;
    case 16: ok = twohop_tw<16>(lv, match, sc.prop, ctrl, hs, hflag, s); break;
    case 32: ok = twohop_tw<32>(lv, match, sc.prop, ctrl, hs, hflag, s); break;
    default: ok = twohop_tw<64>(lv, match, sc.prop, ctrl, hs, hflag, s); break;
  }
  if (!ok) return false;
  const int ntiles = (lv.n + kTileV - 1) / kTileV;
  const int g = grid_for(ntiles, 1, 2048);
  ProfScope ps(PK_ISO, 0, 0.0, s);
  k_iso_count<<<g, kBlock, 0, s>>>(lv, match, ctrl, sc.tile_lead, ntiles);
  KCHECK();
  k_iso_scan<<<1, kBlock, 0, s>>>(ctrl, sc.tile_lead, ntiles);
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
  const double n = lv.n;
  {
    ProfScope ps(PK_CONTRACT_COUNT, 0, 4 * n + 4 * (n + 1) + 8 * n, s);
    k_contract_count<<<g, kBlock, 0, s>>>(lv, match, ctrl, sc.tile_lead, sc.tile_ub, ntiles,
                                          sc.partials);
  }
  KCHECK();
  k_contract_scan<<<1, kBlock, 0, s>>>(ctrl, sc.tile_lead, sc.tile_ub, ntiles, sc.partials, g);
  KCHECK();
  {
    ProfScope ps(PK_CONTRACT_MAP, 0, 4 * n + 4 * (n + 1) + 16 * n + 4 * n, s);
    const int ntc = (lv.n + kTileC - 1) / kTileC;
    k_contract_map<<<g, kBlock, 0, s>>>(lv, match, vc, vg, sc.tile_lead, sc.tile_ub, cmap, cvc,
                                        cvg, sc.cmem0, sc.cmem1, sc.toff, ntiles, sc.tile_cnt,
                                        ntc > 0 ? ntc : 1);
  }
  KCHECK();
  return true;
}

// nc_max: an upper bound of the coarse vertex count (sizes the grids).  The
// coarse rows are written straight into cadj / cw at their upper-bound
// offsets; cxadj / cxend get their begins and ends.
bool launch_contract_b(const LevelView& lv, const int32_t* cmap, Ctrl* ctrl, const Scratch& sc,
                       int32_t nc_max, int32_t* cxadj, int32_t* cxend, int32_t* cadj,
                       int64_t* cw, hipStream_t s) {
  const int ntc = (nc_max + kTileC - 1) / kTileC;
  const int ntc1 = ntc > 0 ? ntc : 1;
  {
    // algorithmic bytes are set after the level (they depend on the long rows)
    // rows of <= 32 candidates; the others are listed per segment in
    // sc.tmpk (free here; at least n slots), with their counts in
    // sc.partials, then sorted by the row kernel
    static_assert(kPartials >= kContractSegMax / 2 + 2 * kContractSegMax,
                  "partials hold the segment counts and totals");
    const int nseg = grid_for((int64_t)nc_max * 32, kBlock, kContractSegMax);
    int32_t* dcnt = (int32_t*)sc.partials;
    int64_t* sio = sc.partials + kContractSegMax / 2;
    {
      ProfScope ps(PK_CONTRACT_SHORT, 0, 0.0, s);
      k_contract_short<<<nseg, kBlock, 0, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj,
                                               cw, sc.cnt, sc.tmpk, dcnt, sio);
    }
    // the profiler's byte count of the two row kernels needs the totals
    if (g_prof) k_contract_sums<<<1, kBlock, 0, s>>>(ctrl, dcnt, sio, nseg);
    ProfScope ps(PK_CONTRACT_ROWS, 0, 0.0, s);
    k_contract_rows<<<nseg, kBlock, 0, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj, cw,
                                            sc.cnt, sc.tile_cnt, sc.longlist, ctrl, ntc1, sc.prop,
                                            sc.tmpk, dcnt);
  }
  KCHECK();
  {
    ProfScope ps(PK_CONTRACT_LONG, 0, 0.0, s);
    // rows of kWaveCap..kLongWave candidates, one wave each: up to one wave
    // per row, at most the twenty waves per compute unit that the LDS holds
    const int gw = nc_max < 5120 ? (nc_max > 0 ? nc_max : 1) : 5120;
    // (no tile counts: only the coarsest level's compaction needs them, and
    // it recounts them from the row lengths)
    k_contract_long<<<gw, 64, 0, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj, cw,
                                      sc.cnt, nullptr, sc.longlist);
  }
  KCHECK();
  // the dense window plus a staged copy of one row (96 KB)
  const size_t dyn = (size_t)(kWin + kSortCap) * (sizeof(int64_t) + sizeof(int32_t));
  static const bool huge_attr =
      hipFuncSetAttribute((const void*)k_contract_huge, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)dyn) == hipSuccess;
  if (!huge_attr) return false;
  {
    ProfScope ps(PK_CONTRACT_HUGE, 0, 0.0, s);
    // the rest of the long rows (sc.prop is free during contraction: it holds
    // their list), one block each
    // up to one block per row; one block per compute unit fits the LDS
    const int glong = nc_max < 512 ? (nc_max > 0 ? nc_max : 1) : 512;
    k_contract_huge<<<glong, kBlock, dyn, s>>>(lv, cmap, sc.cmem0, sc.cmem1, sc.toff, ctrl, cadj,
                                               cw, sc.cnt, nullptr, sc.prop, ntc1);
  }
  KCHECK();
  k_contract_ends<<<grid_for(nc_max, kBlock), kBlock, 0, s>>>(ctrl, sc.toff, sc.cnt, cxadj,
                                                               cxend);
  KCHECK();
  return true;
}

// The coarse level just built by launch_contract_b, made compact: the
// per-tile entry counts are scanned, the rows are copied in order to
// tmpk / tmpv and back, and cxadj gets the n + 1 exact offsets.
bool launch_compact_level(Ctrl* ctrl, const Scratch& sc, int32_t nc, int32_t nnz,
                          int32_t* cxadj, int32_t* cadj, int64_t* cw, hipStream_t s) {
  const int ntc = (nc + kTileC - 1) / kTileC;
  const int ntc1 = ntc > 0 ? ntc : 1;
  k_tile_count<<<grid_for(ntc1, kBlock / 64), kBlock, 0, s>>>(ctrl, sc.cnt, sc.tile_cnt, ntc1);
  KCHECK();
  k_tile_scan<<<1, kBlock, 0, s>>>(ctrl, sc.tile_cnt, ntc1);
  KCHECK();
  {
    ProfScope ps(PK_CONTRACT_COMPACT, 0, 24.0 * nnz + 16.0 * nc, s);
    k_contract_compact<<<grid_for(ntc1, 1, 4096), kBlock, 0, s>>>(
        ctrl, sc.toff, sc.cnt, sc.tile_cnt, cadj, cw, cxadj, sc.tmpk, sc.tmpv, ntc1);
  }
  KCHECK();
  if (nnz > 0 &&
      (hipMemcpyAsync(cadj, sc.tmpk, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice,
                      s) != hipSuccess ||
       hipMemcpyAsync(cw, sc.tmpv, sizeof(int64_t) * (size_t)nnz, hipMemcpyDeviceToDevice,
                      s) != hipSuccess))
    return false;
  return true;
}

// the gain launch; *grid_out = its block count (the number of partials)
template <int TW>
static bool gain_tw(const LevelView& lv, const int8_t* part, RefCtl* rc, Cand* list,
                    int64_t* partials, const RefArrays& ra, int* grid_out, hipStream_t s) {
  // one row per team: the row loads of all vertices are in flight at once
  const int grid = grid_for((int64_t)lv.n * TW, kBlock);
  ProfScope ps(PK_REFINE_GAIN, TW, 4.0 * (lv.n + 1) + 12.0 * lv.nnz + 17.0 * lv.n, s);
  k_refine_gain<TW><<<grid, kBlock, 0, s>>>(lv, part, rc, list, partials, ra.ext, ra.inn, ra.b1);
  KCHECK();
  *grid_out = grid;
  return true;
}

template <int TW>
static bool delta_tw(const LevelView& lv, const int8_t* part, const RefCtl* rc, const Cand* list,
                     const RefArrays& ra, int p, hipStream_t s) {
  // one team per listed candidate (at most n of them)
  const int grid = grid_for((int64_t)lv.n * TW, kBlock, 2048);
  ProfScope ps(PK_REFINE_DELTA, TW, 0.0, s);
  k_refine_delta<TW><<<grid, kBlock, 0, s>>>(lv, part, ra.mark, ra.ext, ra.inn, rc, list, p);
  KCHECK();
  return true;
}

// decision, moves and pass bookkeeping after a candidate launch of `grid`
// blocks: one block on levels of at most kSettleMax vertices, else decide ->
// apply -> finish
static bool pass_tail(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                      int64_t* partials, int grid, int32_t* pass_out, int32_t* mark,
                      hipStream_t s) {
  if (lv.n <= kSettleMax) {
    ProfScope ps(PK_REFINE_SETTLE, 0, 0.0, s);
    k_refine_settle<<<1, kBlock, 0, s>>>(lv.n, part, rc, list, partials, grid, pass_out, mark);
    KCHECK();
    return true;
  }
  k_refine_decide<<<1, kBlock, 0, s>>>(lv.n, rc, list, partials, grid);
  KCHECK();
  {
    ProfScope ps(PK_REFINE_APPLY, 0, 0.0, s);
    k_refine_apply<<<grid_for(lv.n, kBlock * 8, 1024), kBlock, 0, s>>>(part, rc, list, pass_out,
                                                                       mark);
  }
  KCHECK();
  k_refine_finish<<<1, 64, 0, s>>>(rc, pass_out);
  KCHECK();
  return true;
}

template <int TW>
static bool vol_pass_tw(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                        int64_t* partials, int32_t* pass_out, const int64_t* out, int32_t* cnt,
                        hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * TW, kBlock);
  k_vol_count<TW><<<grid, kBlock, 0, s>>>(lv, part, cnt);
  KCHECK();
  k_vol_gain<TW><<<grid, kBlock, 0, s>>>(lv, part, out, cnt, rc, list, partials);
  KCHECK();
  return pass_tail(lv, part, rc, list, partials, grid, pass_out, nullptr, s);
}

bool launch_vol_out(const LevelView& lv, int64_t* out, int tw, hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * tw, kBlock);
  switch (tw) {
    case 4: k_vol_out<4><<<grid, kBlock, 0, s>>>(lv, out); break;
    case 8: k_vol_out<8><<<grid, kBlock, 0, s>>>(lv, out); break;
    case 16: k_vol_out<16><<<grid, kBlock, 0, s>>>(lv, out); break;
    case 32: k_vol_out<32><<<grid, kBlock, 0, s>>>(lv, out); break;
    default: k_vol_out<64><<<grid, kBlock, 0, s>>>(lv, out); break;
  }
  KCHECK();
  return true;
}

bool launch_vol_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                     int64_t* partials, int32_t* pass_out, const int64_t* out, int32_t* cnt,
                     int tw, hipStream_t s) {
  switch (tw) {
    case 4: return vol_pass_tw<4>(lv, part, rc, list, partials, pass_out, out, cnt, s);
    case 8: return vol_pass_tw<8>(lv, part, rc, list, partials, pass_out, out, cnt, s);
    case 16: return vol_pass_tw<16>(lv, part, rc, list, partials, pass_out, out, cnt, s);
    case 32: return vol_pass_tw<32>(lv, part, rc, list, partials, pass_out, out, cnt, s);
    default: return vol_pass_tw<64>(lv, part, rc, list, partials, pass_out, out, cnt, s);
  }
}

bool launch_vol_total(const LevelView& lv, const int8_t* part, const int64_t* out, Ctrl* ctrl,
                      int tw, hipStream_t s) {
  k_vol_reset<<<1, 64, 0, s>>>(ctrl);
  KCHECK();
  const int grid = grid_for((int64_t)lv.n * tw, kBlock);
  switch (tw) {
    case 4: k_vol_total<4><<<grid, kBlock, 0, s>>>(lv, part, out, ctrl); break;
    case 8: k_vol_total<8><<<grid, kBlock, 0, s>>>(lv, part, out, ctrl); break;
    case 16: k_vol_total<16><<<grid, kBlock, 0, s>>>(lv, part, out, ctrl); break;
    case 32: k_vol_total<32><<<grid, kBlock, 0, s>>>(lv, part, out, ctrl); break;
    default: k_vol_total<64><<<grid, kBlock, 0, s>>>(lv, part, out, ctrl); break;
  }
  KCHECK();
  return true;
}

bool launch_refine_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                        int64_t* partials, int tw, int32_t* pass_out, int p, int npass,
                        const RefArrays& ra, hipStream_t s) {
  bool ok;
  int grid = 0;
  if (p == 0) {
    // the first pass of a level reads the rows and keeps every vertex's
    // external and internal weight
    switch (tw) {
      case 4: ok = gain_tw<4>(lv, part, rc, list, partials, ra, &grid, s); break;
      case 8: ok = gain_tw<8>(lv, part, rc, list, partials, ra, &grid, s); break;
      case 16: ok = gain_tw<16>(lv, part, rc, list, partials, ra, &grid, s); break;
      case 32: ok = gain_tw<32>(lv, part, rc, list, partials, ra, &grid, s); break;
      default: ok = gain_tw<64>(lv, part, rc, list, partials, ra, &grid, s); break;
    }
    if (!ok) return false;
  } else {
    grid = grid_for(lv.n, kBlock);
    ProfScope ps(PK_REFINE_SCAN, 0, 25.0 * lv.n, s);
    k_refine_scan<<<grid, kBlock, 0, s>>>(lv.n, part, lv.b, ra.b1, ra.ext, ra.inn, rc, list,
                                          partials);
    KCHECK();
  }
  if (!pass_tail(lv, part, rc, list, partials, grid, pass_out, ra.mark, s)) return false;
  if (p + 1 >= npass) return true;  // no pass reads the weights after the last one
  switch (tw) {
    case 4: return delta_tw<4>(lv, part, rc, list, ra, p, s);
    case 8: return delta_tw<8>(lv, part, rc, list, ra, p, s);
    case 16: return delta_tw<16>(lv, part, rc, list, ra, p, s);
    case 32: return delta_tw<32>(lv, part, rc, list, ra, p, s);
    default: return delta_tw<64>(lv, part, rc, list, ra, p, s);
  }
}

bool launch_project(int32_t n, const int32_t* cmap, const int8_t* cpart, int8_t* part, RefCtl* rc,
                    int npass, int32_t* mark, hipStream_t s) {
  ProfScope ps(PK_PROJECT, 0, 10.0 * n, s);
  k_project<<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, cmap, cpart, part, rc, npass, mark);
  KCHECK();
  return true;
}

bool launch_time_bounds(Ctrl* ctrl, int64_t maxw0, int64_t maxw1, int npass, hipStream_t s) {
  k_time_bounds<<<1, 64, 0, s>>>(ctrl, maxw0, maxw1, npass);
  KCHECK();
  return true;
}

bool launch_start_level(RefCtl* rc, int npass, hipStream_t s) {
  k_start_level<<<1, 64, 0, s>>>(rc, npass);
  KCHECK();
  return true;
}

bool launch_final_stats(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const int8_t* part, Ctrl* ctrl, int tw, int64_t* partials,
                        hipStream_t s) {
  const int grid = grid_for((int64_t)lv.n * tw, kBlock * 2);
  {
    ProfScope ps(PK_FINAL_STATS, tw, 4.0 * (lv.n + 1) + 12.0 * lv.nnz + 25.0 * lv.n, s);
    switch (tw) {
      case 4: k_final_stats<4><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl, partials); break;
      case 8: k_final_stats<8><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl, partials); break;
      case 16: k_final_stats<16><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl, partials); break;
      case 32: k_final_stats<32><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl, partials); break;
      default: k_final_stats<64><<<grid, kBlock, 0, s>>>(lv, vc, vg, part, ctrl, partials); break;
    }
  }
  KCHECK();
  k_final_reduce<<<1, kBlock, 0, s>>>(ctrl, partials, grid);
  KCHECK();
  return true;
}

bool launch_init(const LevelView& lv, int K, int gs, int npass, Ctrl* ctrl, const InitScratch& is,
                 int8_t* out_part, hipStream_t s) {
  {
    ProfScope ps(PK_INIT_TOT, 0, 0.0, s);
    k_init_tot<<<grid_for((int64_t)lv.n * kInitTotTeam, kBlock), kBlock, 0, s>>>(lv, is.tot);
  }
  KCHECK();
  // each of the K trials reads the coarsest graph once (xadj, adj + w, b,
  // incident sums) and writes its assignment
  const double trial_bytes =
      (double)K * (4.0 * (lv.n + 1) + 12.0 * lv.nnz + 16.0 * lv.n + 1.0 * lv.n);
  ProfScope ps(PK_INIT_TRIALS, 0, lv.n <= kTrialLdsMax ? trial_bytes : 0.0, s);
  if (lv.n <= kTrialLdsMax) {
    const size_t dyn = trial_lds_bytes(lv.n, kTrialBlock);
    const int max_dyn = (int)trial_lds_bytes(kTrialLdsMax, kTrialBlock);
    // more than 64 KB of dynamic LDS must be allowed once (thread-safe statics)
    static const bool lds_attr =
        hipFuncSetAttribute((const void*)k_init_trials_lds<kTrialBlock, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn) == hipSuccess &&
        hipFuncSetAttribute((const void*)k_init_trials_lds<kTrialBlock, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn) == hipSuccess;
    if (!lds_attr) return false;
    // rows longer than two entries per lane on average: the form that reads
    // the pick's row with the whole block (both forms give the same result)
    if (lv.nnz > (int64_t)kTrialLongDeg * lv.n)
      k_init_trials_lds<kTrialBlock, true><<<K, kTrialBlock, dyn, s>>>(
          lv, is.tot, K, gs, npass, ctrl, is.ctl, is.part, is.res, out_part);
    else
      k_init_trials_lds<kTrialBlock, false><<<K, kTrialBlock, dyn, s>>>(
          lv, is.tot, K, gs, npass, ctrl, is.ctl, is.part, is.res, out_part);
    KCHECK();
    return true;
  }
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
