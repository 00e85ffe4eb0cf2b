// gp_launch.h - host-side launchers of the gfx950 kernels (internal).
#pragma once

#include "gp_internal.h"

namespace gpk {

// scratch of the level kernels, sized for the level-0 graph
struct Scratch {
  int32_t* prop;       // n
  int32_t* tile_lead;  // ceil(n / kTileV)
  int64_t* tile_ub;    // ceil(n / kTileV)
  int32_t* cmem0;      // n
  int32_t* cmem1;      // n
  int64_t* toff;       // n
  int32_t* cnt;        // n
  int64_t* tile_cnt;   // ceil(n / kTileC)
  int32_t* tmpk;       // nnz
  int64_t* tmpv;       // nnz
  int32_t* longlist;   // n
  Cand* list;          // n
};

// scratch of the initial bisection, sized for the coarsest graph and K trials
struct InitScratch {
  int64_t* tot;        // n
  RefCtl* ctl;         // K
  int8_t* part;        // K * n
  int64_t* conn;       // K * n
  int32_t* adjc;       // K * n
  Cand* list;          // K * n
  int64_t* res;        // 2K
};

int team_width_for(int32_t n, int64_t nnz);

bool launch_level_reset(Ctrl* ctrl, int promote, hipStream_t s);
bool launch_match_round(const LevelView& lv, int32_t* match, int32_t* prop, Ctrl* ctrl, int round,
                        uint64_t hs, int tw, hipStream_t s);
bool launch_twohop(const LevelView& lv, int32_t* match, Ctrl* ctrl, const Scratch& sc,
                   uint64_t hs, int tw, hipStream_t s);
bool launch_contract_a(const LevelView& lv, const int32_t* match, const int64_t* vc,
                       const int64_t* vg, Ctrl* ctrl, const Scratch& sc, int32_t* cmap,
                       int64_t* cvc, int64_t* cvg, hipStream_t s);
bool launch_contract_b(const LevelView& lv, const int32_t* cmap, Ctrl* ctrl, const Scratch& sc,
                       int32_t nc_max, int32_t* cxadj, int32_t* cadj, int64_t* cw,
                       hipStream_t s);
bool launch_refine_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list, int tw,
                        hipStream_t s);
bool launch_project(int32_t n, const int32_t* cmap, const int8_t* cpart, int8_t* part, RefCtl* rc,
                    int npass, hipStream_t s);
bool launch_start_level(RefCtl* rc, int npass, hipStream_t s);
bool launch_final_stats(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const int8_t* part, Ctrl* ctrl, int tw, hipStream_t s);
bool launch_init(const LevelView& lv, int K, int gs, int npass, Ctrl* ctrl, const InitScratch& is,
                 int8_t* out_part, hipStream_t s);
bool launch_validate(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                     const int64_t* vc, const int64_t* vg, Ctrl* ctrl, int stage, hipStream_t s);
bool launch_sort_rows(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                      int32_t* oadj, int64_t* ow, Ctrl* ctrl, hipStream_t s);
bool launch_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg, hipStream_t s);

}  // namespace gpk
