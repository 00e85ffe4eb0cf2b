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
  int64_t* partials;   // 5 x 4096: per-block partial results of a reduction
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

// ---- per-launch profiling (HIP events), enabled by the driver for one call
enum ProfKind {
  PK_MATCH_ROUND, PK_MATCH_FREE, PK_MATCH_SETTLE, PK_HUB, PK_TWOHOP, PK_ISO, PK_CONTRACT_COUNT,
  PK_CONTRACT_MAP, PK_CONTRACT_SHORT, PK_CONTRACT_ROWS, PK_CONTRACT_LONG, PK_CONTRACT_HUGE, PK_CONTRACT_COMPACT,
  PK_INIT_TOT,
  PK_INIT_TRIALS, PK_REFINE_GAIN, PK_REFINE_SCAN, PK_REFINE_DELTA, PK_REFINE_SETTLE,
  PK_REFINE_APPLY, PK_PROJECT, PK_FINAL_STATS, PK_N
};
extern const char* const kProfNames[PK_N];

struct ProfRec {
  int kind, tw, level, idx;   // idx: matching round or refinement pass
  double bytes;               // algorithmic bytes if the launch does its work (0: undefined)
  hipEvent_t a, b;
  int executed;
};

struct Prof {
  ProfRec* recs = nullptr;
  int nrec = 0, cap = 0;
  hipEvent_t* pool = nullptr;
  int npool = 0, used = 0;
  int level = 0, idx = 0;
  bool failed = false;
};
extern thread_local Prof* g_prof;  // set by the driver around a profiled call, per host thread

// records events around one launch when profiling is on
struct ProfScope {
  ProfRec* r = nullptr;
  hipStream_t s;
  ProfScope(int kind, int tw, double bytes, hipStream_t st);
  ~ProfScope();
};

bool launch_level_reset(Ctrl* ctrl, int promote, hipStream_t s);
// R matching rounds (from the second on, a settle of the previous round that
// marks the free vertices in fr and lists them, then the proposals of the
// listed vertices), then the last settled; fr: uint8[n] scratch, left
// cleared by the last settle (the two-hop pass's hub flags); list_a /
// list_b: two int32[n] lists; seg_cnt: int32[2 kMatchSegMax] list lengths;
// prop_a / prop_b: two int32[n] proposal buffers
bool launch_match_rounds(const LevelView& lv, int32_t* match, uint8_t* fr, int32_t* list_a,
                         int32_t* list_b, int32_t* seg_cnt, int32_t* prop_a, int32_t* prop_b,
                         Ctrl* ctrl, int R, uint64_t hs, int tw, hipStream_t s);
// two-hop pass and isolated pairs; hflag: uint8[n] cleared flags (the
// matching's fr after R >= 1 rounds) that let the pairing read only the rows
// of hubs, or nullptr to read every row
bool launch_twohop(const LevelView& lv, int32_t* match, Ctrl* ctrl, const Scratch& sc,
                   uint64_t hs, int tw, uint8_t* hflag, hipStream_t s);
bool launch_contract_a(const LevelView& lv, const int32_t* match, const int64_t* vc,
                       const int64_t* vg, Ctrl* ctrl, const Scratch& sc, int32_t* cmap,
                       int64_t* cvc, int64_t* cvg, hipStream_t s);
bool launch_contract_b(const LevelView& lv, const int32_t* cmap, Ctrl* ctrl, const Scratch& sc,
                       int32_t nc_max, int32_t* cxadj, int32_t* cxend, int32_t* cadj,
                       int64_t* cw, hipStream_t s);
// makes the level built by the last launch_contract_b compact (nnz entries)
bool launch_compact_level(Ctrl* ctrl, const Scratch& sc, int32_t nc, int32_t nnz,
                          int32_t* cxadj, int32_t* cadj, int64_t* cw, hipStream_t s);
// per-vertex state of the passes of one level, sized for level 0
struct RefArrays {
  int64_t* ext;   // n: weight to the other side, kept up to date across passes
  int64_t* inn;   // n: weight to the own side
  int32_t* mark;  // n: p + 1 for the vertices moved by pass p, cleared by the projection
  const int64_t* b1;  // side 1's weight column when the sides use different ones, else null
};

// Pass p (of npass) of a level: the first pass computes every vertex's
// external and internal weight from the rows, later ones read them; the
// moves' effect on those weights is applied after each pass but the last.
// partials: 4 int64 per block of the gain kernel (grids are capped at 4096)
bool launch_refine_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                        int64_t* partials, int tw, int32_t* pass_out, int p, int npass,
                        const RefArrays& ra, hipStream_t s);
bool launch_project(int32_t n, const int32_t* cmap, const int8_t* cpart, int8_t* part, RefCtl* rc,
                    int npass, int32_t* mark, hipStream_t s);
bool launch_start_level(RefCtl* rc, int npass, hipStream_t s);
// communication volume: out = each vertex's largest edge to a successor; one
// pass with the volume gain (cnt: int32[n] scratch); the volume into
// ctrl->res_vol
bool launch_vol_out(const LevelView& lv, int64_t* out, int tw, hipStream_t s);
bool launch_vol_pass(const LevelView& lv, int8_t* part, RefCtl* rc, Cand* list,
                     int64_t* partials, int32_t* pass_out, const int64_t* out, int32_t* cnt,
                     int tw, hipStream_t s);
bool launch_vol_total(const LevelView& lv, const int8_t* part, const int64_t* out, Ctrl* ctrl,
                      int tw, hipStream_t s);
// time balance: loads from the last statistics launch, bounds (maxw0, maxw1)
bool launch_time_bounds(Ctrl* ctrl, int64_t maxw0, int64_t maxw1, int npass, hipStream_t s);
// partials: 5 int64 per block (grids are capped at 4096)
bool launch_final_stats(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const int8_t* part, Ctrl* ctrl, int tw, int64_t* partials,
                        hipStream_t s);
bool launch_init(const LevelView& lv, int K, int gs, int npass, Ctrl* ctrl, const InitScratch& is,
                 int8_t* out_part, hipStream_t s);
bool launch_validate(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                     const int64_t* vc, const int64_t* vg, Ctrl* ctrl, int stage, hipStream_t s);
bool launch_sort_rows(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                      int32_t* oadj, int64_t* ow, Ctrl* ctrl, hipStream_t s);
bool launch_split_vwgt(int32_t n, const int64_t* vwgt, int64_t* vc, int64_t* vg, hipStream_t s);

// ---- k-way partition by recursive bisection (gp_kway.hip)
bool launch_kw_zero(int32_t* label, int32_t n, int64_t* acc, int nacc, hipStream_t s);
// subgraph of the vertices labelled lo: per-tile member and entry counts and
// their scans; tot[0..1] = vertices and entries of the subgraph
bool launch_kw_extract_a(int32_t n, const int32_t* xadj, const int32_t* adj, const int32_t* label,
                         int32_t lo, int32_t* keep, int64_t* tile_m, int64_t* tile_e,
                         int64_t* tot, hipStream_t s);
// its ids, CSR (rows in order, neighbour ids renumbered) and vertex weights
bool launch_kw_extract_b(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                         const int64_t* vc, const int64_t* vg, const int32_t* label, int32_t lo,
                         const int32_t* keep, const int64_t* tile_m, const int64_t* tile_e,
                         const int64_t* tot, int32_t* newid, int32_t* sxadj, int32_t* sadj,
                         int64_t* sw, int64_t* svwgt, hipStream_t s);
bool launch_kw_apply(int32_t n, int32_t* label, int32_t lo, int32_t mid, const int32_t* newid,
                     const int8_t* spart, hipStream_t s);
bool launch_kw_stats(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                     const int32_t* label, const int64_t* b, int64_t* ext_sum, int64_t* load,
                     hipStream_t s);

}  // namespace gpk
