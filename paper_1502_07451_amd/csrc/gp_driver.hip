// gp_driver.hip - C ABI and host driver of the single-graph path.
//
// The driver owns a device copy of the input graph (level 0) and the
// buffers of every coarse level; they are kept across calls, so repeated
// partitions of one handle allocate nothing after the first call.  Work is
// queued on the handle's stream; the host waits only once per coarse level
// (to learn the coarse graph's size) and once at the end.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <utility>
#include <vector>

constexpr int kKwayMax = 1024;

#include "../../include/gp.h"
#include "gp_launch.h"
#include "gp_mpnn.h"

using namespace gpk;

namespace {

// Device bytes a handle holds in its buffers and the most it may hold (-1:
// no limit).  A call on a handle charges every buffer it grows or frees to
// the handle's budget through tl_ws, set for the call's duration by WsScope.
struct WsBudget {
  int64_t cap = -1;
  int64_t used = 0;
};
thread_local WsBudget* tl_ws = nullptr;
struct WsScope {
  WsBudget* prev;
  explicit WsScope(WsBudget* b) : prev(tl_ws) { tl_ws = b; }
  ~WsScope() { tl_ws = prev; }
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t cap = 0;
  bool ensure(size_t n) {
    if (n == 0) n = 1;
    if (p && n <= cap) return true;
    // refuse before freeing, so a refused call leaves the buffer as it was
    const int64_t grow = (int64_t)((n - cap) * sizeof(T));
    if (tl_ws && tl_ws->cap >= 0 && tl_ws->used + grow > tl_ws->cap) return false;
    release();
    if (hipMalloc((void**)&p, n * sizeof(T)) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return false;
    }
    cap = n;
    if (tl_ws) tl_ws->used += (int64_t)(n * sizeof(T));
    return true;
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (tl_ws) tl_ws->used -= (int64_t)(cap * sizeof(T));
    }
    p = nullptr;
    cap = 0;
  }
};

struct Level {
  int32_t n = 0;
  int64_t nnz = 0;   // entries
  bool gapped = false;  // rows at their upper-bound offsets: xe holds the row ends
  int64_t span = 0;     // with gaps: the extent of adj / w in use
  DBuf<int32_t> xadj, xe, adj, match, cmap;
  DBuf<int64_t> w, vc, vg;
  DBuf<int8_t> part;
  bool ensure(int64_t ncap, int64_t nnzcap) {
    return xadj.ensure(ncap + 1) && xe.ensure(ncap) && adj.ensure(nnzcap) && w.ensure(nnzcap) &&
           vc.ensure(ncap) && vg.ensure(ncap) && match.ensure(ncap) && cmap.ensure(ncap) &&
           part.ensure(ncap);
  }
  void release() {
    xadj.release(); xe.release(); adj.release(); match.release(); cmap.release();
    w.release(); vc.release(); vg.release(); part.release();
  }
  LevelView view(int bal) const {
    LevelView v;
    v.n = n;
    v.nnz = (int32_t)nnz;
    v.xadj = xadj.p;
    v.xend = gapped ? xe.p : xadj.p + 1;
    v.adj = adj.p;
    v.w = w.p;
    v.b = bal ? vg.p : vc.p;
    return v;
  }
};

uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

}  // namespace

struct gp_graph {
  hipStream_t stream = nullptr;
  int flags = 0;
  WsBudget ws;              // this handle's buffers
  WsBudget* wsp = &ws;      // the budget they are charged to (a k-way parent's for its subgraphs)
  int32_t n = 0;
  int64_t nnz = 0;
  int64_t sum[2] = {0, 0};
  int64_t maxv[2] = {0, 0};
  std::vector<Level*> lv;
  int32_t last_levels = -1;  // coarse levels built by the last partition (-1: none yet)
  // level scratch
  DBuf<int32_t> prop, tile_lead, cmem0, cmem1, cnt, tmpk, longlist;
  DBuf<int64_t> tile_ub, toff, tile_cnt, tmpv;
  DBuf<int64_t> partials;  // <= 5 per block of a multi-block reduction (grids of <= 4096)
  DBuf<int64_t> r_ext, r_inn;  // refinement: per-vertex external / internal weight
  DBuf<int32_t> r_mark;        // refinement: vertices moved by the current pass
  DBuf<Cand> list;
  // initial bisection scratch
  DBuf<int64_t> i_tot, i_conn, i_res;
  DBuf<RefCtl> i_ctl;
  DBuf<int8_t> i_part;
  DBuf<int32_t> i_adjc;
  DBuf<Cand> i_list;
  // learned proposal scratch
  DBuf<uint16_t> m_ha, m_hb;
  DBuf<float> m_inv, m_score;
  DBuf<int32_t> m_order;
  DBuf<int8_t> m_lp, m_save;  // refined learned proposal (coarsest), plain level-0 result
  // k-way partition: labels, subgraph extraction and the subgraph's bisection
  DBuf<int32_t> kw_label, kw_keep, kw_newid, kw_sxadj, kw_sadj;
  DBuf<int64_t> kw_tiles, kw_tot, kw_sw, kw_svwgt, kw_acc;
  DBuf<int8_t> kw_spart;
  Ctrl* ctrl = nullptr;
  Ctrl* hctrl = nullptr;  // pinned
  // profiling
  bool profiling = false;
  Prof prof;
  std::vector<gp_prof_row> prof_rows;

  Scratch scratch() const {
    Scratch s;
    s.prop = prop.p;
    s.tile_lead = tile_lead.p;
    s.tile_ub = tile_ub.p;
    s.cmem0 = cmem0.p;
    s.cmem1 = cmem1.p;
    s.toff = toff.p;
    s.cnt = cnt.p;
    s.tile_cnt = tile_cnt.p;
    s.tmpk = tmpk.p;
    s.tmpv = tmpv.p;
    s.longlist = longlist.p;
    s.list = list.p;
    s.partials = partials.p;
    return s;
  }
  bool ensure_scratch() {
    const int64_t n1 = n > 0 ? n : 1;
    return prop.ensure(n1) && tile_lead.ensure(n1 / kTileV + 2) &&
           tile_ub.ensure(n1 / kTileV + 2) && cmem0.ensure(n1) && cmem1.ensure(n1) &&
           toff.ensure(n1) && cnt.ensure(n1) && tile_cnt.ensure(n1 / kTileC + 2) &&
           tmpk.ensure(nnz > n1 ? nnz : n1) && tmpv.ensure(nnz) && longlist.ensure(n1) &&
           list.ensure(n1) &&
           partials.ensure(kPartials) && r_ext.ensure(n1) && r_inn.ensure(n1) &&
           r_mark.ensure(n1);
  }
  bool ensure_init(int32_t nl, int K) {
    const int64_t kn = (int64_t)K * (nl > 0 ? nl : 1);
    return i_tot.ensure(nl) && i_ctl.ensure(K) && i_part.ensure(kn) && i_conn.ensure(kn) &&
           i_adjc.ensure(kn) && i_list.ensure(kn) && i_res.ensure(2 * (size_t)K);
  }
  InitScratch init_scratch() const {
    InitScratch s;
    s.tot = i_tot.p;
    s.ctl = i_ctl.p;
    s.part = i_part.p;
    s.conn = i_conn.p;
    s.adjc = i_adjc.p;
    s.list = i_list.p;
    s.res = i_res.p;
    return s;
  }
  ~gp_graph() {
    for (Level* l : lv) {
      l->release();
      delete l;
    }
    prop.release(); tile_lead.release(); cmem0.release(); cmem1.release(); cnt.release();
    tmpk.release(); longlist.release(); tile_ub.release(); toff.release(); tile_cnt.release();
    tmpv.release(); list.release(); partials.release();
    r_ext.release(); r_inn.release(); r_mark.release();
    i_tot.release(); i_conn.release(); i_res.release(); i_ctl.release(); i_part.release();
    i_adjc.release(); i_list.release();
    m_ha.release(); m_hb.release(); m_inv.release(); m_score.release(); m_order.release();
    m_lp.release(); m_save.release();
    kw_label.release(); kw_keep.release(); kw_newid.release(); kw_sxadj.release();
    kw_sadj.release(); kw_tiles.release(); kw_tot.release(); kw_sw.release(); kw_svwgt.release();
    kw_acc.release(); kw_spart.release();
    if (ctrl) (void)hipFree(ctrl);
    if (hctrl) (void)hipHostFree(hctrl);
    for (int i = 0; i < prof.npool; i++)
      if (prof.pool[i]) (void)hipEventDestroy(prof.pool[i]);
    free(prof.pool);
    free(prof.recs);
  }
};

// ------------------------------------------------------------------ helpers
#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) {               \
      (void)hipGetLastError();             \
      return GP_EDEVICE;                   \
    }                                      \
  } while (0)
#define LCHK(x)                \
  do {                         \
    if (!(x)) return GP_EDEVICE; \
  } while (0)

static gp_status read_ctrl(gp_graph* g) {
  HIPCHK(hipMemcpyAsync(g->hctrl, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return GP_OK;
}

// marks which recorded launches of a level did their work
static void prof_mark(gp_graph* g, int level, bool coarsening) {
  if (!g->profiling) return;
  const Ctrl& h = *g->hctrl;
  for (int i = 0; i < g->prof.nrec; i++) {
    ProfRec& r = g->prof.recs[i];
    if (r.level != level) continue;
    if (coarsening && (r.kind == PK_MATCH_ROUND || r.kind == PK_MATCH_FREE))
      r.executed = (r.idx <= 1 || h.made[r.idx - 1] > 0) ? 1 : 0;
    if (coarsening) {
      // the split of the coarse rows between the row kernels is known only
      // now: fine entries read (adj, w, cmap of the neighbour: 16 B), coarse
      // entries written (12 B), plus per-row bookkeeping
      const double nf = g->lv[level]->n, mf = g->lv[level]->nnz;
      const double nc = h.nc, mc = h.nnz_c, li = (double)h.long_in, lo = (double)h.long_out;
      const double hi = (double)h.huge_in, ho = (double)h.huge_out;
      const double si = (double)h.short_in, so = (double)h.short_out;
      // the short-row kernel reads every row's members and offsets; the row
      // kernel those of the rows it was left, and their list entries
      const double nd = (double)h.deferred;
      if (r.kind == PK_CONTRACT_SHORT) r.bytes = 16 * si + 12 * so + 8 * nf + 20 * nc;
      if (r.kind == PK_CONTRACT_ROWS)
        r.bytes = 16 * (mf - si - li - hi) + 12 * (mc - so - lo - ho) + 40 * nd;
      if (r.kind == PK_CONTRACT_LONG) r.bytes = 16 * li + 12 * lo;
      if (r.kind == PK_CONTRACT_HUGE) r.bytes = 16 * hi + 12 * ho;
      if (r.kind == PK_CONTRACT_COMPACT) r.bytes = 24 * mc + 16 * nc + 4;
    }
    if (!coarsening && (r.kind == PK_REFINE_GAIN || r.kind == PK_REFINE_SCAN ||
                        r.kind == PK_REFINE_SETTLE || r.kind == PK_REFINE_APPLY))
      r.executed = r.idx < h.lvl_pass[level] ? 1 : 0;
  }
}

// folds the recorded launches of one call into the per-kernel rows
static void prof_collect(gp_graph* g) {
  Prof& p = g->prof;
  for (int i = 0; i < p.nrec; i++) {
    const ProfRec& r = p.recs[i];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0.f;
    }
    char name[40];
    if (r.tw > 0) snprintf(name, sizeof(name), "%s<%d>", kProfNames[r.kind], r.tw);
    else snprintf(name, sizeof(name), "%s", kProfNames[r.kind]);
    gp_prof_row* row = nullptr;
    for (auto& x : g->prof_rows)
      if (strcmp(x.name, name) == 0) row = &x;
    if (!row) {
      gp_prof_row z;
      memset(&z, 0, sizeof(z));
      snprintf(z.name, sizeof(z.name), "%s", name);
      g->prof_rows.push_back(z);
      row = &g->prof_rows.back();
    }
    row->launches++;
    row->ms += ms;
    if (r.executed) {
      row->executed++;
      row->bytes += r.bytes;
    }
  }
  p.nrec = 0;
  p.used = 0;
  p.failed = false;
}

static gp_status check_options(const gp_options* o) {
  if (!o) return GP_EINVAL;
  const int64_t lim = (int64_t)1 << 40;
  if (o->ratio[0] < 0 || o->ratio[1] < 0 || o->ratio[0] >= lim || o->ratio[1] >= lim ||
      o->ratio[0] + o->ratio[1] == 0)
    return GP_EINVAL;
  if (o->eps_ppm < 0 || o->eps_ppm > 1000000) return GP_EINVAL;
  if (o->balance_on != 0 && o->balance_on != 1) return GP_EINVAL;
  if (o->coarsen_to < 1 || o->match_rounds < 0 || o->match_rounds > kMaxRounds ||
      o->refine_passes < 0 || o->refine_passes > 64 || o->init_trials < 1 || o->init_trials > 64)
    return GP_EINVAL;
  if (o->flags & GP_LEARNED) {
    const MpModel* m = (const MpModel*)o->model;
    if (!m || m->magic != kMpMagic) return GP_EMODEL;
    if (o->flags & GP_TIME_BALANCE) return GP_EINVAL;
  }
  if ((o->flags & GP_VOLUME) && (o->flags & (GP_LEARNED | GP_TIME_BALANCE))) return GP_EINVAL;
  return GP_OK;
}

// Eq. (1)-(2) bounds: tgt_p = floor(W r_p / R), maxw_p = ceil(W r_p (1e6+eps) / (R 1e6))
static void host_balance(int64_t W, const int64_t* r, int32_t eps, int64_t* tgt, int64_t* maxw) {
  const __int128 R = (__int128)r[0] + r[1];
  for (int p = 0; p < 2; p++) {
    tgt[p] = (int64_t)(((__int128)W * r[p]) / R);
    const __int128 num = (__int128)W * r[p] * (1000000 + eps);
    const __int128 den = R * 1000000;
    maxw[p] = (int64_t)((num + den - 1) / den);
  }
}

// ------------------------------------------------------------------- C ABI
extern "C" {

void gp_options_default(gp_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->ratio[0] = 1;
  o->ratio[1] = 4;
  o->eps_ppm = 30000;
  o->balance_on = 0;
  o->seed = 0;
  o->coarsen_to = 2048;
  o->match_rounds = 8;
  o->refine_passes = 8;
  o->init_trials = 16;
  o->flags = 0;
  o->model = nullptr;
}

gp_status gp_ratio_from_times(int64_t t_cpu, int64_t t_gpu, int64_t ratio[2]) {
  if (!ratio || t_cpu < 0 || t_gpu < 0 || (t_cpu == 0 && t_gpu == 0)) return GP_EINVAL;
  int64_t a = t_gpu, b = t_cpu;
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  ratio[0] = t_gpu / a;
  ratio[1] = t_cpu / a;
  return GP_OK;
}

const char* gp_strerror(gp_status s) {
  switch (s) {
    case GP_OK: return "ok";
    case GP_EINVAL: return "invalid argument, option or row offsets";
    case GP_EASYM: return "edge u-v without v-u of equal weight";
    case GP_EDUP: return "neighbour listed twice in one row";
    case GP_ESELF: return "self loop";
    case GP_ERANGE: return "neighbour id out of range or negative weight";
    case GP_EOVERFLOW: return "sum of weights reaches 2^62";
    case GP_ENOMEM: return "out of memory";
    case GP_EDEVICE: return "HIP runtime error";
    case GP_EMODEL: return "learned proposal requested without a usable model";
  }
  return "unknown status";
}

gp_status gp_set_stream(gp_graph* g, void* stream) {
  if (!g) return GP_EINVAL;
  g->stream = (hipStream_t)stream;
  return GP_OK;
}

void gp_destroy(gp_graph* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  WsScope ws(g->wsp);
  delete g;
}

gp_status gp_set_workspace_limit(gp_graph* g, int64_t bytes) {
  if (!g || bytes < -1) return GP_EINVAL;
  g->ws.cap = bytes;
  return GP_OK;
}

int64_t gp_workspace_bytes(const gp_graph* g) { return g ? g->ws.used : -1; }

}  // extern "C"

// gp_create with its buffers charged to budget (the new handle's own when
// null); a k-way partition charges its subgraphs to the parent handle
static gp_status create_graph(gp_graph** out, int32_t n, const int32_t* xadj,
                              const int32_t* adjncy, const int64_t* adjwgt, const int64_t* vwgt,
                              int32_t flags, void* stream, WsBudget* budget) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  if (n < 0) return GP_EINVAL;
  if (n > 0 && (!xadj || !vwgt)) return GP_EINVAL;
  gp_graph* g = new (std::nothrow) gp_graph();
  if (!g) return GP_ENOMEM;
  if (budget) g->wsp = budget;
  WsScope ws(g->wsp);
  g->stream = (hipStream_t)stream;
  g->flags = flags;
  g->n = n;
  const bool host = (flags & GP_HOST_PTRS) != 0;
  const hipMemcpyKind kin = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  gp_status st = GP_OK;
  do {
    if (hipMalloc((void**)&g->ctrl, sizeof(Ctrl)) != hipSuccess) { st = GP_ENOMEM; break; }
    if (hipHostMalloc((void**)&g->hctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
      g->hctrl = nullptr;
      st = GP_ENOMEM;
      break;
    }
    memset(g->hctrl, 0, sizeof(Ctrl));
    Level* l0 = new (std::nothrow) Level();
    if (!l0) { st = GP_ENOMEM; break; }
    g->lv.push_back(l0);
    if (n == 0) break;
    int32_t nnz32 = 0;
    if (host) {
      nnz32 = xadj[n];
    } else {
      if (hipMemcpy(&nnz32, xadj + n, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
        st = GP_EDEVICE;
        break;
      }
    }
    if (nnz32 < 0) { st = GP_EINVAL; break; }
    if (nnz32 > 0 && (!adjncy || !adjwgt)) { st = GP_EINVAL; break; }
    g->nnz = nnz32;
    l0->n = n;
    l0->nnz = nnz32;
    DBuf<int64_t> vtmp;
    if (!l0->ensure(n, nnz32) || !vtmp.ensure(2 * (size_t)n)) { st = GP_ENOMEM; break; }
    hipStream_t s = g->stream;
    if (hipMemcpyAsync(l0->xadj.p, xadj, sizeof(int32_t) * (n + 1), kin, s) != hipSuccess ||
        (nnz32 > 0 &&
         (hipMemcpyAsync(l0->adj.p, adjncy, sizeof(int32_t) * nnz32, kin, s) != hipSuccess ||
          hipMemcpyAsync(l0->w.p, adjwgt, sizeof(int64_t) * nnz32, kin, s) != hipSuccess)) ||
        hipMemcpyAsync(vtmp.p, vwgt, sizeof(int64_t) * 2 * n, kin, s) != hipSuccess ||
        hipMemsetAsync(g->ctrl, 0, sizeof(Ctrl), s) != hipSuccess) {
      vtmp.release();
      st = GP_EDEVICE;
      break;
    }
    if (!launch_split_vwgt(n, vtmp.p, l0->vc.p, l0->vg.p, s) ||
        !launch_validate(n, l0->xadj.p, l0->adj.p, l0->w.p, l0->vc.p, l0->vg.p, g->ctrl, 0, s)) {
      vtmp.release();
      st = GP_EDEVICE;
      break;
    }
    st = read_ctrl(g);
    vtmp.release();
    if (st != GP_OK) break;
    if (g->hctrl->verr & kVInval) { st = GP_EINVAL; break; }
    if (!launch_validate(n, l0->xadj.p, l0->adj.p, l0->w.p, l0->vc.p, l0->vg.p, g->ctrl, 1, s)) {
      st = GP_EDEVICE;
      break;
    }
    if ((st = read_ctrl(g)) != GP_OK) break;
    uint32_t e = g->hctrl->verr;
    if (e & kVRange) { st = GP_ERANGE; break; }
    if (e & kVSelf) { st = GP_ESELF; break; }
    if (g->hctrl->vunsorted) {
      DBuf<int32_t> na;
      DBuf<int64_t> nw;
      if (!na.ensure(nnz32) || !nw.ensure(nnz32)) {
        na.release();
        nw.release();
        st = GP_ENOMEM;
        break;
      }
      if (!launch_sort_rows(n, l0->xadj.p, l0->adj.p, l0->w.p, na.p, nw.p, g->ctrl, s) ||
          (st = read_ctrl(g)) != GP_OK) {
        na.release();
        nw.release();
        if (st == GP_OK) st = GP_EDEVICE;
        break;
      }
      std::swap(l0->adj, na);
      std::swap(l0->w, nw);
      na.release();
      nw.release();
      if (g->hctrl->verr & kVDup) { st = GP_EDUP; break; }
    }
    if (!launch_validate(n, l0->xadj.p, l0->adj.p, l0->w.p, l0->vc.p, l0->vg.p, g->ctrl, 2, s)) {
      st = GP_EDEVICE;
      break;
    }
    if ((st = read_ctrl(g)) != GP_OK) break;
    e = g->hctrl->verr;
    if (e & kVAsym) { st = GP_EASYM; break; }
    if (e & kVOverflow) { st = GP_EOVERFLOW; break; }
    g->sum[0] = (int64_t)g->hctrl->vsum_c;
    g->sum[1] = (int64_t)g->hctrl->vsum_g;
    g->maxv[0] = g->hctrl->vmax_c;
    g->maxv[1] = g->hctrl->vmax_g;
  } while (0);
  if (st != GP_OK) {
    delete g;
    return st;
  }
  *out = g;
  return GP_OK;
}

extern "C" gp_status gp_create(gp_graph** out, int32_t n, const int32_t* xadj,
                               const int32_t* adjncy, const int64_t* adjwgt, const int64_t* vwgt,
                               int32_t flags, void* stream) {
  return create_graph(out, n, xadj, adjncy, adjwgt, vwgt, flags, stream, nullptr);
}

extern "C" {

static gp_status run_partition_inner(gp_graph* g, const gp_options* o, int8_t* part,
                                     gp_result* res, int64_t* trace, int32_t trace_cap);

static gp_status run_partition(gp_graph* g, const gp_options* o, int8_t* part, gp_result* res,
                               int64_t* trace, int32_t trace_cap) {
  if (g && g->profiling) g_prof = &g->prof;
  WsScope ws(g ? g->wsp : tl_ws);
  gp_status st = run_partition_inner(g, o, part, res, trace, trace_cap);
  if (g && g->profiling) {
    (void)hipStreamSynchronize(g->stream);
    prof_collect(g);
    g_prof = nullptr;
  }
  return st;
}

static gp_status run_partition_inner(gp_graph* g, const gp_options* o, int8_t* part,
                                     gp_result* res, int64_t* trace, int32_t trace_cap) {
  if (!g || !res || (g->n > 0 && !part)) return GP_EINVAL;
  gp_status st = check_options(o);
  if (st != GP_OK) return st;
  g->last_levels = -1;  // the levels are rebuilt; none is readable until the run completes
  const int32_t n = g->n;
  const int bal = o->balance_on;
  gp_result r;
  memset(&r, 0, sizeof(r));
  const int64_t W = g->sum[bal];
  int64_t tgt[2], maxw[2];
  host_balance(W, o->ratio, o->eps_ppm, tgt, maxw);
  if (n == 0) {
    r.feasible = 1;
    *res = r;
    return GP_OK;
  }
  hipStream_t s = g->stream;
  if (!g->ensure_scratch()) return GP_ENOMEM;
  const int64_t C = o->coarsen_to;
  const int R = o->match_rounds, P = o->refine_passes;
  // control block
  Ctrl& h = *g->hctrl;
  memset(&h, 0, sizeof(Ctrl));
  h.tgt[0] = tgt[0];
  h.tgt[1] = tgt[1];
  h.ref.maxw[0] = maxw[0];
  h.ref.maxw[1] = maxw[1];
  h.cap = (int64_t)(((__int128)3 * W + 2 * (__int128)C - 1) / (2 * (__int128)C));
  h.maxb = g->maxv[bal];
  HIPCHK(hipMemcpyAsync(g->ctrl, g->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  const Scratch sc = g->scratch();
  std::vector<int64_t> pairs(kMaxLevels + 1, 0);
  int L = 0;
  while (g->lv[L]->n > C) {
    Level* f = g->lv[L];
    if ((int)g->lv.size() <= L + 1) {
      Level* nl = new (std::nothrow) Level();
      if (!nl) return GP_ENOMEM;
      g->lv.push_back(nl);
    }
    Level* c = g->lv[L + 1];
    if (!c->ensure(f->n, f->nnz)) return GP_ENOMEM;
    const LevelView fv = f->view(bal);
    LCHK(launch_level_reset(g->ctrl, L > 0, s));
    const int tw = team_width_for(f->n, f->nnz);
    const uint64_t hs = host_mix64(o->seed ^ (uint64_t)(uint32_t)L);
    if (R == 0) HIPCHK(hipMemsetAsync(f->match.p, 0xff, sizeof(int32_t) * f->n, s));
    g->prof.level = L;
    g->prof.idx = 0;
    // the long-row list is free during matching: it is the second proposal buffer
    // the level's part array is free until the uncoarsening (the free
    // flags), the contraction's member lists and the reduction partials
    // until the contraction (the free lists and their lengths)
    static_assert(kPartials * sizeof(int64_t) >= 2 * kMatchSegMax * sizeof(int32_t),
                  "partials hold both list-length arrays");
    LCHK(launch_match_rounds(fv, f->match.p, (uint8_t*)f->part.p, sc.cmem0, sc.cmem1,
                             (int32_t*)sc.partials, sc.prop, sc.longlist, g->ctrl, R, hs, tw,
                             s));
    LCHK(launch_twohop(fv, f->match.p, g->ctrl, sc, hs, tw,
                       R > 0 ? (uint8_t*)f->part.p : nullptr, s));
    LCHK(launch_contract_a(fv, f->match.p, f->vc.p, f->vg.p, g->ctrl, sc, f->cmap.p, c->vc.p,
                           c->vg.p, s));
    LCHK(launch_contract_b(fv, f->cmap.p, g->ctrl, sc, f->n, c->xadj.p, c->xe.p, c->adj.p,
                           c->w.p, s));
    if ((st = read_ctrl(g)) != GP_OK) return st;
    prof_mark(g, L, true);
    c->n = h.nc;
    c->nnz = h.nnz_c;
    c->gapped = true;
    c->span = h.ubtot;
    pairs[L] = (int64_t)f->n - c->n;
    L++;
    if (20 * (int64_t)c->n > 19 * (int64_t)f->n || L == kMaxLevels) break;
  }
  // coarsest level: made compact (the trials keep its n + 1 offsets in LDS),
  // then the greedy-growing trials
  Level* cl = g->lv[L];
  if (cl->gapped) {
    LCHK(launch_compact_level(g->ctrl, sc, cl->n, (int32_t)cl->nnz, cl->xadj.p, cl->adj.p,
                              cl->w.p, s));
    cl->gapped = false;
  }
  const bool learned = (o->flags & GP_LEARNED) && cl->n > 0 && cl->n <= kMpMaxN;
  {
    const int K = o->init_trials < cl->n ? o->init_trials : cl->n;
    if (!g->ensure_init(cl->n, K)) return GP_ENOMEM;
    const int gs = o->ratio[0] <= o->ratio[1] ? 0 : 1;
    g->prof.level = L;
    LCHK(launch_init(cl->view(bal), K, gs, P, g->ctrl, g->init_scratch(), cl->part.p, s));
    if (learned) {
      const size_t nh = (size_t)cl->n * kMpH;
      if (!g->m_ha.ensure(nh) || !g->m_hb.ensure(nh) || !g->m_inv.ensure(cl->n) ||
          !g->m_score.ensure(cl->n) || !g->m_order.ensure(cl->n) || !g->m_lp.ensure(cl->n) ||
          !g->m_save.ensure(n))
        return GP_ENOMEM;
      MpScratch ms{g->m_ha.p, g->m_hb.p, g->m_inv.p, g->m_score.p, g->m_order.p};
      LCHK(launch_mpnn(cl->view(bal), cl->vc.p, cl->vg.p, o->model, gs, P, g->ctrl, ms,
                       g->m_lp.p, g->ctrl->lpw, s));
    }
  }
  // Time balance: from here on, side 0 is measured by its CPU cost and side
  // 1 by its GPU cost, each against its own bound; the coarsest bisection is
  // refined once more under the two bounds before the uncoarsening
  const bool time_mode = (o->flags & GP_TIME_BALANCE) != 0;
  const int rbal = time_mode ? 0 : bal;  // the refinement's side-0 column
  if (time_mode) {
    int64_t tt[2], mt[2];
    host_balance(g->sum[0], o->ratio, o->eps_ppm, tt, mt);
    maxw[0] = mt[0];
    host_balance(g->sum[1], o->ratio, o->eps_ppm, tt, mt);
    maxw[1] = mt[1];
    LCHK(launch_final_stats(cl->view(bal), cl->vc.p, cl->vg.p, cl->part.p, g->ctrl,
                            team_width_for(cl->n, cl->nnz), sc.partials, s));
    LCHK(launch_time_bounds(g->ctrl, maxw[0], maxw[1], P, s));
    if (cl->n > 0) {
      HIPCHK(hipMemsetAsync(g->r_mark.p, 0, sizeof(int32_t) * cl->n, s));
      const RefArrays ra{g->r_ext.p, g->r_inn.p, g->r_mark.p, cl->vg.p};
      const int tw = team_width_for(cl->n, cl->nnz);
      for (int p = 0; p < P; p++)
        LCHK(launch_refine_pass(cl->view(0), cl->part.p, &g->ctrl->ref, sc.list, sc.partials, tw,
                                &g->ctrl->lvl_pass[L], p, P, ra, s));
    }
  }
  // per-level statistics of the current bisection of level l (GP_TRACE)
  auto record = [&](int l, bool coarsest, int64_t* tr) -> gp_status {
    if (!tr || l >= trace_cap) return GP_OK;
    Level* lvl = g->lv[l];
    LCHK(launch_final_stats(lvl->view(bal), lvl->vc.p, lvl->vg.p, lvl->part.p, g->ctrl,
                            team_width_for(lvl->n, lvl->nnz), sc.partials, s));
    gp_status e2 = read_ctrl(g);
    if (e2 != GP_OK) return e2;
    int64_t* t = tr + 8 * l;
    t[0] = lvl->n;
    t[1] = lvl->nnz;
    t[2] = coarsest ? 0 : h.ref.pass;
    t[3] = coarsest ? 0 : h.ref.total_moves;
    t[4] = h.res_ext / 2;
    t[5] = time_mode ? h.res_time[0] : h.res_load[0];
    t[6] = time_mode ? h.res_time[1] : h.res_load[1];
    t[7] = pairs[l];
    return GP_OK;
  };
  // projection and refinement from the coarsest level down to level 0, then
  // the statistics of the level-0 bisection (read back into h)
  auto uncoarsen = [&](int64_t* tr) -> gp_status {
    gp_status e2 = record(L, true, tr);
    if (e2 != GP_OK) return e2;
    for (int l = L - 1; l >= 0; l--) {
      Level* f = g->lv[l];
      Level* c = g->lv[l + 1];
      g->prof.level = l;
      g->prof.idx = 0;
      const RefArrays ra{g->r_ext.p, g->r_inn.p, g->r_mark.p, time_mode ? f->vg.p : nullptr};
      LCHK(launch_project(f->n, f->cmap.p, c->part.p, f->part.p, &g->ctrl->ref, P, ra.mark, s));
      const int tw = team_width_for(f->n, f->nnz);
      const LevelView fv = f->view(rbal);
      for (int p = 0; p < P; p++) {
        g->prof.idx = p;
        LCHK(launch_refine_pass(fv, f->part.p, &g->ctrl->ref, sc.list, sc.partials, tw,
                                &g->ctrl->lvl_pass[l], p, P, ra, s));
      }
      if ((e2 = record(l, false, tr)) != GP_OK) return e2;
    }
    Level* l0 = g->lv[0];
    LCHK(launch_final_stats(l0->view(bal), l0->vc.p, l0->vg.p, l0->part.p, g->ctrl,
                            team_width_for(l0->n, l0->nnz), sc.partials, s));
    return read_ctrl(g);
  };
  if ((st = uncoarsen(trace)) != GP_OK) return st;
  for (int l = L - 1; l >= 0; l--) prof_mark(g, l, false);
  Level* l0 = g->lv[0];
  int64_t volume = 0;
  if (o->flags & GP_VOLUME) {
    // communication-volume passes on the input graph after its edge-cut
    // refinement; r_ext holds each task's output size, r_mark the counts of
    // successors on the other side
    const LevelView v0 = l0->view(bal);
    const int tw = team_width_for(l0->n, l0->nnz);
    LCHK(launch_vol_out(v0, g->r_ext.p, tw, s));
    LCHK(launch_start_level(&g->ctrl->ref, P, s));
    for (int p = 0; p < P; p++)
      LCHK(launch_vol_pass(v0, l0->part.p, &g->ctrl->ref, sc.list, sc.partials,
                           &g->ctrl->lvl_pass[0], g->r_ext.p, g->r_mark.p, tw, s));
    LCHK(launch_final_stats(v0, l0->vc.p, l0->vg.p, l0->part.p, g->ctrl, tw, sc.partials, s));
    LCHK(launch_vol_total(v0, l0->part.p, g->r_ext.p, g->ctrl, tw, s));
    if ((st = read_ctrl(g)) != GP_OK) return st;
    volume = h.res_vol;
  }
  int used_learned = 0;
  if (learned) {
    // the plain bisection judges the learned one on the input graph: the
    // learned proposal is carried through the same uncoarsening and kept
    // only when it ends strictly better in (infeasible, cut)
    const int64_t p_ext = h.res_ext, p_load[2] = {h.res_load[0], h.res_load[1]};
    const int64_t p_time[2] = {h.res_time[0], h.res_time[1]};
    HIPCHK(hipMemcpyAsync(g->m_save.p, l0->part.p, (size_t)n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(cl->part.p, g->m_lp.p, (size_t)cl->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(g->ctrl->ref.pw, g->ctrl->lpw, 2 * sizeof(int64_t),
                          hipMemcpyDeviceToDevice, s));
    std::vector<int64_t> ltr(trace ? 8 * (size_t)trace_cap : 0, 0);
    if ((st = uncoarsen(trace ? ltr.data() : nullptr)) != GP_OK) return st;
    const int inf_p = (p_load[0] > maxw[0] || p_load[1] > maxw[1]) ? 1 : 0;
    const int inf_l = (h.res_load[0] > maxw[0] || h.res_load[1] > maxw[1]) ? 1 : 0;
    if (inf_l < inf_p || (inf_l == inf_p && h.res_ext < p_ext)) {
      used_learned = 1;
      if (trace) memcpy(trace, ltr.data(), sizeof(int64_t) * ltr.size());
    } else {
      HIPCHK(hipMemcpyAsync(l0->part.p, g->m_save.p, (size_t)n, hipMemcpyDeviceToDevice, s));
      h.res_ext = p_ext;
      h.res_load[0] = p_load[0];
      h.res_load[1] = p_load[1];
      h.res_time[0] = p_time[0];
      h.res_time[1] = p_time[1];
    }
  }
  const hipMemcpyKind kout =
      (g->flags & GP_HOST_PTRS) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HIPCHK(hipMemcpyAsync(part, l0->part.p, (size_t)n, kout, s));
  HIPCHK(hipStreamSynchronize(s));
  r.cut = h.res_ext / 2;
  r.load[0] = time_mode ? h.res_time[0] : h.res_load[0];
  r.load[1] = time_mode ? h.res_time[1] : h.res_load[1];
  r.time[0] = h.res_time[0];
  r.time[1] = h.res_time[1];
  r.feasible = (r.load[0] <= maxw[0] && r.load[1] <= maxw[1]) ? 1 : 0;
  r.levels = L;
  g->last_levels = L;
  r.used_learned = used_learned;
  r.status = GP_OK;
  r.volume = volume;
  *res = r;
  return GP_OK;
}

gp_status gp_model_scores(const void* model, gp_graph* g, float* scores) {
  const MpModel* m = (const MpModel*)model;
  if (!g || !m || m->magic != kMpMagic || (g->n > 0 && !scores)) return GP_EINVAL;
  if (g->n == 0) return GP_OK;
  WsScope ws(g->wsp);
  Level* l0 = g->lv[0];
  const size_t nh = (size_t)g->n * kMpH;
  if (!g->m_ha.ensure(nh) || !g->m_hb.ensure(nh) || !g->m_inv.ensure(g->n) ||
      !g->m_score.ensure(g->n) || !g->m_order.ensure(g->n))
    return GP_ENOMEM;
  MpScratch ms{g->m_ha.p, g->m_hb.p, g->m_inv.p, g->m_score.p, g->m_order.p};
  LCHK(launch_mpnn_scores(l0->view(0), l0->vc.p, l0->vg.p, model, ms, g->stream));
  const hipMemcpyKind k = (g->flags & GP_HOST_PTRS) ? hipMemcpyDeviceToHost
                                                     : hipMemcpyDeviceToDevice;
  HIPCHK(hipMemcpyAsync(scores, ms.score, sizeof(float) * g->n, k, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return GP_OK;
}

gp_status gp_profile_enable(gp_graph* g, int32_t on) {
  if (!g) return GP_EINVAL;
  g->profiling = on != 0;
  return GP_OK;
}

int32_t gp_profile_read(gp_graph* g, gp_prof_row* rows, int32_t cap, int32_t reset) {
  if (!g || (cap > 0 && !rows)) return -1;
  const int32_t n = (int32_t)g->prof_rows.size();
  for (int32_t i = 0; i < n && i < cap; i++) rows[i] = g->prof_rows[i];
  if (reset) g->prof_rows.clear();
  return n;
}

gp_status gp_partition(gp_graph* g, const gp_options* o, int8_t* part, gp_result* res) {
  return run_partition(g, o, part, res, nullptr, 0);
}

gp_status gp_partition_trace(gp_graph* g, const gp_options* o, int8_t* part, gp_result* res,
                             int64_t* trace, int32_t trace_cap) {
  return run_partition(g, o, part, res, trace, trace_cap);
}

gp_status gp_level_read(gp_graph* g, int32_t level, int32_t* n, int64_t* nnz, int32_t* xadj,
                        int32_t* adjncy, int64_t* adjwgt, int64_t* vwgt, int32_t* match,
                        int8_t* part) {
  if (!g || level < 0 || level > g->last_levels || level >= (int32_t)g->lv.size())
    return GP_EINVAL;
  const Level* l = g->lv[level];
  if (n) *n = l->n;
  if (nnz) *nnz = l->nnz;
  hipStream_t s = g->stream;
  const size_t nv = (size_t)l->n, ne = (size_t)l->nnz;
  if (l->gapped && nv > 0 && (xadj || adjncy || adjwgt)) {
    // rows at their upper-bound offsets: gathered into compact form here
    std::vector<int32_t> b(nv), e(nv), ka((size_t)l->span);
    std::vector<int64_t> wa((size_t)l->span);
    HIPCHK(hipMemcpyAsync(b.data(), l->xadj.p, 4 * nv, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(e.data(), l->xe.p, 4 * nv, hipMemcpyDeviceToHost, s));
    if (l->span > 0) {
      HIPCHK(hipMemcpyAsync(ka.data(), l->adj.p, 4 * (size_t)l->span, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(wa.data(), l->w.p, 8 * (size_t)l->span, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    size_t o = 0;
    for (size_t v = 0; v < nv; v++) {
      if (xadj) xadj[v] = (int32_t)o;
      for (int32_t q = b[v]; q < e[v]; q++, o++) {
        if (adjncy) adjncy[o] = ka[q];
        if (adjwgt) adjwgt[o] = wa[q];
      }
    }
    if (xadj) xadj[nv] = (int32_t)o;
  } else {
    if (xadj) HIPCHK(hipMemcpyAsync(xadj, l->xadj.p, 4 * (nv + 1), hipMemcpyDeviceToHost, s));
    if (adjncy && ne)
      HIPCHK(hipMemcpyAsync(adjncy, l->adj.p, 4 * ne, hipMemcpyDeviceToHost, s));
    if (adjwgt && ne)
      HIPCHK(hipMemcpyAsync(adjwgt, l->w.p, 8 * ne, hipMemcpyDeviceToHost, s));
  }
  if (vwgt && nv) {
    HIPCHK(hipMemcpy2DAsync(vwgt, 16, l->vc.p, 8, 8, nv, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpy2DAsync(vwgt + 1, 16, l->vg.p, 8, 8, nv, hipMemcpyDeviceToHost, s));
  }
  if (match && nv && level < g->last_levels)
    HIPCHK(hipMemcpyAsync(match, l->match.p, 4 * nv, hipMemcpyDeviceToHost, s));
  if (part && nv) HIPCHK(hipMemcpyAsync(part, l->part.p, nv, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return GP_OK;
}

// k-way partition by recursive bisection of part ranges (see gp_kway.hip)
gp_status gp_partition_kway(gp_graph* g, int32_t k, const int64_t* ratio, const gp_options* o,
                            int32_t* part, int64_t* load, gp_kway_result* res) {
  if (!g || !ratio || !res || k < 1 || k > kKwayMax || (g->n > 0 && !part)) return GP_EINVAL;
  const int64_t lim = (int64_t)1 << 40;
  int64_t rsum = 0;
  for (int i = 0; i < k; i++) {
    if (ratio[i] < 0 || ratio[i] >= lim) return GP_EINVAL;
    rsum += ratio[i];
  }
  if (rsum == 0 || rsum >= lim) return GP_EINVAL;
  gp_options o2 = *o;
  o2.ratio[0] = 1;
  o2.ratio[1] = 1;
  if (o2.flags & GP_LEARNED) return GP_EMODEL;
  if (o2.flags & (GP_TIME_BALANCE | GP_VOLUME)) return GP_EINVAL;
  gp_status st = check_options(&o2);
  if (st != GP_OK) return st;
  const int32_t n = g->n;
  gp_kway_result r;
  memset(&r, 0, sizeof(r));
  r.feasible = 1;
  if (n == 0) {
    if (load)
      for (int i = 0; i < k; i++) load[i] = 0;
    *res = r;
    return GP_OK;
  }
  hipStream_t s = g->stream;
  WsScope ws(g->wsp);
  Level* l0 = g->lv[0];
  const int ntiles = (n + 1023) / 1024;
  if (!g->kw_label.ensure(n) || !g->kw_keep.ensure(n) || !g->kw_newid.ensure(n) ||
      !g->kw_sxadj.ensure((size_t)n + 1) || !g->kw_sadj.ensure((size_t)g->nnz) ||
      !g->kw_sw.ensure((size_t)g->nnz) || !g->kw_svwgt.ensure(2 * (size_t)n) ||
      !g->kw_tiles.ensure(2 * (size_t)ntiles) || !g->kw_tot.ensure(2) ||
      !g->kw_acc.ensure((size_t)k + 1) || !g->kw_spart.ensure(n))
    return GP_ENOMEM;
  int32_t* label = g->kw_label.p;
  LCHK(launch_kw_zero(label, n, g->kw_acc.p, k + 1, s));
  // ranges still to split, depth first; the subproblems are independent, so
  // the order does not change the result
  std::vector<std::pair<int32_t, int32_t>> todo{{0, k}};
  while (!todo.empty()) {
    const int32_t lo = todo.back().first, hi = todo.back().second;
    todo.pop_back();
    if (hi - lo < 2) continue;
    const int32_t mid = lo + (hi - lo) / 2;
    int64_t r0 = 0, r1 = 0;
    for (int i = lo; i < mid; i++) r0 += ratio[i];
    for (int i = mid; i < hi; i++) r1 += ratio[i];
    LCHK(launch_kw_extract_a(n, l0->xadj.p, l0->adj.p, label, lo, g->kw_keep.p, g->kw_tiles.p,
                             g->kw_tiles.p + ntiles, g->kw_tot.p, s));
    int64_t tot[2];
    HIPCHK(hipMemcpyAsync(tot, g->kw_tot.p, sizeof(tot), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tot[0] == 0) continue;  // no vertex carries this range
    LCHK(launch_kw_extract_b(n, l0->xadj.p, l0->adj.p, l0->w.p, l0->vc.p, l0->vg.p, label, lo,
                             g->kw_keep.p, g->kw_tiles.p, g->kw_tiles.p + ntiles, g->kw_tot.p,
                             g->kw_newid.p, g->kw_sxadj.p, g->kw_sadj.p, g->kw_sw.p,
                             g->kw_svwgt.p, s));
    if (r0 + r1 > 0) {
      gp_graph* sub = nullptr;
      st = create_graph(&sub, (int32_t)tot[0], g->kw_sxadj.p, g->kw_sadj.p, g->kw_sw.p,
                        g->kw_svwgt.p, 0, s, g->wsp);
      if (st != GP_OK) return st;
      o2.ratio[0] = r0;
      o2.ratio[1] = r1;
      gp_result br;
      st = run_partition(sub, &o2, g->kw_spart.p, &br, nullptr, 0);
      gp_destroy(sub);
      if (st != GP_OK) return st;
      r.feasible &= br.feasible;
      r.bisections++;
      LCHK(launch_kw_apply(n, label, lo, mid, g->kw_newid.p, g->kw_spart.p, s));
    }
    todo.push_back({mid, hi});
    todo.push_back({lo, mid});
  }
  const int64_t* b = o->balance_on ? l0->vg.p : l0->vc.p;
  LCHK(launch_kw_stats(n, l0->xadj.p, l0->adj.p, l0->w.p, label, b, g->kw_acc.p,
                       g->kw_acc.p + 1, s));
  std::vector<int64_t> acc((size_t)k + 1);
  HIPCHK(hipMemcpyAsync(acc.data(), g->kw_acc.p, sizeof(int64_t) * (k + 1),
                        hipMemcpyDeviceToHost, s));
  const hipMemcpyKind kout =
      (g->flags & GP_HOST_PTRS) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HIPCHK(hipMemcpyAsync(part, label, sizeof(int32_t) * (size_t)n, kout, s));
  HIPCHK(hipStreamSynchronize(s));
  r.cut = acc[0] / 2;
  if (load)
    for (int i = 0; i < k; i++) load[i] = acc[1 + i];
  *res = r;
  return GP_OK;
}

}  // extern "C"
