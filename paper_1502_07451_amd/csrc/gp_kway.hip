// gp_kway.hip - kernels of the k-way partition by recursive bisection.
//
// The paper leaves more than two processors (CPU + GPU + further
// accelerators) to future work, with each processor's share following the
// generalisation of Eq. (1): inversely proportional to its execution time.
// Here a k-way partition is built by recursive bisection: the vertices that
// carry part range [lo, hi) are split by the two-way pipeline into the
// ranges [lo, mid) and [mid, hi), mid = lo + (hi - lo) / 2, with the target
// ratio (sum of the shares of [lo, mid), sum of the shares of [mid, hi)).
// label[v] is the lower end of the range vertex v currently belongs to; it
// ends as v's part.  Each bisection runs on the subgraph induced by the
// vertices labelled lo, in ascending id order (so its rows stay sorted),
// extracted here from the input graph.  All arithmetic is integer.
#include "gp_launch.h"
#include "gp_phases.h"

namespace gpk {

constexpr int kKwTile = 1024;  // vertices per tile of the ordered scans (4 per thread)

// per tile: members of the subgraph (label == lo) and the entries their rows
// keep (neighbours also labelled lo); keep[v] = the kept count of member v
__global__ __launch_bounds__(kBlock) void k_kw_count(int32_t n, const int32_t* xadj,
                                                     const int32_t* adj, const int32_t* label,
                                                     int32_t lo, int32_t* keep,
                                                     int64_t* tile_m, int64_t* tile_e) {
  __shared__ int64_t sml[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kKwTile + threadIdx.x * 4;
  int64_t m = 0, e = 0;
  for (int j = 0; j < 4; j++) {
    const int64_t v = base + j;
    if (v >= n || label[v] != lo) continue;
    int32_t k = 0;
    const int32_t e1 = xadj[v + 1];
    for (int32_t q = xadj[v]; q < e1; q++) k += label[adj[q]] == lo;
    keep[v] = k;
    m++;
    e += k;
  }
  m = block_sum<kBlock, int64_t>(m, sml);
  e = block_sum<kBlock, int64_t>(e, sml);
  if (threadIdx.x == 0) {
    tile_m[blockIdx.x] = m;
    tile_e[blockIdx.x] = e;
  }
}

// exclusive scans of the tile totals (one block); tot[0..1] = member and
// entry totals
__global__ __launch_bounds__(kBlock) void k_kw_scan(int64_t* tile_m, int64_t* tile_e, int ntiles,
                                                    int64_t* tot) {
  __shared__ int64_t sml[kBlock / 64];
  int64_t cm = 0, ce = 0;
  for (int t0 = 0; t0 < ntiles; t0 += kBlock) {
    const int t = t0 + threadIdx.x;
    const int64_t a = t < ntiles ? tile_m[t] : 0, b = t < ntiles ? tile_e[t] : 0;
    int64_t ta, tb;
    const int64_t ea = block_exscan<kBlock, int64_t>(a, sml, &ta);
    const int64_t eb = block_exscan<kBlock, int64_t>(b, sml, &tb);
    if (t < ntiles) {
      tile_m[t] = cm + ea;
      tile_e[t] = ce + eb;
    }
    cm += ta;
    ce += tb;
  }
  if (threadIdx.x == 0) {
    tot[0] = cm;
    tot[1] = ce;
  }
}

// new ids (ascending old id), row offsets and vertex weights of the subgraph
__global__ __launch_bounds__(kBlock) void k_kw_ids(int32_t n, const int32_t* label, int32_t lo,
                                                   const int32_t* keep, const int64_t* tile_m,
                                                   const int64_t* tile_e, const int64_t* vc,
                                                   const int64_t* vg, int32_t* newid,
                                                   int32_t* sxadj, int64_t* svwgt,
                                                   const int64_t* tot) {
  __shared__ int64_t sml[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kKwTile + threadIdx.x * 4;
  int64_t m = 0, e = 0;
  bool mem[4];
  for (int j = 0; j < 4; j++) {
    const int64_t v = base + j;
    mem[j] = v < n && label[v] == lo;
    if (mem[j]) {
      m++;
      e += keep[v];
    }
  }
  int64_t tm, te;
  int64_t id = tile_m[blockIdx.x] + block_exscan<kBlock, int64_t>(m, sml, &tm);
  int64_t off = tile_e[blockIdx.x] + block_exscan<kBlock, int64_t>(e, sml, &te);
  for (int j = 0; j < 4; j++) {
    if (!mem[j]) continue;
    const int64_t v = base + j;
    newid[v] = (int32_t)id;
    sxadj[id] = (int32_t)off;
    svwgt[2 * id] = vc[v];
    svwgt[2 * id + 1] = vg[v];
    off += keep[v];
    id++;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sxadj[tot[0]] = (int32_t)tot[1];
}

// the kept entries of each member row, in row order (a 16-lane team per row)
__global__ __launch_bounds__(kBlock) void k_kw_fill(int32_t n, const int32_t* xadj,
                                                    const int32_t* adj, const int64_t* w,
                                                    const int32_t* label, int32_t lo,
                                                    const int32_t* newid, const int32_t* sxadj,
                                                    int32_t* sadj, int64_t* sw) {
  constexpr int TW = 16;
  const int lane = threadIdx.x & (TW - 1);
  const int64_t team = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / TW;
  const int64_t nteams = (int64_t)gridDim.x * kBlock / TW;
  const int tb = lane_id() & ~(TW - 1);
  const int64_t iters = (n + nteams - 1) / nteams;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t v = team + it * nteams;
    const bool member = v < n && label[v] == lo;
    int32_t out = member ? sxadj[newid[v]] : 0;
    const int32_t e0 = member ? xadj[v] : 0, e1 = member ? xadj[v + 1] : 0;
    // every lane of the wave runs the same number of chunks for the ballots
    int32_t len = e1 - e0;
    int32_t chunks = (len + TW - 1) / TW;
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      const int32_t oc = __shfl_xor(chunks, o, 64);
      chunks = oc > chunks ? oc : chunks;
    }
    for (int32_t c = 0; c < chunks; c++) {
      const int32_t q = e0 + c * TW + lane;
      const bool in = q < e1;
      const int32_t u = in ? adj[q] : 0;
      const bool kp = in && label[u] == lo;
      const uint64_t bm = __ballot(kp);
      const uint64_t mine = (bm >> tb) & 0xffffull;
      if (kp) {
        const int pos = __popcll(mine & ((1ull << lane) - 1ull));
        sadj[out + pos] = newid[u];
        sw[out + pos] = w[q];
      }
      out += __popcll(mine);
    }
  }
}

// vertices on side 1 of the subgraph's bisection move to range [mid, hi)
__global__ __launch_bounds__(kBlock) void k_kw_apply(int32_t n, int32_t* label, int32_t lo,
                                                     int32_t mid, const int32_t* newid,
                                                     const int8_t* spart) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock)
    if (label[v] == lo && spart[newid[v]] == 1) label[v] = mid;
}

// cut (sum over vertices of the weight to other parts) and the balance
// weight of every part, by integer atomics (order-independent)
__global__ __launch_bounds__(kBlock) void k_kw_stats(int32_t n, const int32_t* xadj,
                                                     const int32_t* adj, const int64_t* w,
                                                     const int32_t* label, const int64_t* b,
                                                     int64_t* ext_sum, int64_t* load) {
  __shared__ int64_t sml[kBlock / 64];
  int64_t ext = 0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t p = label[v];
    const int32_t e1 = xadj[v + 1];
    for (int32_t q = xadj[v]; q < e1; q++)
      if (label[adj[q]] != p) ext += w[q];
    atomicAdd((unsigned long long*)&load[p], (unsigned long long)b[v]);
  }
  ext = block_sum<kBlock, int64_t>(ext, sml);
  if (threadIdx.x == 0 && ext) atomicAdd((unsigned long long*)ext_sum, (unsigned long long)ext);
}

__global__ void k_kw_zero(int32_t* label, int32_t n, int64_t* acc, int nacc) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    label[v] = 0;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nacc; i += blockDim.x) acc[i] = 0;
}

static int kw_grid(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

#define KW_CHECK()                         \
  do {                                     \
    if (hipGetLastError() != hipSuccess)   \
      return false;                        \
  } while (0)

bool launch_kw_zero(int32_t* label, int32_t n, int64_t* acc, int nacc, hipStream_t s) {
  k_kw_zero<<<kw_grid(n, kBlock, 4096), kBlock, 0, s>>>(label, n, acc, nacc);
  KW_CHECK();
  return true;
}

bool launch_kw_extract_a(int32_t n, const int32_t* xadj, const int32_t* adj, const int32_t* label,
                         int32_t lo, int32_t* keep, int64_t* tile_m, int64_t* tile_e,
                         int64_t* tot, hipStream_t s) {
  const int ntiles = (n + kKwTile - 1) / kKwTile;
  k_kw_count<<<ntiles > 0 ? ntiles : 1, kBlock, 0, s>>>(n, xadj, adj, label, lo, keep, tile_m,
                                                        tile_e);
  KW_CHECK();
  k_kw_scan<<<1, kBlock, 0, s>>>(tile_m, tile_e, ntiles, tot);
  KW_CHECK();
  return true;
}

bool launch_kw_extract_b(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                         const int64_t* vc, const int64_t* vg, const int32_t* label, int32_t lo,
                         const int32_t* keep, const int64_t* tile_m, const int64_t* tile_e,
                         const int64_t* tot, int32_t* newid, int32_t* sxadj, int32_t* sadj,
                         int64_t* sw, int64_t* svwgt, hipStream_t s) {
  const int ntiles = (n + kKwTile - 1) / kKwTile;
  k_kw_ids<<<ntiles > 0 ? ntiles : 1, kBlock, 0, s>>>(n, label, lo, keep, tile_m, tile_e, vc, vg,
                                                      newid, sxadj, svwgt, tot);
  KW_CHECK();
  k_kw_fill<<<kw_grid((int64_t)n * 16, kBlock, 8192), kBlock, 0, s>>>(n, xadj, adj, w, label, lo,
                                                                      newid, sxadj, sadj, sw);
  KW_CHECK();
  return true;
}

bool launch_kw_apply(int32_t n, int32_t* label, int32_t lo, int32_t mid, const int32_t* newid,
                     const int8_t* spart, hipStream_t s) {
  k_kw_apply<<<kw_grid(n, kBlock, 4096), kBlock, 0, s>>>(n, label, lo, mid, newid, spart);
  KW_CHECK();
  return true;
}

bool launch_kw_stats(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                     const int32_t* label, const int64_t* b, int64_t* ext_sum, int64_t* load,
                     hipStream_t s) {
  k_kw_stats<<<kw_grid(n, kBlock, 4096), kBlock, 0, s>>>(n, xadj, adj, w, label, b, ext_sum,
                                                         load);
  KW_CHECK();
  return true;
}

}  // namespace gpk
