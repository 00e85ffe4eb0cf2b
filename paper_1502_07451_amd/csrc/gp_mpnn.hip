// gp_mpnn.hip - learned coarsest-level proposal: inference kernels.
//
// A 3-layer message-passing network (hidden size 64, BF16 weights, FP32
// accumulation) scores the vertices of the coarsest graph; the best scores
// fill the grown side; the LDS refinement of the initial bisection follows.
// That bisection is projected and refined down to the input graph beside the
// plain one, and replaces it only when it ends strictly better in
// (infeasible, cut) there.  The network orders vertices, nothing more: the
// partition arithmetic stays integer.
//
// Inference uses only correctly rounded FP32 fma and multiplication in a
// fixed order, and round-to-nearest-even to BF16, so it is reproducible
// exactly on a CPU:
//   phi(x)  = (bitlen(x) - 1) + (8 bits after the leading one) / 256, phi(0) = 0
//   x_v     = [phi(cpu), phi(gpu), phi(deg), phi(sum of incident w)]
//   e_vu    = phi(w_vu) / 64, inv_v = 1/deg_v (0 for deg 0)
//   h0[j]   = bf16(relu(fma chain k=0..3 of Win[j][k] x[k] from b_in[j]))
//   m[k]    = bf16((fma chain over the row, in row order, of e_vu h_u[k] from 0) * inv_v)
//   h'[j]   = bf16(relu(fma chain of Ws[j][k] h[k], k ascending, then Wn[j][k] m[k],
//                       k ascending, from b[j]))
//   score   = fma chain of wo[k] h3[k], k ascending, from bo
// Parameter blob (BF16 bits): Win[64][4], b_in[64], 3 x (Ws[64][64],
// Wn[64][64], b[64]), wo[64], bo - 25,153 values.
#include <stdio.h>
#include <string.h>

#include <new>

#include "../../include/gp.h"
#include "gp_launch.h"
#include "gp_mpnn.h"
#include "gp_phases.h"

namespace gpk {

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float relu_f(float a) { return a > 0.0f ? a : 0.0f; }

// input layer: one wave per vertex, lane j computes h0[j]
__global__ __launch_bounds__(kBlock) void k_mp_input(LevelView lv, const int64_t* vc,
                                                     const int64_t* vg, const uint16_t* P,
                                                     uint16_t* h0, float* inv) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int64_t nw = (int64_t)gridDim.x * kBlock / 64;
  for (int64_t v = wv; v < lv.n; v += nw) {
    const int32_t e0 = lv.xadj[v], e1 = lv.xend[v];
    int64_t tw = 0;
    for (int32_t q = e0 + lane; q < e1; q += 64) tw += lv.w[q];
    tw = team_sum<64>(tw);
    const int64_t deg = e1 - e0;
    float x[4] = {mp_phi(vc[v]), mp_phi(vg[v]), mp_phi(deg), mp_phi(tw)};
    float acc = bf2f(P[kMpOffBin + lane]);
#pragma unroll
    for (int k = 0; k < 4; k++) acc = __builtin_fmaf(bf2f(P[kMpOffWin + lane * 4 + k]), x[k], acc);
    h0[v * kMpH + lane] = f2bf(relu_f(acc));
    if (lane == 0) inv[v] = e1 > e0 ? __frcp_rn((float)(e1 - e0)) : 0.0f;
  }
}

// message-passing layer l: one wave per vertex, lane k aggregates m[k],
// lane j produces h'[j]; the layer's weights are staged transposed in LDS
__global__ __launch_bounds__(kBlock) void k_mp_layer(LevelView lv, const uint16_t* P, int l,
                                                     const uint16_t* hin, uint16_t* hout,
                                                     const float* inv) {
  __shared__ uint16_t WsT[kMpH * kMpH];
  __shared__ uint16_t WnT[kMpH * kMpH];
  __shared__ uint16_t bb[kMpH];
  const uint16_t* Ws = P + kMpOffL(l);
  const uint16_t* Wn = Ws + kMpH * kMpH;
  for (int i = threadIdx.x; i < kMpH * kMpH; i += kBlock) {
    const int j = i / kMpH, k = i % kMpH;
    WsT[k * kMpH + j] = Ws[i];
    WnT[k * kMpH + j] = Wn[i];
  }
  if (threadIdx.x < kMpH) bb[threadIdx.x] = Wn[kMpH * kMpH + threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int64_t nw = (int64_t)gridDim.x * kBlock / 64;
  for (int64_t v = wv; v < lv.n; v += nw) {
    float acc = 0.0f;
    for (int32_t q = lv.xadj[v]; q < lv.xend[v]; q++) {
      const float e = mp_phi(lv.w[q]) / 64.0f;
      acc = __builtin_fmaf(e, bf2f(hin[(int64_t)lv.adj[q] * kMpH + lane]), acc);
    }
    const float m = bf2f(f2bf(acc * inv[v]));
    const float hv = bf2f(hin[v * kMpH + lane]);
    float a = bf2f(bb[lane]);
    for (int k = 0; k < kMpH; k++) a = __builtin_fmaf(bf2f(WsT[k * kMpH + lane]), __shfl(hv, k, 64), a);
    for (int k = 0; k < kMpH; k++) a = __builtin_fmaf(bf2f(WnT[k * kMpH + lane]), __shfl(m, k, 64), a);
    hout[v * kMpH + lane] = f2bf(relu_f(a));
  }
}

__global__ __launch_bounds__(kBlock) void k_mp_score(int32_t n, const uint16_t* P,
                                                     const uint16_t* h, float* score) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int64_t nw = (int64_t)gridDim.x * kBlock / 64;
  for (int64_t v = wv; v < n; v += nw) {
    const float hv = bf2f(h[v * kMpH + lane]);
    const float wo = bf2f(P[kMpOffWo + lane]);
    float acc = bf2f(P[kMpOffBo]);
    for (int k = 0; k < kMpH; k++) acc = __builtin_fmaf(__shfl(wo, k, 64), __shfl(hv, k, 64), acc);
    if (lane == 0) score[v] = acc;
  }
}

// Proposal and refinement for the coarsest graph, one block.  Phase 1 sorts
// (score key desc, id asc) in LDS and writes the order to `order`; phase 2
// fills the grown side, computes the gains of that assignment and refines
// it.  The refined bisection goes to lp_out and its part weights to
// lpw_out; the host driver carries it through the uncoarsening beside the
// plain one and keeps the better of the two on the input graph.
__global__ __launch_bounds__(kBlock) void k_mp_propose(LevelView lv, const float* score,
                                                       int32_t* order, int gs, int npass,
                                                       const Ctrl* ctrl, int8_t* lp_out,
                                                       int64_t* lpw_out) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ SelShared sel;
  __shared__ RefCtl srf;
  __shared__ int64_t sml[kBlock / 64];
  const int32_t n = lv.n;
  const int gb = 1 - gs;
  // ---- phase 1: order by (score desc, id asc)
  {
    uint64_t* key = (uint64_t*)lds;
    const int P2 = next_pow2(n);
    for (int i = threadIdx.x; i < P2; i += kBlock) {
      uint64_t k = 0;
      if (i < n) {
        const int32_t b = __float_as_int(score[i]);
        const uint32_t sk = (uint32_t)(b < 0 ? (b ^ 0x7fffffff) : b) ^ 0x80000000u;
        k = ((uint64_t)sk << 32) | (uint32_t)(~(uint32_t)i);
      }
      key[i] = k;  // padding (0) sorts last in descending order
    }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < P2 / 2; i += kBlock) {
          const int lo = (i / stride) * stride * 2 + (i % stride), hi = lo + stride;
          const bool desc = (lo & size) == 0;
          const uint64_t a = key[lo], b = key[hi];
          if ((a < b) == desc && a != b) {
            key[lo] = b;
            key[hi] = a;
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += kBlock) order[i] = (int32_t)(~(uint32_t)key[i]);
    __syncthreads();
  }
  // ---- phase 2: fill, gains, refinement
  int64_t* s_gain = (int64_t*)lds;
  int64_t* s_b = s_gain + n;
  int8_t* s_part = (int8_t*)(s_b + n);
  int8_t* s_adj = s_part + n;
  int8_t* s_mv = s_adj + n;
  int64_t W = 0;
  for (int32_t v = threadIdx.x; v < n; v += kBlock) {
    s_b[v] = lv.b[v];
    s_part[v] = (int8_t)gb;
    s_adj[v] = 0;
    s_mv[v] = 0;
    W += s_b[v];
  }
  W = block_sum<kBlock, int64_t>(W, sml);
  __shared__ int64_t s_pg;
  if (threadIdx.x == 0) {
    const int64_t tg = ctrl->tgt[gs], mg = ctrl->ref.maxw[gs];
    int64_t pg = 0;
    for (int32_t i = 0; i < n && pg < tg; i++) {
      const int32_t v = order[i];
      if (pg + s_b[v] <= mg) {
        s_part[v] = (int8_t)gs;
        pg += s_b[v];
      }
    }
    s_pg = pg;
  }
  __syncthreads();
  for (int32_t v = threadIdx.x; v < n; v += kBlock) {
    int64_t g = 0;
    const int8_t pv = s_part[v];
    constexpr int U = 8;  // row entries in flight per thread
    const int32_t e1 = lv.xend[v];
    for (int32_t e = lv.xadj[v]; e < e1; e += U) {
      int32_t y[U];
      int64_t w[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        y[u] = e + u < e1 ? lv.adj[e + u] : 0;
        w[u] = e + u < e1 ? lv.w[e + u] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; u++)
        if (e + u < e1) g += s_part[y[u]] != pv ? w[u] : -w[u];
    }
    s_gain[v] = g;
  }
  if (threadIdx.x == 0) {
    memset(&srf, 0, sizeof(srf));
    srf.maxw[0] = ctrl->ref.maxw[0];
    srf.maxw[1] = ctrl->ref.maxw[1];
    srf.pw[gs] = s_pg;
    srf.pw[gb] = W - s_pg;
    srf.pass = 0;
    srf.z = 0;
    srf.npass = npass;
    srf.done = npass <= 0 ? 1 : 0;
  }
  __syncthreads();
  lds_refine<kBlock>(lv, s_gain, s_b, s_part, s_mv, srf, sel);
  for (int32_t v = threadIdx.x; v < n; v += kBlock) lp_out[v] = s_part[v];
  if (threadIdx.x == 0) {
    lpw_out[0] = srf.pw[0];
    lpw_out[1] = srf.pw[1];
  }
}

bool launch_mpnn_scores(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const void* model, const MpScratch& ms, hipStream_t s);

bool launch_mpnn(const LevelView& lv, const int64_t* vc, const int64_t* vg, const void* model,
                 int gs, int npass, const Ctrl* ctrl, const MpScratch& ms, int8_t* lp_out,
                 int64_t* lpw_out, hipStream_t s) {
  if (!launch_mpnn_scores(lv, vc, vg, model, ms, s)) return false;
  const size_t dyn = (size_t)lv.n * 19 + 16 > (size_t)next_pow2_host(lv.n) * 8
                         ? (size_t)lv.n * 19 + 16
                         : (size_t)next_pow2_host(lv.n) * 8;
  k_mp_propose<<<1, kBlock, dyn, s>>>(lv, ms.score, ms.order, gs, npass, ctrl, lp_out, lpw_out);
  return hipGetLastError() == hipSuccess;
}

bool launch_mpnn_scores(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const void* model, const MpScratch& ms, hipStream_t s) {
  const MpModel* m = (const MpModel*)model;
  const int grid = (int)((lv.n + 3) / 4 < 4096 ? (lv.n + 3) / 4 : 4096);
  const int g1 = grid > 0 ? grid : 1;
  k_mp_input<<<g1, kBlock, 0, s>>>(lv, vc, vg, m->p, ms.ha, ms.inv);
  if (hipGetLastError() != hipSuccess) return false;
  uint16_t* hin = ms.ha;
  uint16_t* hout = ms.hb;
  for (int l = 0; l < 3; l++) {
    k_mp_layer<<<g1, kBlock, 0, s>>>(lv, m->p, l, hin, hout, ms.inv);
    if (hipGetLastError() != hipSuccess) return false;
    uint16_t* t = hin;
    hin = hout;
    hout = t;
  }
  k_mp_score<<<g1, kBlock, 0, s>>>(lv.n, m->p, hin, ms.score);
  return hipGetLastError() == hipSuccess;
}

}  // namespace gpk

using namespace gpk;

extern "C" {

gp_status gp_model_create(const uint16_t* params, int32_t count, const void** model) {
  if (!model || !params || count != kMpNParam) return GP_EINVAL;
  *model = nullptr;
  MpModel* m = new (std::nothrow) MpModel();
  if (!m) return GP_ENOMEM;
  if (hipMalloc((void**)&m->p, sizeof(uint16_t) * kMpNParam) != hipSuccess) {
    (void)hipGetLastError();
    delete m;
    return GP_ENOMEM;
  }
  if (hipMemcpy(m->p, params, sizeof(uint16_t) * kMpNParam, hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(m->p);
    delete m;
    return GP_EDEVICE;
  }
  m->magic = kMpMagic;
  *model = m;
  return GP_OK;
}

gp_status gp_model_load(const char* path, const void** model) {
  if (!model || !path) return GP_EINVAL;
  *model = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return GP_EINVAL;
  // the file is the raw blob: kMpNParam little-endian BF16 values, nothing else
  uint16_t* buf = new (std::nothrow) uint16_t[kMpNParam + 1];
  if (!buf) {
    fclose(f);
    return GP_ENOMEM;
  }
  const size_t got = fread(buf, sizeof(uint16_t), kMpNParam + 1, f);
  const bool err = ferror(f) != 0;
  fclose(f);
  gp_status st = (err || got != (size_t)kMpNParam) ? GP_EMODEL
                                                   : gp_model_create(buf, kMpNParam, model);
  delete[] buf;
  return st;
}

void gp_model_free(const void* model) {
  MpModel* m = (MpModel*)model;
  if (!m || m->magic != kMpMagic) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(m->p);
  m->magic = 0;
  delete m;
}

}  // extern "C"
