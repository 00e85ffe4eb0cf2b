// gp_train.hip - training kernels of the learned coarsest-level proposal.
//
// The network of gp_mpnn.hip is trained on coarsest graphs produced by the
// partition pipeline, with labels = the plain pipeline's refined coarsest
// bisection (1 = vertex on the grown side).  Loss: binary cross-entropy with
// logits, vertex v of graph g weighted by b_v / W_g, averaged over the
// graphs of a mini-batch.  Optimiser: Adam on FP32 master weights; the
// forward pass uses their BF16 copies.
//
// Dense layers [H | M] x [Ws | Wn]^T and their backward products run on the
// matrix cores (v_mfma_f32_32x32x8_bf16, FP32 accumulation); message
// aggregation and its transpose are CSR gathers (the graph is symmetric, so
// the transpose reuses the same rows).  Training is not bit-exact: its
// gradients are checked against an FP64 reference within a tolerance.
//
// MFMA 32x32x8 operand layout (per wave of 64 lanes, l = lane):
//   A (32 x 8):  lane l holds A[l % 32][4 (l / 32) + v], v = 0..3
//   B (8 x 32):  lane l holds B[4 (l / 32) + v][l % 32]
//   D (32 x 32): lane l, element e holds D[8 (e / 4) + 4 (l / 32) + e % 4][l % 32]
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/gp.h"
#include "gp_dev.h"
#include "gp_mpnn.h"

namespace gpk {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float tbf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t tf2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------- training set
// Global-id CSR of all training graphs (graph g: vertices voff[g]..voff[g+1]),
// per-vertex inputs x (4), 1/deg, loss weight b_v / W_g and label, per-entry
// edge coefficient.
struct TrainData {
  int32_t G;
  int64_t N, NNZ;
  int64_t* voff;   // G+1
  int64_t* xadj;   // N+1, global entry offsets
  int32_t* adj;    // NNZ, global vertex ids
  float* e;        // NNZ
  float* x;        // N x 4
  float* inv;      // N
  float* cw;       // N
  float* y;        // N
};

// one block per graph: global ids, inputs, weights
__global__ __launch_bounds__(kBlock) void k_tr_prep(int32_t G, const int64_t* voff,
                                                    const int64_t* eoff, const int32_t* xadj,
                                                    const int32_t* adj, const int64_t* w,
                                                    const int64_t* vwgt, const int8_t* label,
                                                    int bal, TrainData d) {
  __shared__ int64_t sml[kBlock / 64];
  for (int g = blockIdx.x; g < G; g += gridDim.x) {
    const int64_t v0 = voff[g], e0 = eoff[g];
    const int32_t n = (int32_t)(voff[g + 1] - v0);
    const int32_t* xa = xadj + v0 + g;
    int64_t W = 0;
    for (int32_t v = threadIdx.x; v < n; v += kBlock) W += vwgt[2 * (v0 + v) + bal];
    W = block_sum<kBlock, int64_t>(W, sml);
    for (int32_t v = threadIdx.x; v < n; v += kBlock) {
      const int64_t gv = v0 + v;
      const int32_t a = xa[v], b = xa[v + 1];
      int64_t tw = 0;
      for (int32_t q = a; q < b; q++) {
        d.adj[e0 + q] = (int32_t)(v0 + adj[e0 + q]);
        d.e[e0 + q] = mp_phi(w[e0 + q]) / 64.0f;
        tw += w[e0 + q];
      }
      d.xadj[gv] = e0 + a;
      if (v == n - 1) d.xadj[gv + 1] = e0 + b;
      const int64_t deg = b - a;
      d.x[4 * gv + 0] = mp_phi(vwgt[2 * gv]);
      d.x[4 * gv + 1] = mp_phi(vwgt[2 * gv + 1]);
      d.x[4 * gv + 2] = mp_phi(deg);
      d.x[4 * gv + 3] = mp_phi(tw);
      d.inv[gv] = b > a ? __frcp_rn((float)(b - a)) : 0.0f;
      const int64_t bv = vwgt[2 * gv + bal];
      d.cw[gv] = W > 0 ? (float)((double)bv / (double)W) : 1.0f / (float)n;
      d.y[gv] = label[gv] ? 1.0f : 0.0f;
    }
  }
}

// --------------------------------------------------------------- forward
// rows [v0, v0 + nb) of the training set form the mini-batch
__global__ __launch_bounds__(kBlock) void k_tr_input(TrainData d, int64_t v0, int32_t nb,
                                                    const uint16_t* Pb, uint16_t* H0,
                                                    uint8_t* mask0) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)nb * kMpH;
       i += (int64_t)gridDim.x * kBlock) {
    const int64_t r = i / kMpH;
    const int j = (int)(i % kMpH);
    const float* x = d.x + 4 * (v0 + r);
    float z = tbf2f(Pb[kMpOffBin + j]);
    for (int k = 0; k < 4; k++) z = __builtin_fmaf(tbf2f(Pb[kMpOffWin + j * 4 + k]), x[k], z);
    H0[i] = tf2bf(z > 0.0f ? z : 0.0f);
    mask0[i] = z > 0.0f;
  }
}

// M[r] = bf16(inv_r * sum over the row of e * H[u]); one wave per vertex
__global__ __launch_bounds__(kBlock) void k_tr_agg(TrainData d, int64_t v0, int32_t nb,
                                                  const uint16_t* H, uint16_t* M) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; r < nb;
       r += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t gv = v0 + r;
    float acc = 0.0f;
    for (int64_t q = d.xadj[gv]; q < d.xadj[gv + 1]; q++)
      acc = __builtin_fmaf(d.e[q], tbf2f(H[(d.adj[q] - v0) * kMpH + lane]), acc);
    M[r * kMpH + lane] = tf2bf(acc * d.inv[gv]);
  }
}

__device__ __forceinline__ bf16x4_t load4(const uint16_t* p) {
  const uint2 u = *(const uint2*)p;
  bf16x4_t r;
  r[0] = (short)(u.x & 0xffff);
  r[1] = (short)(u.x >> 16);
  r[2] = (short)(u.y & 0xffff);
  r[3] = (short)(u.y >> 16);
  return r;
}

// Z = [H | M] [Ws | Wn]^T + b for 32 rows per wave; Hout = bf16(relu(Z))
__global__ __launch_bounds__(kBlock) void k_tr_dense(int32_t nb, const uint16_t* H,
                                                    const uint16_t* M, const uint16_t* Pb, int l,
                                                    uint16_t* Hout, uint8_t* mask) {
  const int lane = threadIdx.x & 63;
  const uint16_t* Ws = Pb + kMpOffL(l);
  const uint16_t* Wn = Ws + kMpH * kMpH;
  const uint16_t* bb = Wn + kMpH * kMpH;
  const int64_t ntiles = (nb + 31) / 32;
  for (int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; t < ntiles;
       t += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t r0 = t * 32;
    const int64_t ra = r0 + (lane & 31);
    f32x16_t acc0 = {0}, acc1 = {0};
    for (int ks = 0; ks < 16; ks++) {
      const uint16_t* src = ks < 8 ? H : M;
      const uint16_t* W = ks < 8 ? Ws : Wn;
      const int kk = (ks & 7) * 8 + 4 * (lane >> 5);
      bf16x4_t a = {0, 0, 0, 0};
      if (ra < nb) a = load4(src + ra * kMpH + kk);
      const bf16x4_t b0 = load4(W + (lane & 31) * kMpH + kk);
      const bf16x4_t b1 = load4(W + (32 + (lane & 31)) * kMpH + kk);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b1, acc1, 0, 0, 0);
    }
    for (int e = 0; e < 16; e++) {
      const int64_t row = r0 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
      if (row >= nb) continue;
      const int c0 = lane & 31, c1 = 32 + (lane & 31);
      const float z0 = acc0[e] + tbf2f(bb[c0]);
      const float z1 = acc1[e] + tbf2f(bb[c1]);
      Hout[row * kMpH + c0] = tf2bf(z0 > 0.0f ? z0 : 0.0f);
      Hout[row * kMpH + c1] = tf2bf(z1 > 0.0f ? z1 : 0.0f);
      mask[row * kMpH + c0] = z0 > 0.0f;
      mask[row * kMpH + c1] = z1 > 0.0f;
    }
  }
}

// scores, loss, dS, output-layer gradients, dH3 = dS wo
__global__ __launch_bounds__(kBlock) void k_tr_score(TrainData d, int64_t v0, int32_t nb,
                                                    float scale, const uint16_t* H3,
                                                    const uint16_t* Pb, float* dH, float* grad,
                                                    float* loss) {
  __shared__ float s_gwo[kMpH];
  __shared__ float s_gbo, s_loss;
  if (threadIdx.x < kMpH) s_gwo[threadIdx.x] = 0.0f;
  if (threadIdx.x == 0) {
    s_gbo = 0.0f;
    s_loss = 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const float wo = tbf2f(Pb[kMpOffWo + lane]);
  const float bo = tbf2f(Pb[kMpOffBo]);
  float gwo = 0.0f, gbo = 0.0f, ls = 0.0f;
  for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; r < nb;
       r += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t gv = v0 + r;
    const float h = tbf2f(H3[r * kMpH + lane]);
    float s = team_sum<64>(wo * h) + bo;
    const float c = d.cw[gv] * scale, y = d.y[gv];
    const float sig = 1.0f / (1.0f + expf(-s));
    const float ds = c * (sig - y);
    if (lane == 0) {
      ls += c * ((s > 0 ? s : 0.0f) + log1pf(expf(-fabsf(s))) - y * s);
      gbo += ds;
    }
    gwo += ds * h;
    dH[r * kMpH + lane] = ds * wo;
  }
  atomicAdd(&s_gwo[lane], gwo);
  if (lane == 0) {
    atomicAdd(&s_gbo, gbo);
    atomicAdd(&s_loss, ls);
  }
  __syncthreads();
  if (threadIdx.x < kMpH) atomicAdd(&grad[kMpOffWo + threadIdx.x], s_gwo[threadIdx.x]);
  if (threadIdx.x == 0) {
    atomicAdd(&grad[kMpOffBo], s_gbo);
    atomicAdd(loss, s_loss);
  }
}

// dZ = bf16(dH * mask), and the bias gradient sum over rows
__global__ __launch_bounds__(kBlock) void k_tr_dz(int32_t nb, const float* dH,
                                                 const uint8_t* mask, uint16_t* dZ, float* gb) {
  __shared__ float s_gb[kMpH];
  if (threadIdx.x < kMpH) s_gb[threadIdx.x] = 0.0f;
  __syncthreads();
  const int j = threadIdx.x & 63;
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)nb * kMpH;
       i += (int64_t)gridDim.x * kBlock) {
    const float g = mask[i] ? dH[i] : 0.0f;
    dZ[i] = tf2bf(g);
    acc += g;
  }
  atomicAdd(&s_gb[j], acc);
  __syncthreads();
  if (threadIdx.x < kMpH) atomicAdd(&gb[threadIdx.x], s_gb[threadIdx.x]);
}

// gradients of Ws and Wn: dZ^T H and dZ^T M, K = the rows of one chunk;
// wave w of the block computes output tile (w / 2, w % 2) of both matrices
__global__ __launch_bounds__(kBlock) void k_tr_wgrad(int32_t nb, const uint16_t* dZ,
                                                    const uint16_t* H, const uint16_t* M,
                                                    float* gWs, float* gWn, int chunk) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int ti = wave >> 1, tj = wave & 1;
  const int i = 32 * ti + (lane & 31), j = 32 * tj + (lane & 31);
  for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < nb; c0 += (int64_t)gridDim.x * chunk) {
    const int64_t c1 = c0 + chunk < nb ? c0 + chunk : nb;
    f32x16_t as = {0}, an = {0};
    for (int64_t n0 = c0; n0 < c1; n0 += 8) {
      bf16x4_t a, bh, bm;
      for (int v = 0; v < 4; v++) {
        const int64_t n = n0 + 4 * (lane >> 5) + v;
        const bool ok = n < c1;
        a[v] = ok ? (short)dZ[n * kMpH + i] : (short)0;
        bh[v] = ok ? (short)H[n * kMpH + j] : (short)0;
        bm[v] = ok ? (short)M[n * kMpH + j] : (short)0;
      }
      as = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bh, as, 0, 0, 0);
      an = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bm, an, 0, 0, 0);
    }
    for (int e = 0; e < 16; e++) {
      const int r = 32 * ti + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
      const int c = 32 * tj + (lane & 31);
      atomicAdd(&gWs[r * kMpH + c], as[e]);
      atomicAdd(&gWn[r * kMpH + c], an[e]);
    }
  }
}

// dHd = dZ Ws, dM = dZ Wn (32 rows per wave)
__global__ __launch_bounds__(kBlock) void k_tr_bwd_data(int32_t nb, const uint16_t* dZ,
                                                       const uint16_t* Pb, int l, float* dHd,
                                                       float* dM) {
  const int lane = threadIdx.x & 63;
  const uint16_t* Ws = Pb + kMpOffL(l);
  const uint16_t* Wn = Ws + kMpH * kMpH;
  const int64_t ntiles = (nb + 31) / 32;
  for (int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; t < ntiles;
       t += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t r0 = t * 32;
    const int64_t ra = r0 + (lane & 31);
    f32x16_t s0 = {0}, s1 = {0}, n0a = {0}, n1a = {0};
    for (int ks = 0; ks < 8; ks++) {
      const int kk = ks * 8 + 4 * (lane >> 5);
      bf16x4_t a = {0, 0, 0, 0};
      if (ra < nb) a = load4(dZ + ra * kMpH + kk);
      bf16x4_t bs0, bs1, bn0, bn1;
      for (int v = 0; v < 4; v++) {
        const int jj = kk + v;  // the contracted index (output unit of the layer)
        bs0[v] = (short)Ws[jj * kMpH + (lane & 31)];
        bs1[v] = (short)Ws[jj * kMpH + 32 + (lane & 31)];
        bn0[v] = (short)Wn[jj * kMpH + (lane & 31)];
        bn1[v] = (short)Wn[jj * kMpH + 32 + (lane & 31)];
      }
      s0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bs0, s0, 0, 0, 0);
      s1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bs1, s1, 0, 0, 0);
      n0a = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bn0, n0a, 0, 0, 0);
      n1a = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bn1, n1a, 0, 0, 0);
    }
    for (int e = 0; e < 16; e++) {
      const int64_t row = r0 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
      if (row >= nb) continue;
      const int c0 = lane & 31, c1 = 32 + (lane & 31);
      dHd[row * kMpH + c0] = s0[e];
      dHd[row * kMpH + c1] = s1[e];
      dM[row * kMpH + c0] = n0a[e];
      dM[row * kMpH + c1] = n1a[e];
    }
  }
}

// dHprev[u] = dHd[u] + sum over the row of u of e_uv inv_v dM[v]
__global__ __launch_bounds__(kBlock) void k_tr_agg_bwd(TrainData d, int64_t v0, int32_t nb,
                                                      const float* dHd, const float* dM,
                                                      float* dHprev) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; r < nb;
       r += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t gu = v0 + r;
    float acc = dHd[r * kMpH + lane];
    for (int64_t q = d.xadj[gu]; q < d.xadj[gu + 1]; q++) {
      const int64_t v = d.adj[q];
      acc += d.e[q] * d.inv[v] * dM[(v - v0) * kMpH + lane];
    }
    dHprev[r * kMpH + lane] = acc;
  }
}

// input layer gradients: gWin = dZ0^T x, gbin = sum dZ0
__global__ __launch_bounds__(kBlock) void k_tr_input_bwd(TrainData d, int64_t v0, int32_t nb,
                                                        const float* dH0, const uint8_t* mask0,
                                                        float* grad) {
  __shared__ float s_g[kMpH * 5];
  for (int i = threadIdx.x; i < kMpH * 5; i += kBlock) s_g[i] = 0.0f;
  __syncthreads();
  const int j = threadIdx.x & 63;
  float gw[4] = {0, 0, 0, 0}, gbv = 0.0f;
  for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64; r < nb;
       r += (int64_t)gridDim.x * kBlock / 64) {
    const int64_t i = r * kMpH + j;
    const float g = mask0[i] ? dH0[i] : 0.0f;
    const float* x = d.x + 4 * (v0 + r);
    for (int k = 0; k < 4; k++) gw[k] += g * x[k];
    gbv += g;
  }
  for (int k = 0; k < 4; k++) atomicAdd(&s_g[j * 4 + k], gw[k]);
  atomicAdd(&s_g[kMpH * 4 + j], gbv);
  __syncthreads();
  for (int i = threadIdx.x; i < kMpH * 4; i += kBlock) atomicAdd(&grad[kMpOffWin + i], s_g[i]);
  if (threadIdx.x < kMpH) atomicAdd(&grad[kMpOffBin + threadIdx.x], s_g[kMpH * 4 + threadIdx.x]);
}

__global__ void k_tr_adam(int32_t np, float* P, float* m, float* v, float* g, uint16_t* Pb,
                          float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    P[i] = p;
    Pb[i] = tf2bf(p);
    g[i] = 0.0f;
  }
}

__global__ void k_tr_tobf16(int32_t np, const float* P, uint16_t* Pb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
    Pb[i] = tf2bf(P[i]);
}

}  // namespace gpk

// ===================================================================== host
using namespace gpk;

namespace {
template <class T>
struct TBuf {
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

struct gp_trainer {
  hipStream_t stream = nullptr;
  TrainData d;
  std::vector<int64_t> hvoff;
  TBuf<int64_t> voff, xadj;
  TBuf<int32_t> adj;
  TBuf<float> e, x, inv, cw, y;
  // parameters
  TBuf<float> P, m, v, g, loss;
  TBuf<uint16_t> Pb;
  int64_t step = 0;
  // activations (sized for the largest mini-batch)
  TBuf<uint16_t> H[4], M[3], dZ;
  TBuf<uint8_t> mask[4];
  TBuf<float> dH, dHd, dM;
  size_t act_rows = 0;
  ~gp_trainer() {
    voff.release(); xadj.release(); adj.release(); e.release(); x.release(); inv.release();
    cw.release(); y.release(); P.release(); m.release(); v.release(); g.release();
    loss.release(); Pb.release(); dZ.release(); dH.release(); dHd.release(); dM.release();
    for (auto& b : H) b.release();
    for (auto& b : M) b.release();
    for (auto& b : mask) b.release();
  }
};

static int tgrid(int64_t items, int per) {
  int64_t g = (items + per - 1) / per;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// forward + backward of graphs [g0, g1); gradients accumulate into t->g
static gp_status tr_forward_backward(gp_trainer* t, int32_t g0, int32_t g1) {
  hipStream_t s = t->stream;
  const int64_t v0 = t->hvoff[g0];
  const int64_t nb64 = t->hvoff[g1] - v0;
  if (nb64 <= 0) return GP_OK;
  if (nb64 > INT32_MAX / kMpH) return GP_EINVAL;
  const int32_t nb = (int32_t)nb64;
  const size_t rows = (size_t)nb * kMpH;
  if (rows > t->act_rows) {
    for (auto& b : t->H) if (!b.ensure(rows)) return GP_ENOMEM;
    for (auto& b : t->M) if (!b.ensure(rows)) return GP_ENOMEM;
    for (auto& b : t->mask) if (!b.ensure(rows)) return GP_ENOMEM;
    if (!t->dZ.ensure(rows) || !t->dH.ensure(rows) || !t->dHd.ensure(rows) || !t->dM.ensure(rows))
      return GP_ENOMEM;
    t->act_rows = rows;
  }
  const float scale = 1.0f / (float)(g1 - g0);
  const int gw = tgrid(nb, kBlock / 64);      // one wave per vertex
  const int gt = tgrid((nb + 31) / 32, kBlock / 64);
  const int ge = tgrid((int64_t)rows, kBlock);
  k_tr_input<<<ge, kBlock, 0, s>>>(t->d, v0, nb, t->Pb.p, t->H[0].p, t->mask[0].p);
  for (int l = 0; l < 3; l++) {
    k_tr_agg<<<gw, kBlock, 0, s>>>(t->d, v0, nb, t->H[l].p, t->M[l].p);
    k_tr_dense<<<gt, kBlock, 0, s>>>(nb, t->H[l].p, t->M[l].p, t->Pb.p, l, t->H[l + 1].p,
                                     t->mask[l + 1].p);
  }
  k_tr_score<<<gw, kBlock, 0, s>>>(t->d, v0, nb, scale, t->H[3].p, t->Pb.p, t->dH.p, t->g.p,
                                   t->loss.p);
  for (int l = 2; l >= 0; l--) {
    float* gWs = t->g.p + kMpOffL(l);
    float* gWn = gWs + kMpH * kMpH;
    float* gb = gWn + kMpH * kMpH;
    k_tr_dz<<<ge, kBlock, 0, s>>>(nb, t->dH.p, t->mask[l + 1].p, t->dZ.p, gb);
    const int chunk = 512;
    k_tr_wgrad<<<tgrid(nb, chunk), kBlock, 0, s>>>(nb, t->dZ.p, t->H[l].p, t->M[l].p, gWs, gWn,
                                                   chunk);
    k_tr_bwd_data<<<gt, kBlock, 0, s>>>(nb, t->dZ.p, t->Pb.p, l, t->dHd.p, t->dM.p);
    k_tr_agg_bwd<<<gw, kBlock, 0, s>>>(t->d, v0, nb, t->dHd.p, t->dM.p, t->dH.p);
  }
  k_tr_input_bwd<<<gw, kBlock, 0, s>>>(t->d, v0, nb, t->dH.p, t->mask[0].p, t->g.p);
  if (hipGetLastError() != hipSuccess) return GP_EDEVICE;
  return GP_OK;
}

extern "C" {

gp_status gp_train_create(gp_trainer** out, const float* init_params, int32_t count,
                          void* stream) {
  if (!out || !init_params || count != kMpNParam) return GP_EINVAL;
  *out = nullptr;
  gp_trainer* t = new (std::nothrow) gp_trainer();
  if (!t) return GP_ENOMEM;
  t->stream = (hipStream_t)stream;
  memset(&t->d, 0, sizeof(t->d));
  if (!t->P.ensure(kMpNParam) || !t->m.ensure(kMpNParam) || !t->v.ensure(kMpNParam) ||
      !t->g.ensure(kMpNParam) || !t->Pb.ensure(kMpNParam) || !t->loss.ensure(1)) {
    delete t;
    return GP_ENOMEM;
  }
  hipStream_t s = t->stream;
  if (hipMemcpyAsync(t->P.p, init_params, sizeof(float) * kMpNParam, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemsetAsync(t->m.p, 0, sizeof(float) * kMpNParam, s) != hipSuccess ||
      hipMemsetAsync(t->v.p, 0, sizeof(float) * kMpNParam, s) != hipSuccess ||
      hipMemsetAsync(t->g.p, 0, sizeof(float) * kMpNParam, s) != hipSuccess) {
    delete t;
    return GP_EDEVICE;
  }
  k_tr_tobf16<<<tgrid(kMpNParam, 256), 256, 0, s>>>(kMpNParam, t->P.p, t->Pb.p);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    delete t;
    return GP_EDEVICE;
  }
  *out = t;
  return GP_OK;
}

void gp_train_destroy(gp_trainer* t) {
  if (!t) return;
  (void)hipStreamSynchronize(t->stream);
  delete t;
}

gp_status gp_train_set_data(gp_trainer* t, int32_t G, const int64_t* voff, const int64_t* eoff,
                            const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                            const int64_t* vwgt, const int8_t* labels, int32_t balance_on) {
  if (!t || G <= 0 || !voff || !eoff || !xadj || !vwgt || !labels ||
      (balance_on != 0 && balance_on != 1))
    return GP_EINVAL;
  hipStream_t s = t->stream;
  t->hvoff.assign((size_t)G + 1, 0);
  std::vector<int64_t> he((size_t)G + 1, 0);
  if (hipMemcpyAsync(t->hvoff.data(), voff, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(he.data(), eoff, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GP_EDEVICE;
  const int64_t N = t->hvoff[G], NNZ = he[G];
  if (N <= 0 || (NNZ > 0 && (!adjncy || !adjwgt))) return GP_EINVAL;
  if (!t->voff.ensure(G + 1) || !t->xadj.ensure(N + 1) || !t->adj.ensure(NNZ) ||
      !t->e.ensure(NNZ) || !t->x.ensure(4 * N) || !t->inv.ensure(N) || !t->cw.ensure(N) ||
      !t->y.ensure(N))
    return GP_ENOMEM;
  if (hipMemcpyAsync(t->voff.p, voff, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return GP_EDEVICE;
  TrainData d;
  d.G = G;
  d.N = N;
  d.NNZ = NNZ;
  d.voff = t->voff.p;
  d.xadj = t->xadj.p;
  d.adj = t->adj.p;
  d.e = t->e.p;
  d.x = t->x.p;
  d.inv = t->inv.p;
  d.cw = t->cw.p;
  d.y = t->y.p;
  t->d = d;
  k_tr_prep<<<tgrid(G, 1), kBlock, 0, s>>>(G, voff, eoff, xadj, adjncy, adjwgt, vwgt, labels,
                                            balance_on, d);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return GP_EDEVICE;
  return GP_OK;
}

// gradient (host float[count]) and loss of graphs [g0, g1), no update
gp_status gp_train_grad(gp_trainer* t, int32_t g0, int32_t g1, float* grad, float* loss) {
  if (!t || !grad || !loss || g0 < 0 || g1 <= g0 || g1 > t->d.G) return GP_EINVAL;
  hipStream_t s = t->stream;
  if (hipMemsetAsync(t->g.p, 0, sizeof(float) * kMpNParam, s) != hipSuccess ||
      hipMemsetAsync(t->loss.p, 0, sizeof(float), s) != hipSuccess)
    return GP_EDEVICE;
  gp_status st = tr_forward_backward(t, g0, g1);
  if (st != GP_OK) return st;
  if (hipMemcpyAsync(grad, t->g.p, sizeof(float) * kMpNParam, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(loss, t->loss.p, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemsetAsync(t->g.p, 0, sizeof(float) * kMpNParam, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GP_EDEVICE;
  return GP_OK;
}

// one Adam step on graphs [g0, g1); *loss (host) receives the batch loss
gp_status gp_train_step(gp_trainer* t, int32_t g0, int32_t g1, float lr, float* loss) {
  if (!t || g0 < 0 || g1 <= g0 || g1 > t->d.G || !(lr > 0.0f)) return GP_EINVAL;
  hipStream_t s = t->stream;
  if (hipMemsetAsync(t->loss.p, 0, sizeof(float), s) != hipSuccess) return GP_EDEVICE;
  gp_status st = tr_forward_backward(t, g0, g1);
  if (st != GP_OK) return st;
  t->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t->step), c2 = 1.0f - powf(b2, (float)t->step);
  k_tr_adam<<<tgrid(kMpNParam, 256), 256, 0, s>>>(kMpNParam, t->P.p, t->m.p, t->v.p, t->g.p,
                                                  t->Pb.p, lr, b1, b2, 1e-8f, c1, c2);
  if (hipGetLastError() != hipSuccess) return GP_EDEVICE;
  if (loss) {
    if (hipMemcpyAsync(loss, t->loss.p, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return GP_EDEVICE;
  }
  return GP_OK;
}

// FP32 master weights and their BF16 copy (host arrays of count values)
gp_status gp_train_params(gp_trainer* t, float* f32, uint16_t* bf16) {
  if (!t) return GP_EINVAL;
  hipStream_t s = t->stream;
  if ((f32 && hipMemcpyAsync(f32, t->P.p, sizeof(float) * kMpNParam, hipMemcpyDeviceToHost, s) !=
                  hipSuccess) ||
      (bf16 && hipMemcpyAsync(bf16, t->Pb.p, sizeof(uint16_t) * kMpNParam,
                              hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return GP_EDEVICE;
  return GP_OK;
}

}  // extern "C"
