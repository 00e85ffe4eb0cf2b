/*
 * mpnn.c - oracle side of the learned coarsest-level proposal.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Shares no code with the HIP
 * implementation.
 *
 * The paper leaves the partitioner's initial bisection to its black-box
 * library (Section III-B).  This project adds a learned proposal for the
 * coarsest graph: a 3-layer message-passing network (hidden size 64, BF16
 * weights) scores every coarsest vertex; the highest scores fill the grown
 * side; the usual refinement follows; the plain greedy-growing result stays
 * the fallback and the yardstick.  The partition arithmetic stays integer: the
 * network only orders vertices.
 *
 * Inference is specified exactly, so that a CPU emulation reproduces the
 * GPU's float results bit for bit: only correctly rounded FP32 fused
 * multiply-adds and multiplications, in a fixed order, and round-to-nearest-
 * even conversion to BF16.
 *
 *   phi(x)  (x >= 0 integer) = (bitlen(x) - 1) + (the 8 bits after the
 *           leading one) / 256, and phi(0) = 0 - exact in FP32.
 *   input   x_v = [phi(cpu), phi(gpu), phi(deg), phi(sum of incident w)]
 *   edge    e_uv = phi(w_uv) / 64;  inv_v = 1 / deg_v (FP32), 0 if deg_v = 0
 *   h0_v[j] = bf16(relu(fma-chain over k = 0..3 of Win[j][k] x_v[k], from b_in[j]))
 *   layer l = 1..3:
 *     m_v[k]  = bf16( (fma-chain over the row of v, in row order, of e_vu h_u[k],
 *                     from 0) * inv_v )
 *     h'_v[j] = bf16(relu(fma-chain of Ws[j][k] h_v[k] for k ascending, then of
 *                    Wn[j][k] m_v[k] for k ascending, from b[j]))
 *   score_v = fma-chain of wo[k] h3_v[k], k ascending, from bo
 *   relu(a) = a > 0 ? a : +0.
 *
 * Parameter blob: 25,153 BF16 values (uint16 bits) in this order:
 *   Win[64][4], b_in[64], then for l = 1..3: Ws[64][64], Wn[64][64], b[64],
 *   then wo[64], bo.  Matrices are row-major [output][input].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define MP_H 64
#define MP_F 4
#define MP_OFF_WIN 0
#define MP_OFF_BIN (MP_OFF_WIN + MP_H * MP_F)
#define MP_LAYER (2 * MP_H * MP_H + MP_H)
#define MP_OFF_L(l) (MP_OFF_BIN + MP_H + (l) * MP_LAYER)
#define MP_OFF_WO MP_OFF_L(3)
#define MP_OFF_BO (MP_OFF_WO + MP_H)
#define MP_NPARAM (MP_OFF_BO + 1)

int32_t or_mpnn_nparam(void) { return MP_NPARAM; }

static float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* round to nearest, ties to even */
static uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static float relu_f(float a) { return a > 0.0f ? a : 0.0f; }

/* phi(x) = (bitlen(x) - 1) + next 8 bits / 256 */
float or_phi(int64_t x) {
  if (x <= 0) return 0.0f;
  int L = 64 - __builtin_clzll((uint64_t)x);
  uint64_t f;
  if (L - 1 >= 8) f = ((uint64_t)x >> (L - 1 - 8)) & 0xffu;
  else f = ((uint64_t)x << (8 - (L - 1))) & 0xffu;
  return (float)(L - 1) + (float)f * (1.0f / 256.0f);
}

/* FP32 inputs of the network: x (n x 4), e (per CSR entry), inv (per vertex) */
static void mp_inputs(const OG* g, float* x, float* e, float* inv) {
  for (int32_t v = 0; v < g->n; v++) {
    int64_t deg = g->xadj[v + 1] - g->xadj[v], tw = 0;
    for (int32_t k = g->xadj[v]; k < g->xadj[v + 1]; k++) {
      tw += g->w[k];
      e[k] = or_phi(g->w[k]) / 64.0f;
    }
    x[4 * v + 0] = or_phi(g->vc[v]);
    x[4 * v + 1] = or_phi(g->vg[v]);
    x[4 * v + 2] = or_phi(deg);
    x[4 * v + 3] = or_phi(tw);
    inv[v] = deg > 0 ? 1.0f / (float)deg : 0.0f;
  }
}

/* exact emulation of the inference; scores: float[n] */
int or_mpnn_scores(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                   const int64_t* vc, const int64_t* vg, const uint16_t* P, float* scores) {
  OG g;
  g.n = n;
  g.xadj = (int32_t*)xadj;
  g.adj = (int32_t*)adj;
  g.w = (int64_t*)w;
  g.vc = (int64_t*)vc;
  g.vg = (int64_t*)vg;
  int64_t nnz = n > 0 ? xadj[n] : 0;
  float* x = (float*)malloc(sizeof(float) * 4 * (size_t)(n > 0 ? n : 1));
  float* e = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
  float* inv = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  uint16_t* h = (uint16_t*)malloc(sizeof(uint16_t) * MP_H * (size_t)(n > 0 ? n : 1));
  uint16_t* hn = (uint16_t*)malloc(sizeof(uint16_t) * MP_H * (size_t)(n > 0 ? n : 1));
  if (!x || !e || !inv || !h || !hn) {
    free(x); free(e); free(inv); free(h); free(hn);
    return 7;
  }
  mp_inputs(&g, x, e, inv);
  for (int32_t v = 0; v < n; v++)
    for (int j = 0; j < MP_H; j++) {
      float acc = bf16_to_f32(P[MP_OFF_BIN + j]);
      for (int k = 0; k < MP_F; k++) acc = fmaf(bf16_to_f32(P[MP_OFF_WIN + j * MP_F + k]), x[4 * v + k], acc);
      h[v * MP_H + j] = f32_to_bf16(relu_f(acc));
    }
  for (int l = 0; l < 3; l++) {
    const uint16_t* Ws = P + MP_OFF_L(l);
    const uint16_t* Wn = Ws + MP_H * MP_H;
    const uint16_t* bb = Wn + MP_H * MP_H;
    for (int32_t v = 0; v < n; v++) {
      float m[MP_H], hv[MP_H];
      for (int k = 0; k < MP_H; k++) {
        float acc = 0.0f;
        for (int32_t q = xadj[v]; q < xadj[v + 1]; q++)
          acc = fmaf(e[q], bf16_to_f32(h[adj[q] * MP_H + k]), acc);
        m[k] = bf16_to_f32(f32_to_bf16(acc * inv[v]));
        hv[k] = bf16_to_f32(h[v * MP_H + k]);
      }
      for (int j = 0; j < MP_H; j++) {
        float acc = bf16_to_f32(bb[j]);
        for (int k = 0; k < MP_H; k++) acc = fmaf(bf16_to_f32(Ws[j * MP_H + k]), hv[k], acc);
        for (int k = 0; k < MP_H; k++) acc = fmaf(bf16_to_f32(Wn[j * MP_H + k]), m[k], acc);
        hn[v * MP_H + j] = f32_to_bf16(relu_f(acc));
      }
    }
    uint16_t* t = h;
    h = hn;
    hn = t;
  }
  for (int32_t v = 0; v < n; v++) {
    float acc = bf16_to_f32(P[MP_OFF_BO]);
    for (int k = 0; k < MP_H; k++)
      acc = fmaf(bf16_to_f32(P[MP_OFF_WO + k]), bf16_to_f32(h[v * MP_H + k]), acc);
    scores[v] = acc;
  }
  free(x); free(e); free(inv); free(h); free(hn);
  return 0;
}

/* order-preserving int32 image of a float */
static int32_t f32_key(float f) {
  int32_t b;
  memcpy(&b, &f, 4);
  return b < 0 ? (int32_t)(b ^ 0x7fffffff) : b;
}

typedef struct { int32_t key; int32_t v; } ScoreKey;

static int score_cmp(const void* a, const void* b) {
  const ScoreKey* x = (const ScoreKey*)a;
  const ScoreKey* y = (const ScoreKey*)b;
  if (x->key != y->key) return x->key > y->key ? -1 : 1;
  return (x->v > y->v) - (x->v < y->v);
}

/* Proposal: vertices in order of (score desc, id asc); each vertex joins the
 * grown side gs when it fits (pw_gs + b <= maxw_gs); filling stops as soon as
 * pw_gs >= tgt_gs.  The rest stays on the other side. */
int or_learned_proposal(const OG* g, const int64_t* b, const void* model, int gs,
                        const int64_t* tgt, const int64_t* maxw, int8_t* part, int64_t* pw) {
  int32_t n = g->n;
  float* sc = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  ScoreKey* ord = (ScoreKey*)malloc(sizeof(ScoreKey) * (size_t)(n > 0 ? n : 1));
  if (!sc || !ord) { free(sc); free(ord); return 7; }
  int rc = or_mpnn_scores(n, g->xadj, g->adj, g->w, g->vc, g->vg, (const uint16_t*)model, sc);
  if (rc) { free(sc); free(ord); return rc; }
  for (int32_t v = 0; v < n; v++) { ord[v].key = f32_key(sc[v]); ord[v].v = v; }
  qsort(ord, (size_t)n, sizeof(ScoreKey), score_cmp);
  int gb = 1 - gs;
  int64_t W = 0;
  for (int32_t v = 0; v < n; v++) { part[v] = (int8_t)gb; W += b[v]; }
  int64_t pg = 0;
  for (int32_t i = 0; i < n; i++) {
    if (pg >= tgt[gs]) break;
    int32_t v = ord[i].v;
    if (pg + b[v] <= maxw[gs]) { part[v] = (int8_t)gs; pg += b[v]; }
  }
  pw[gs] = pg;
  pw[gb] = W - pg;
  free(sc);
  free(ord);
  return 0;
}

/* The proposal alone on plain arrays (exported for tests): b is the balance
 * column; the caller passes the grown side gs and the bounds. */
int or_learned_fill(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                    const int64_t* vc, const int64_t* vg, const int64_t* b, const void* model,
                    int32_t gs, const int64_t* tgt, const int64_t* maxw, int8_t* part,
                    int64_t* pw) {
  OG g;
  g.n = n;
  g.xadj = (int32_t*)xadj;
  g.adj = (int32_t*)adj;
  g.w = (int64_t*)w;
  g.vc = (int64_t*)vc;
  g.vg = (int64_t*)vg;
  return or_learned_proposal(&g, b, model, gs, tgt, maxw, part, pw);
}

/* ------------------------------------------------------------------------ */
/* FP64 reference of the training objective and its gradient.              */
/* The same network without rounding (all FP64, weights as given).  Loss:   */
/* BCE with logits, each vertex weighted by b_v / sum(b) (1/n if the sum is */
/* 0), label y_v = 1 when the vertex is on the grown side in the plain      */
/* pipeline's refined coarsest partition.                                    */
/* Returns the loss; grad receives d loss / d parameter (MP_NPARAM).        */
/* ------------------------------------------------------------------------ */
static double softplus(double s) { return (s > 0 ? s : 0) + log1p(exp(-fabs(s))); }

double or_mpnn_loss_grad_f64(int32_t n, const int32_t* xadj, const int32_t* adj,
                             const int64_t* w, const int64_t* vc, const int64_t* vg,
                             const int64_t* bw, const int8_t* y, const double* P, double* grad) {
  OG g;
  g.n = n;
  g.xadj = (int32_t*)xadj;
  g.adj = (int32_t*)adj;
  g.w = (int64_t*)w;
  g.vc = (int64_t*)vc;
  g.vg = (int64_t*)vg;
  int64_t nnz = n > 0 ? xadj[n] : 0;
  size_t NH = (size_t)(n > 0 ? n : 1) * MP_H;
  float* xf = (float*)malloc(sizeof(float) * 4 * (size_t)(n > 0 ? n : 1));
  float* ef = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
  float* invf = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  double* Hs[4];
  double* Ms[3];
  double* Zs[4];
  for (int i = 0; i < 4; i++) { Hs[i] = (double*)calloc(NH, sizeof(double)); Zs[i] = (double*)calloc(NH, sizeof(double)); }
  for (int i = 0; i < 3; i++) Ms[i] = (double*)calloc(NH, sizeof(double));
  double* s = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* dh = (double*)calloc(NH, sizeof(double));
  double* dhp = (double*)calloc(NH, sizeof(double));
  double* dm = (double*)calloc(NH, sizeof(double));
  mp_inputs(&g, xf, ef, invf);
  memset(grad, 0, sizeof(double) * MP_NPARAM);
  /* forward */
  for (int32_t v = 0; v < n; v++)
    for (int j = 0; j < MP_H; j++) {
      double z = P[MP_OFF_BIN + j];
      for (int k = 0; k < MP_F; k++) z += P[MP_OFF_WIN + j * MP_F + k] * (double)xf[4 * v + k];
      Zs[0][v * MP_H + j] = z;
      Hs[0][v * MP_H + j] = z > 0 ? z : 0;
    }
  for (int l = 0; l < 3; l++) {
    const double* Ws = P + MP_OFF_L(l);
    const double* Wn = Ws + MP_H * MP_H;
    const double* bb = Wn + MP_H * MP_H;
    for (int32_t v = 0; v < n; v++) {
      for (int k = 0; k < MP_H; k++) {
        double a = 0;
        for (int32_t q = xadj[v]; q < xadj[v + 1]; q++) a += (double)ef[q] * Hs[l][adj[q] * MP_H + k];
        Ms[l][v * MP_H + k] = a * (double)invf[v];
      }
      for (int j = 0; j < MP_H; j++) {
        double z = bb[j];
        for (int k = 0; k < MP_H; k++) z += Ws[j * MP_H + k] * Hs[l][v * MP_H + k];
        for (int k = 0; k < MP_H; k++) z += Wn[j * MP_H + k] * Ms[l][v * MP_H + k];
        Zs[l + 1][v * MP_H + j] = z;
        Hs[l + 1][v * MP_H + j] = z > 0 ? z : 0;
      }
    }
  }
  double Wt = 0;
  for (int32_t v = 0; v < n; v++) Wt += (double)bw[v];
  double loss = 0;
  for (int32_t v = 0; v < n; v++) {
    double a = P[MP_OFF_BO];
    for (int k = 0; k < MP_H; k++) a += P[MP_OFF_WO + k] * Hs[3][v * MP_H + k];
    s[v] = a;
    double cw = Wt > 0 ? (double)bw[v] / Wt : 1.0 / n;
    loss += cw * (softplus(a) - (double)y[v] * a);
    double ds = cw * (1.0 / (1.0 + exp(-a)) - (double)y[v]);
    grad[MP_OFF_BO] += ds;
    for (int k = 0; k < MP_H; k++) {
      grad[MP_OFF_WO + k] += ds * Hs[3][v * MP_H + k];
      dh[v * MP_H + k] = ds * P[MP_OFF_WO + k];
    }
  }
  /* backward through the three layers */
  for (int l = 2; l >= 0; l--) {
    const double* Ws = P + MP_OFF_L(l);
    const double* Wn = Ws + MP_H * MP_H;
    double* gWs = grad + MP_OFF_L(l);
    double* gWn = gWs + MP_H * MP_H;
    double* gb = gWn + MP_H * MP_H;
    memset(dhp, 0, sizeof(double) * NH);
    memset(dm, 0, sizeof(double) * NH);
    for (int32_t v = 0; v < n; v++)
      for (int j = 0; j < MP_H; j++) {
        double dz = Zs[l + 1][v * MP_H + j] > 0 ? dh[v * MP_H + j] : 0;
        if (dz == 0) continue;
        gb[j] += dz;
        for (int k = 0; k < MP_H; k++) {
          gWs[j * MP_H + k] += dz * Hs[l][v * MP_H + k];
          gWn[j * MP_H + k] += dz * Ms[l][v * MP_H + k];
          dhp[v * MP_H + k] += Ws[j * MP_H + k] * dz;
          dm[v * MP_H + k] += Wn[j * MP_H + k] * dz;
        }
      }
    /* m_v = inv_v sum_u e_vu h_u  ->  dh_u += sum_v e_vu inv_v dm_v */
    for (int32_t v = 0; v < n; v++)
      for (int32_t q = xadj[v]; q < xadj[v + 1]; q++) {
        int32_t u = adj[q];
        double c = (double)ef[q] * (double)invf[v];
        for (int k = 0; k < MP_H; k++) dhp[u * MP_H + k] += c * dm[v * MP_H + k];
      }
    memcpy(dh, dhp, sizeof(double) * NH);
  }
  for (int32_t v = 0; v < n; v++)
    for (int j = 0; j < MP_H; j++) {
      double dz = Zs[0][v * MP_H + j] > 0 ? dh[v * MP_H + j] : 0;
      grad[MP_OFF_BIN + j] += dz;
      for (int k = 0; k < MP_F; k++) grad[MP_OFF_WIN + j * MP_F + k] += dz * (double)xf[4 * v + k];
    }
  free(xf); free(ef); free(invf); free(s); free(dh); free(dhp); free(dm);
  for (int i = 0; i < 4; i++) { free(Hs[i]); free(Zs[i]); }
  for (int i = 0; i < 3; i++) free(Ms[i]);
  return loss;
}

/* exported for tests: float -> bf16 bits (round to nearest even) */
uint16_t or_bf16_round(float f) { return f32_to_bf16(f); }
