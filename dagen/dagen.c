/*
 * dagen.c - seeded synthetic task-DAG generators (input side only).
 *
 * These generators produce the weighted task graphs that the partitioner
 * consumes: vertices are kernels, arrows are data dependencies (Section III-B:
 * node weight = kernel cost per processor, edge weight = transfer cost).  The
 * paper measured its weights offline on its own machine; here every weight
 * comes from a closed form or a seeded distribution so that any run can
 * regenerate the same graph.
 *
 * This module holds none of the partitioning method.  It is shared, as an
 * input source only, by the CPU oracle tests and by the HIP path.
 *
 * Random numbers: one counter-based generator, u64 = F(seed, stream, index),
 * built from the SplitMix64 output finaliser (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014; constants as
 * published by S. Vigna).  Draws never depend on call order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DG_OK 0
#define DG_EINVAL 1
#define DG_ENOMEM 7

/* streams: one per kind of draw */
enum { S_JITTER = 1, S_DEG = 2, S_OFF = 3, S_TGT = 4, S_EBYTES = 5, S_VCOST = 6,
       S_SIZE = 7, S_GRAPH = 8 };

static uint64_t sm_fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t dg_rand(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t key = sm_fin(seed + 0x9e3779b97f4a7c15ULL * (stream + 1));
  return sm_fin(key ^ sm_fin(idx + 0x632be59bd9b4e019ULL));
}

/* uniform double in [0,1) and in (0,1] */
static double u01(uint64_t r) { return (double)(r >> 11) * 0x1p-53; }
static double u01_open0(uint64_t r) { return (double)((r >> 11) + 1) * 0x1p-53; }

/* lognormal(mu, sigma) via Box-Muller on two independent draws */
static double lognormal(double mu, double sigma, uint64_t r1, uint64_t r2) {
  double z = sqrt(-2.0 * log(u01_open0(r1))) * cos(6.283185307179586 * u01(r2));
  return exp(mu + sigma * z);
}

static int64_t round_pos(double x) {
  double r = floor(x + 0.5);
  if (r < 1.0) return 1;
  if (r > 4.0e18) return (int64_t)4000000000000000000LL;
  return (int64_t)r;
}

/* Poisson(lambda) by inversion of the CDF (capped at 63 out-edges) */
static int poisson(double lambda, uint64_t r) {
  double u = u01(r);
  double p = exp(-lambda), F = p;
  int k = 0;
  while (u >= F && k < 63) {
    k++;
    p *= lambda / k;
    F += p;
  }
  return k;
}

/* apply per-mille jitter j in [-J, J] to a flop count */
static int64_t jittered(int64_t flops, int jitter_pm, uint64_t seed, int64_t task) {
  if (jitter_pm <= 0) return flops;
  uint64_t r = dg_rand(seed, S_JITTER, (uint64_t)task);
  int64_t j = (int64_t)(r % (uint64_t)(2 * jitter_pm + 1)) - jitter_pm;
  __int128 f = (__int128)flops * (1000 + j);
  return (int64_t)(f / 1000);
}

static void set_cost(int64_t* vwgt, int64_t v, int64_t cpu, int64_t rate) {
  if (cpu < 1) cpu = 1;
  int64_t gpu = cpu / (rate > 0 ? rate : 1);
  if (gpu < 1) gpu = 1;
  vwgt[2 * v] = cpu;
  vwgt[2 * v + 1] = gpu;
}

/* ---------------------------------------------------------------------- */
/* Tiled right-looking Cholesky, T x T tiles of side b.                    */
/* Kernels: POTRF(k), TRSM(i,k), SYRK(i,k), GEMM(i,j,k) for i > j > k.      */
/* Task ids follow program order: for k { POTRF; TRSM(i>k); for i>k {      */
/* SYRK(i,k); GEMM(i,j,k) j=k+1..i-1 } }.                                   */
/* ---------------------------------------------------------------------- */
void dg_cholesky_size(int T, int64_t* n, int64_t* ne) {
  int64_t t = T;
  *n = t + t * (t - 1) + t * (t - 1) * (t - 2) / 6;
  int64_t c2 = t * (t - 1) / 2, c2m = (t - 1) * (t - 2) / 2;
  int64_t c3 = t * (t - 1) * (t - 2) / 6, c3m = (t - 1) * (t - 2) * (t - 3) / 6;
  *ne = (t > 0 ? t - 1 : 0) + 2 * (c2 + c2m) + 2 * c3 + c3m;
  if (T <= 0) { *n = 0; *ne = 0; }
}

int dg_cholesky(int T, int64_t b, int jitter_pm, int64_t rate, int64_t edge_bytes, uint64_t seed,
                int64_t* vwgt, int32_t* src, int32_t* dst, int64_t* bytes) {
  if (T <= 0) return DG_OK;
  int64_t TT = T;
  int32_t* potrf = (int32_t*)malloc(sizeof(int32_t) * TT);
  int32_t* trsm = (int32_t*)malloc(sizeof(int32_t) * TT * TT);
  int32_t* syrk = (int32_t*)malloc(sizeof(int32_t) * TT * TT);
  int32_t* gemm = (int32_t*)malloc(sizeof(int32_t) * TT * TT * TT);
  if (!potrf || !trsm || !syrk || !gemm) {
    free(potrf); free(trsm); free(syrk); free(gemm);
    return DG_ENOMEM;
  }
  int64_t b3 = b * b * b;
  int64_t id = 0;
  for (int k = 0; k < T; k++) {
    potrf[k] = (int32_t)id;
    set_cost(vwgt, id, jittered(b3 / 3, jitter_pm, seed, id), rate);
    id++;
    for (int i = k + 1; i < T; i++) {
      trsm[(int64_t)i * T + k] = (int32_t)id;
      set_cost(vwgt, id, jittered(b3, jitter_pm, seed, id), rate);
      id++;
    }
    for (int i = k + 1; i < T; i++) {
      syrk[(int64_t)i * T + k] = (int32_t)id;
      set_cost(vwgt, id, jittered(b3, jitter_pm, seed, id), rate);
      id++;
      for (int j = k + 1; j < i; j++) {
        gemm[((int64_t)i * T + j) * T + k] = (int32_t)id;
        set_cost(vwgt, id, jittered(2 * b3, jitter_pm, seed, id), rate);
        id++;
      }
    }
  }
  int64_t e = 0;
#define EDGE(a, c) do { src[e] = (a); dst[e] = (c); bytes[e] = edge_bytes; e++; } while (0)
  for (int k = 0; k < T; k++) {
    if (k >= 1) EDGE(syrk[(int64_t)k * T + (k - 1)], potrf[k]);
    for (int i = k + 1; i < T; i++) {
      int32_t t_ik = trsm[(int64_t)i * T + k];
      EDGE(potrf[k], t_ik);
      if (k >= 1) EDGE(gemm[((int64_t)i * T + k) * T + (k - 1)], t_ik);
    }
    for (int i = k + 1; i < T; i++) {
      int32_t s_ik = syrk[(int64_t)i * T + k];
      EDGE(trsm[(int64_t)i * T + k], s_ik);
      if (k >= 1) EDGE(syrk[(int64_t)i * T + (k - 1)], s_ik);
      for (int j = k + 1; j < i; j++) {
        int32_t g = gemm[((int64_t)i * T + j) * T + k];
        EDGE(trsm[(int64_t)i * T + k], g);
        EDGE(trsm[(int64_t)j * T + k], g);
        if (k >= 1) EDGE(gemm[((int64_t)i * T + j) * T + (k - 1)], g);
      }
    }
  }
#undef EDGE
  free(potrf); free(trsm); free(syrk); free(gemm);
  return DG_OK;
}

/* ---------------------------------------------------------------------- */
/* Tiled right-looking LU without pivoting, T x T tiles.                   */
/* GETRF(k) = 2b^3/3, TRSM-L(k,j) computes U(k,j), TRSM-U(i,k) computes     */
/* L(i,k) (b^3 each), GEMM(i,j,k) = 2b^3 for i,j > k.                       */
/* ---------------------------------------------------------------------- */
void dg_lu_size(int T, int64_t* n, int64_t* ne) {
  int64_t t = T;
  if (T <= 0) { *n = 0; *ne = 0; return; }
  int64_t sq = (t - 1) * t * (2 * t - 1) / 6;       /* sum_{m<T} m^2 */
  int64_t sqm = (t - 2) * (t - 1) * (2 * t - 3) / 6; /* sum_{m<T-1} m^2 */
  if (T < 2) sqm = 0;
  int64_t c2 = t * (t - 1) / 2, c2m = (t - 1) * (t - 2) / 2;
  *n = t + t * (t - 1) + sq;
  *ne = (t - 1) + 2 * (c2 + c2m) + 2 * sq + sqm;
}

int dg_lu(int T, int64_t b, int jitter_pm, int64_t rate, int64_t edge_bytes, uint64_t seed,
          int64_t* vwgt, int32_t* src, int32_t* dst, int64_t* bytes) {
  if (T <= 0) return DG_OK;
  int64_t TT = T;
  int32_t* getrf = (int32_t*)malloc(sizeof(int32_t) * TT);
  int32_t* trl = (int32_t*)malloc(sizeof(int32_t) * TT * TT);
  int32_t* tru = (int32_t*)malloc(sizeof(int32_t) * TT * TT);
  int32_t* gemm = (int32_t*)malloc(sizeof(int32_t) * TT * TT * TT);
  if (!getrf || !trl || !tru || !gemm) {
    free(getrf); free(trl); free(tru); free(gemm);
    return DG_ENOMEM;
  }
  int64_t b3 = b * b * b;
  int64_t id = 0;
  for (int k = 0; k < T; k++) {
    getrf[k] = (int32_t)id;
    set_cost(vwgt, id, jittered(2 * b3 / 3, jitter_pm, seed, id), rate);
    id++;
    for (int j = k + 1; j < T; j++) {
      trl[(int64_t)k * T + j] = (int32_t)id;
      set_cost(vwgt, id, jittered(b3, jitter_pm, seed, id), rate);
      id++;
    }
    for (int i = k + 1; i < T; i++) {
      tru[(int64_t)i * T + k] = (int32_t)id;
      set_cost(vwgt, id, jittered(b3, jitter_pm, seed, id), rate);
      id++;
    }
    for (int i = k + 1; i < T; i++)
      for (int j = k + 1; j < T; j++) {
        gemm[((int64_t)i * T + j) * T + k] = (int32_t)id;
        set_cost(vwgt, id, jittered(2 * b3, jitter_pm, seed, id), rate);
        id++;
      }
  }
  int64_t e = 0;
#define EDGE(a, c) do { src[e] = (a); dst[e] = (c); bytes[e] = edge_bytes; e++; } while (0)
  for (int k = 0; k < T; k++) {
    if (k >= 1) EDGE(gemm[((int64_t)k * T + k) * T + (k - 1)], getrf[k]);
    for (int j = k + 1; j < T; j++) {
      int32_t t = trl[(int64_t)k * T + j];
      EDGE(getrf[k], t);
      if (k >= 1) EDGE(gemm[((int64_t)k * T + j) * T + (k - 1)], t);
    }
    for (int i = k + 1; i < T; i++) {
      int32_t t = tru[(int64_t)i * T + k];
      EDGE(getrf[k], t);
      if (k >= 1) EDGE(gemm[((int64_t)i * T + k) * T + (k - 1)], t);
    }
    for (int i = k + 1; i < T; i++)
      for (int j = k + 1; j < T; j++) {
        int32_t g = gemm[((int64_t)i * T + j) * T + k];
        EDGE(tru[(int64_t)i * T + k], g);
        EDGE(trl[(int64_t)k * T + j], g);
        if (k >= 1) EDGE(gemm[((int64_t)i * T + j) * T + (k - 1)], g);
      }
  }
#undef EDGE
  free(getrf); free(trl); free(tru); free(gemm);
  return DG_OK;
}

/* ---------------------------------------------------------------------- */
/* Random layered DAG: n vertices in L layers (the first n mod L layers     */
/* hold one extra vertex).  A vertex of layer l < L-1 draws Poisson(lambda) */
/* out-edges; each picks a layer offset uniformly in 1..min(3, L-1-l) and  */
/* a target uniformly inside that layer.  Costs and bytes are rounded      */
/* lognormals, clamped to >= 1; gpu = floor(cpu / rate) >= 1.               */
/* ---------------------------------------------------------------------- */
static int64_t layer_size(int64_t n, int L, int l) { return n / L + (l < n % L ? 1 : 0); }
static int64_t layer_start(int64_t n, int L, int l) {
  int64_t q = n / L, r = n % L;
  return (int64_t)l * q + (l < r ? l : r);
}

int64_t dg_layered_edges(int64_t n, int L, double lambda, uint64_t seed) {
  if (n <= 0 || L <= 0) return 0;
  int64_t ne = 0;
  for (int l = 0; l < L - 1; l++) {
    int64_t s = layer_start(n, L, l), sz = layer_size(n, L, l);
    for (int64_t v = s; v < s + sz; v++) ne += poisson(lambda, dg_rand(seed, S_DEG, (uint64_t)v));
  }
  return ne;
}

int dg_layered(int64_t n, int L, double lambda, double mu_v, double sig_v, double mu_e,
               double sig_e, int64_t rate, uint64_t seed, int64_t* vwgt, int32_t* src,
               int32_t* dst, int64_t* bytes) {
  if (n <= 0 || L <= 0) return DG_OK;
  for (int64_t v = 0; v < n; v++) {
    double c = lognormal(mu_v, sig_v, dg_rand(seed, S_VCOST, 2 * (uint64_t)v),
                         dg_rand(seed, S_VCOST, 2 * (uint64_t)v + 1));
    set_cost(vwgt, v, round_pos(c), rate);
  }
  int64_t e = 0;
  for (int l = 0; l < L - 1; l++) {
    int64_t s = layer_start(n, L, l), sz = layer_size(n, L, l);
    int span = L - 1 - l < 3 ? L - 1 - l : 3;
    for (int64_t v = s; v < s + sz; v++) {
      int deg = poisson(lambda, dg_rand(seed, S_DEG, (uint64_t)v));
      for (int k = 0; k < deg; k++) {
        uint64_t q = (uint64_t)v * 64 + (uint64_t)k;
        int off = 1 + (int)(dg_rand(seed, S_OFF, q) % (uint64_t)span);
        int tl = l + off;
        int64_t ts = layer_start(n, L, tl), tsz = layer_size(n, L, tl);
        int64_t t = ts + (int64_t)(dg_rand(seed, S_TGT, q) % (uint64_t)tsz);
        double by = lognormal(mu_e, sig_e, dg_rand(seed, S_EBYTES, 2 * q),
                              dg_rand(seed, S_EBYTES, 2 * q + 1));
        src[e] = (int32_t)v;
        dst[e] = (int32_t)t;
        bytes[e] = round_pos(by);
        e++;
      }
    }
  }
  return DG_OK;
}

/* ---------------------------------------------------------------------- */
/* Directed edge list -> symmetric CSR.  Arrows lose their direction (the   */
/* transfer cost is the same both ways, Section III-B); parallel arrows     */
/* between one pair are merged by summing bytes; rows are sorted by         */
/* neighbour id.  Returns the number of CSR entries written (2 x unique     */
/* undirected edges) or -1 on error.  adj/w must hold 2*ne entries.         */
/* ---------------------------------------------------------------------- */
typedef struct { int32_t v; int64_t w; } dg_pair;

static int cmp_pair(const void* a, const void* b) {
  int32_t x = ((const dg_pair*)a)->v, y = ((const dg_pair*)b)->v;
  return (x > y) - (x < y);
}

int64_t dg_to_csr(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst,
                  const int64_t* bytes, int32_t* xadj, int32_t* adj, int64_t* w) {
  if (n < 0 || ne < 0 || 2 * ne > 2147483647LL) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  dg_pair* buf = (dg_pair*)malloc(sizeof(dg_pair) * (size_t)(2 * ne + 1));
  if (!cnt || !buf) { free(cnt); free(buf); return -1; }
  for (int64_t e = 0; e < ne; e++) {
    if (src[e] == dst[e]) continue;
    cnt[src[e] + 1]++;
    cnt[dst[e] + 1]++;
  }
  for (int64_t v = 0; v < n; v++) cnt[v + 1] += cnt[v];
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!pos) { free(cnt); free(buf); return -1; }
  memcpy(pos, cnt, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t e = 0; e < ne; e++) {
    int32_t a = src[e], c = dst[e];
    if (a == c) continue;
    buf[pos[a]].v = c; buf[pos[a]].w = bytes[e]; pos[a]++;
    buf[pos[c]].v = a; buf[pos[c]].w = bytes[e]; pos[c]++;
  }
  int64_t out = 0;
  xadj[0] = 0;
  for (int64_t v = 0; v < n; v++) {
    int64_t s = cnt[v], t = cnt[v + 1];
    qsort(buf + s, (size_t)(t - s), sizeof(dg_pair), cmp_pair);
    for (int64_t i = s; i < t; i++) {
      if (i > s && buf[i].v == buf[i - 1].v) {
        w[out - 1] += buf[i].w;
      } else {
        adj[out] = buf[i].v;
        w[out] = buf[i].w;
        out++;
      }
    }
    xadj[v + 1] = (int32_t)out;
  }
  free(cnt); free(buf); free(pos);
  return out;
}

/* ---------------------------------------------------------------------- */
/* Batch recipe: graph sizes log-uniform in [lo, hi]; even index ->        */
/* Cholesky with the largest T whose task count fits, odd -> layered.       */
/* ---------------------------------------------------------------------- */
int dg_batch_plan(int G, double lo, double hi, uint64_t seed, int64_t* size, int32_t* kind,
                  int32_t* param, uint64_t* gseed) {
  for (int g = 0; g < G; g++) {
    double u = u01(dg_rand(seed, S_SIZE, (uint64_t)g));
    double s = exp(log(lo) + u * (log(hi) - log(lo)));
    int64_t n = (int64_t)floor(s);
    if (n < (int64_t)lo) n = (int64_t)lo;
    if (n > (int64_t)hi) n = (int64_t)hi;
    gseed[g] = dg_rand(seed, S_GRAPH, (uint64_t)g);
    if (g % 2 == 0) {
      int T = 1;
      for (;;) {
        int64_t nn, ee;
        dg_cholesky_size(T + 1, &nn, &ee);
        if (nn > n) break;
        T++;
      }
      int64_t nn, ee;
      dg_cholesky_size(T, &nn, &ee);
      size[g] = nn;
      kind[g] = 0;
      param[g] = T;
    } else {
      int64_t L = n / 100;
      if (L < 4) L = 4;
      if (L > 64) L = 64;
      size[g] = n;
      kind[g] = 1;
      param[g] = (int32_t)L;
    }
  }
  return DG_OK;
}
