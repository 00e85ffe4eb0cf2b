/*
 * oracle.c - serial CPU oracle of the two-way multilevel partition of a
 * weighted task DAG between a CPU memory node (part 0) and a GPU memory node
 * (part 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the HIP implementation, and the product path never calls it.
 *
 * What the paper fixes (Section III-B, Section IV-C):
 *   - the input is a weighted graph: node weight = cost of a kernel on a
 *     processor, edge weight = cost of the transfer a dependency implies;
 *   - transfers cost the same in both directions, so edges are undirected;
 *   - the target share of each processor follows Eq. (1)-(2):
 *     R_CPU = T_GPU / (T_GPU + T_CPU), R_GPU = 1 - R_CPU;
 *   - the number of parts is 2 and every kernel is pinned to one processor;
 *   - the objective is to keep the load balanced while cutting as little
 *     edge weight as possible.
 * The paper delegates the partition itself to a multilevel library and does
 * not describe its algorithm.  The algorithm below (heavy-edge matching,
 * contraction, greedy growing, prefix-admission refinement) is this
 * project's own deterministic reading; each function states its rule.  The
 * oracle executes those rules one step at a time, in plain loops.
 *
 * All partition arithmetic is integer: int32 vertex ids, int64 weights, cut
 * and loads, 128-bit intermediates for the balance bounds.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = 1, OR_EASYM = 2, OR_EDUP = 3, OR_ESELF = 4, OR_ERANGE = 5,
       OR_EOVERFLOW = 6, OR_ENOMEM = 7, OR_EDEVICE = 8, OR_EMODEL = 9 };

#define OR_MAX_LEVELS 48
#define OR_LIM62 ((int64_t)1 << 62)
#define OR_RATIO_LIM ((int64_t)1 << 40)

#include "oracle_internal.h"

static void og_free(OG* g) {
  free(g->xadj); free(g->adj); free(g->w); free(g->vc); free(g->vg);
  memset(g, 0, sizeof(*g));
}

static int og_alloc(OG* g, int32_t n, int64_t nnz) {
  memset(g, 0, sizeof(*g));
  g->n = n;
  g->xadj = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  g->adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  g->w = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  g->vc = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  g->vg = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  if (!g->xadj || !g->adj || !g->w || !g->vc || !g->vg) { og_free(g); return OR_ENOMEM; }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1)-(2): the CPU share is T_GPU / (T_GPU + T_CPU).  As an integer     */
/* ratio r0:r1 (CPU:GPU) that is T_GPU : T_CPU, reduced by the gcd.          */
/* ------------------------------------------------------------------------ */
int or_ratio_from_times(int64_t t_cpu, int64_t t_gpu, int64_t* ratio) {
  if (t_cpu < 0 || t_gpu < 0 || (t_cpu == 0 && t_gpu == 0)) return OR_EINVAL;
  int64_t a = t_gpu, b = t_cpu;
  while (b != 0) { int64_t t = a % b; a = b; b = t; }
  ratio[0] = t_gpu / a;
  ratio[1] = t_cpu / a;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Target and bound of each part for a total balance weight W and ratio      */
/* r0:r1 (the integer form of Eq. (1)-(2)) with an imbalance tolerance of    */
/* eps_ppm parts per million:                                                */
/*   tgt_p  = floor(W r_p / (r0 + r1))                                       */
/*   maxw_p = ceil (W r_p (1e6 + eps) / ((r0 + r1) 1e6))                     */
/* A partition is feasible when pw_p <= maxw_p for both parts.  The ceiling  */
/* makes maxw_0 + maxw_1 >= W, so at most one part can be over its bound.    */
/* ------------------------------------------------------------------------ */
void or_balance(int64_t W, int64_t r0, int64_t r1, int32_t eps_ppm, int64_t* tgt,
                int64_t* maxw) {
  __int128 R = (__int128)r0 + r1;
  int64_t r[2] = {r0, r1};
  for (int p = 0; p < 2; p++) {
    tgt[p] = (int64_t)(((__int128)W * r[p]) / R);
    __int128 num = (__int128)W * r[p] * (1000000 + eps_ppm);
    __int128 den = R * 1000000;
    maxw[p] = (int64_t)((num + den - 1) / den);
  }
}

/* ------------------------------------------------------------------------ */
/* Input check and canonical form.  The paper feeds its partitioner a        */
/* line-per-vertex adjacency (Section III-B, the DOT-to-METIS translator).   */
/* Here that is a symmetric CSR; the canonical form sorts every row by       */
/* neighbour id.  Checks, each over the whole input, in this order of       */
/* precedence: EINVAL (n < 0, xadj[0] != 0, xadj decreasing), ERANGE         */
/* (neighbour outside [0,n) or a negative weight), ESELF (self loop), EDUP   */
/* (a neighbour listed twice in one row), EASYM (u-v without v-u of the      */
/* same weight), EOVERFLOW (sum of edge weights or of a cost column reaching */
/* 2^62).                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t v; int64_t w; } Pair;

static int pair_cmp(const void* a, const void* b) {
  int32_t x = ((const Pair*)a)->v, y = ((const Pair*)b)->v;
  return (x > y) - (x < y);
}

int or_canonicalize(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                    const int64_t* vwgt, int32_t* oxadj, int32_t* oadj, int64_t* ow) {
  if (n < 0) return OR_EINVAL;
  if (n == 0) { if (oxadj) oxadj[0] = 0; return OR_OK; }
  if (xadj[0] != 0) return OR_EINVAL;
  for (int32_t v = 0; v < n; v++)
    if (xadj[v + 1] < xadj[v]) return OR_EINVAL;
  int64_t nnz = xadj[n];
  for (int64_t e = 0; e < nnz; e++)
    if (adj[e] < 0 || adj[e] >= n || w[e] < 0) return OR_ERANGE;
  for (int64_t i = 0; i < 2 * (int64_t)n; i++)
    if (vwgt[i] < 0) return OR_ERANGE;
  for (int32_t v = 0; v < n; v++)
    for (int32_t e = xadj[v]; e < xadj[v + 1]; e++)
      if (adj[e] == v) return OR_ESELF;
  Pair* row = (Pair*)malloc(sizeof(Pair) * (size_t)(nnz > 0 ? nnz : 1));
  if (!row) return OR_ENOMEM;
  for (int64_t e = 0; e < nnz; e++) { row[e].v = adj[e]; row[e].w = w[e]; }
  for (int32_t v = 0; v < n; v++)
    qsort(row + xadj[v], (size_t)(xadj[v + 1] - xadj[v]), sizeof(Pair), pair_cmp);
  int rc = OR_OK;
  for (int32_t v = 0; v < n && rc == OR_OK; v++)
    for (int32_t e = xadj[v] + 1; e < xadj[v + 1]; e++)
      if (row[e].v == row[e - 1].v) { rc = OR_EDUP; break; }
  /* symmetry: binary search of v in the sorted row of each neighbour */
  for (int32_t v = 0; v < n && rc == OR_OK; v++) {
    for (int32_t e = xadj[v]; e < xadj[v + 1]; e++) {
      int32_t u = row[e].v;
      int32_t lo = xadj[u], hi = xadj[u + 1] - 1, found = -1;
      while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (row[mid].v == v) { found = mid; break; }
        if (row[mid].v < v) lo = mid + 1; else hi = mid - 1;
      }
      if (found < 0 || row[found].w != row[e].w) { rc = OR_EASYM; break; }
    }
  }
  if (rc == OR_OK) {
    __int128 s = 0, sc = 0, sg = 0;
    for (int64_t e = 0; e < nnz; e++) s += row[e].w;
    for (int32_t v = 0; v < n; v++) { sc += vwgt[2 * v]; sg += vwgt[2 * v + 1]; }
    if (s >= OR_LIM62 || sc >= OR_LIM62 || sg >= OR_LIM62) rc = OR_EOVERFLOW;
  }
  if (rc == OR_OK && oxadj) {
    for (int32_t v = 0; v <= n; v++) oxadj[v] = xadj[v];
    for (int64_t e = 0; e < nnz; e++) { oadj[e] = row[e].v; ow[e] = row[e].w; }
  }
  free(row);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Heavy-edge matching by mutual proposals.                                  */
/* Edge order (a strict total order on undirected edges {lo < hi}):          */
/*   heavier edge first; then larger hash h; then smaller lo; then smaller   */
/*   hi, where h = mix(hs ^ (lo << 32 | hi)), hs = mix(seed ^ level) and mix */
/*   is the SplitMix64 output finaliser.  The hash breaks ties among equal   */
/*   weights without favouring low ids; lo/hi settle the (improbable) hash   */
/*   collisions, so the order depends on ids only.                           */
/* Round: each unmatched u proposes to its best eligible neighbour under     */
/* that order; an edge {u,v} is eligible when both ends are unmatched at the */
/* start of the round and b(u) + b(v) <= cap.  u and v match when each      */
/* proposed to the other.  R rounds; vertices still free stay single.       */
/* Returns the number of matched pairs.                                      */
/* ------------------------------------------------------------------------ */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* the finaliser alone (exported so tests can check it against the published */
/* SplitMix64 outputs)                                                        */
uint64_t or_mix64(uint64_t z) { return mix64(z); }

uint64_t or_edge_hash(uint64_t seed, int32_t level, int32_t a, int32_t b) {
  int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  uint64_t hs = mix64(seed ^ (uint64_t)(uint32_t)level);
  return mix64(hs ^ (((uint64_t)(uint32_t)lo << 32) | (uint64_t)(uint32_t)hi));
}

/* 1 when edge (w1, h1, lo1, hi1) comes before edge (w2, h2, lo2, hi2) */
static int edge_before(int64_t w1, uint64_t h1, int32_t lo1, int32_t hi1, int64_t w2,
                       uint64_t h2, int32_t lo2, int32_t hi2) {
  if (w1 != w2) return w1 > w2;
  if (h1 != h2) return h1 > h2;
  if (lo1 != lo2) return lo1 < lo2;
  return hi1 < hi2;
}

int64_t or_match_rounds(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                        const int64_t* b, int64_t cap, uint64_t seed, int32_t level, int32_t R,
                        int32_t* match) {
  int32_t* prop = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!prop) return -1;
  for (int32_t u = 0; u < n; u++) match[u] = -1;
  int64_t pairs = 0;
  for (int32_t r = 0; r < R; r++) {
    for (int32_t u = 0; u < n; u++) {
      prop[u] = -1;
      if (match[u] != -1) continue;
      int32_t best = -1;
      int64_t bw = 0;
      uint64_t bh = 0;
      int32_t blo = 0, bhi = 0;
      for (int32_t e = xadj[u]; e < xadj[u + 1]; e++) {
        int32_t v = adj[e];
        if (match[v] != -1) continue;
        if (b[u] + b[v] > cap) continue;
        int32_t lo = u < v ? u : v, hi = u < v ? v : u;
        uint64_t h = or_edge_hash(seed, level, lo, hi);
        if (best < 0 || edge_before(w[e], h, lo, hi, bw, bh, blo, bhi)) {
          best = v; bw = w[e]; bh = h; blo = lo; bhi = hi;
        }
      }
      prop[u] = best;
    }
    int64_t made = 0;
    for (int32_t u = 0; u < n; u++) {
      int32_t v = prop[u];
      if (v >= 0 && prop[v] == u) { match[u] = v; made++; }
    }
    pairs += made / 2;
    if (made == 0) break; /* a round that matches nothing leaves the state, and every later round, unchanged */
  }
  free(prop);
  return pairs;
}

/* ------------------------------------------------------------------------ */
/* Two-hop pass, after the rounds.  An unmatched vertex u with neighbours    */
/* has a hub: its first neighbour under the edge order, whether or not that */
/* neighbour is matched.  Unmatched vertices with the same hub h, taken in   */
/* ascending id, are paired first-second, third-fourth, ... ; the unmatched  */
/* vertices without neighbours form one more group, also in ascending id.   */
/* A pair is formed only when b(x) + b(y) <= cap; otherwise both stay       */
/* single.  Pairs share a neighbour (or have none), so every group is a set */
/* of leaves around one vertex, the structure that stalls plain matching.   */
/* Returns the number of pairs formed.                                      */
/* ------------------------------------------------------------------------ */
int64_t or_match_twohop(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                        const int64_t* b, int64_t cap, uint64_t seed, int32_t level,
                        int32_t* match) {
  int32_t* hub = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* grp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!hub || !grp) { free(hub); free(grp); return -1; }
  for (int32_t u = 0; u < n; u++) {
    hub[u] = -1;
    if (match[u] != -1) continue;
    int64_t bw = 0;
    uint64_t bh = 0;
    int32_t blo = 0, bhi = 0;
    for (int32_t e = xadj[u]; e < xadj[u + 1]; e++) {
      int32_t v = adj[e];
      int32_t lo = u < v ? u : v, hi = u < v ? v : u;
      uint64_t h = or_edge_hash(seed, level, lo, hi);
      if (hub[u] < 0 || edge_before(w[e], h, lo, hi, bw, bh, blo, bhi)) {
        hub[u] = v; bw = w[e]; bh = h; blo = lo; bhi = hi;
      }
    }
  }
  int64_t pairs = 0;
  /* groups around each hub h: the unmatched vertices of row h whose hub is h */
  for (int32_t h = 0; h < n; h++) {
    int32_t k = 0;
    for (int32_t e = xadj[h]; e < xadj[h + 1]; e++) {
      int32_t x = adj[e];
      if (match[x] == -1 && hub[x] == h) grp[k++] = x;
    }
    for (int32_t i = 0; i + 1 < k; i += 2) {
      int32_t x = grp[i], y = grp[i + 1];
      if (b[x] + b[y] <= cap) { match[x] = y; match[y] = x; pairs++; }
    }
  }
  /* vertices without neighbours */
  int32_t k = 0;
  for (int32_t u = 0; u < n; u++)
    if (match[u] == -1 && xadj[u + 1] == xadj[u]) grp[k++] = u;
  for (int32_t i = 0; i + 1 < k; i += 2) {
    int32_t x = grp[i], y = grp[i + 1];
    if (b[x] + b[y] <= cap) { match[x] = y; match[y] = x; pairs++; }
  }
  free(hub);
  free(grp);
  return pairs;
}

/* R proposal rounds, then the two-hop pass (when twohop != 0) */
int64_t or_match(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                 const int64_t* b, int64_t cap, uint64_t seed, int32_t level, int32_t R,
                 int32_t twohop, int32_t* match) {
  int64_t p1 = or_match_rounds(n, xadj, adj, w, b, cap, seed, level, R, match);
  if (p1 < 0 || !twohop) return p1;
  int64_t p2 = or_match_twohop(n, xadj, adj, w, b, cap, seed, level, match);
  return p2 < 0 ? -1 : p1 + p2;
}

/* ------------------------------------------------------------------------ */
/* Contraction.  A vertex leads its pair when it is single or the smaller    */
/* id of its pair.  Coarse ids follow the leaders in ascending order.  Both  */
/* cost columns of a coarse vertex are the sums over its members.  A coarse  */
/* row holds every member edge to a vertex of another coarse vertex, mapped  */
/* to coarse ids, with parallel entries summed, the internal edge dropped,   */
/* and neighbours in ascending order.                                        */
/* ------------------------------------------------------------------------ */
static int or_contract_og(const OG* g, const int32_t* match, int32_t* cmap, OG* cg) {
  int32_t n = g->n, nc = 0;
  for (int32_t u = 0; u < n; u++)
    if (match[u] < 0 || u < match[u]) cmap[u] = nc++;
  for (int32_t u = 0; u < n; u++)
    if (!(match[u] < 0 || u < match[u])) cmap[u] = cmap[match[u]];
  int64_t nnz = g->xadj[n];
  if (og_alloc(cg, nc, nnz) != OR_OK) return OR_ENOMEM;
  int32_t* lead = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  Pair* tmp = (Pair*)malloc(sizeof(Pair) * (size_t)(nnz > 0 ? nnz : 1));
  if (!lead || !tmp) { free(lead); free(tmp); og_free(cg); return OR_ENOMEM; }
  for (int32_t u = 0; u < n; u++)
    if (match[u] < 0 || u < match[u]) lead[cmap[u]] = u;
  int64_t out = 0;
  cg->xadj[0] = 0;
  for (int32_t c = 0; c < nc; c++) {
    int32_t mem[2] = {lead[c], match[lead[c]]};
    int64_t k = 0;
    cg->vc[c] = 0;
    cg->vg[c] = 0;
    for (int i = 0; i < 2; i++) {
      int32_t u = mem[i];
      if (u < 0) continue;
      cg->vc[c] += g->vc[u];
      cg->vg[c] += g->vg[u];
      for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
        int32_t cx = cmap[g->adj[e]];
        if (cx == c) continue;
        tmp[k].v = cx;
        tmp[k].w = g->w[e];
        k++;
      }
    }
    qsort(tmp, (size_t)k, sizeof(Pair), pair_cmp);
    for (int64_t i = 0; i < k; i++) {
      if (i > 0 && tmp[i].v == tmp[i - 1].v) {
        cg->w[out - 1] += tmp[i].w;
      } else {
        cg->adj[out] = tmp[i].v;
        cg->w[out] = tmp[i].w;
        out++;
      }
    }
    cg->xadj[c + 1] = (int32_t)out;
  }
  free(lead);
  free(tmp);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Gains.  For v in part s: ext(v) = sum of w to the other part, int(v) =    */
/* sum of w to part s, gain(v) = ext(v) - int(v): the drop of the cut if v   */
/* alone changes side.  cut = sum over undirected edges with ends in         */
/* different parts of w = (sum of ext) / 2.                                  */
/* ------------------------------------------------------------------------ */
static void compute_gain(const OG* g, const int8_t* part, int64_t* gain, int64_t* cut) {
  int64_t ext_sum = 0;
  for (int32_t v = 0; v < g->n; v++) {
    int64_t ext = 0, in = 0;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
      if (part[g->adj[e]] != part[v]) ext += g->w[e]; else in += g->w[e];
    }
    gain[v] = ext - in;
    ext_sum += ext;
  }
  if (cut) *cut = ext_sum / 2;
}

int64_t or_cut(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
               const int8_t* part) {
  int64_t s = 0;
  for (int32_t v = 0; v < n; v++)
    for (int32_t e = xadj[v]; e < xadj[v + 1]; e++)
      if (part[adj[e]] != part[v]) s += w[e];
  return s / 2;
}

/* b: weight the candidate adds to the destination side; bs: weight it takes
   from its own side (the same column unless the two sides are measured in
   different columns) */
typedef struct { int32_t v; int64_t gain; int64_t b; int64_t bs; } Cand;

/* candidates in admission order: larger gain first, then smaller id */
static int cand_cmp(const void* a, const void* b) {
  const Cand* x = (const Cand*)a;
  const Cand* y = (const Cand*)b;
  if (x->gain != y->gain) return x->gain > y->gain ? -1 : 1;
  return (x->v > y->v) - (x->v < y->v);
}

/* ------------------------------------------------------------------------ */
/* Synchronous refinement, at most P passes; pass i first recomputes every   */
/* gain from the current assignment.                                         */
/*  - Rebalance pass, taken when a part s is over its bound: order all of s  */
/*    by (gain desc, id asc); take the shortest prefix whose weight covers   */
/*    the excess pw_s - maxw_s, then shorten it to the longest prefix that   */
/*    the other part d can still absorb (pw_d + weight <= maxw_d).           */
/*  - Improvement pass otherwise, from side s = i mod 2 to d: candidates are */
/*    the vertices of s with gain > 0 in the same order; the longest prefix  */
/*    with pw_d + weight <= maxw_d moves (no skipping inside the prefix).    */
/*  Every admitted vertex moves at once.  Because one pass moves in one      */
/*  direction, the cut falls by at least the sum of the admitted gains, so   */
/*  improvement passes never raise the cut.  The loop stops after two        */
/*  consecutive improvement passes that move nothing, or after P passes.     */
/* Returns the passes run; *moves_out gets the number of vertices moved.     */
/* ------------------------------------------------------------------------ */
/* b[p]: the weight column that measures side p (the same array for both
   sides, except in time balance, where side 0 counts CPU cost and side 1 GPU
   cost); a vertex moving from s to d takes b[s][v] from s and adds b[d][v]
   to d. */
static int refine_og2(const OG* g, const int64_t* const b[2], int8_t* part, int64_t* pw,
                      const int64_t* maxw, int P, int64_t* moves_out) {
  int32_t n = g->n;
  int64_t* gain = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  Cand* list = (Cand*)malloc(sizeof(Cand) * (size_t)(n > 0 ? n : 1));
  if (!gain || !list) { free(gain); free(list); return -1; }
  int passes = 0, z = 0;
  int64_t moves = 0;
  for (int i = 0; i < P; i++) {
    compute_gain(g, part, gain, NULL);
    passes++;
    int over = pw[0] > maxw[0] ? 0 : (pw[1] > maxw[1] ? 1 : -1);
    if (over >= 0) {
      int s = over, d = 1 - s;
      int32_t k = 0;
      for (int32_t v = 0; v < n; v++)
        if (part[v] == s) {
          list[k].v = v; list[k].gain = gain[v]; list[k].b = b[d][v]; list[k].bs = b[s][v];
          k++;
        }
      qsort(list, (size_t)k, sizeof(Cand), cand_cmp);
      int64_t excess = pw[s] - maxw[s], budget = maxw[d] - pw[d];
      /* the shortest prefix that takes the excess off s, cut back to the
         longest prefix that d can absorb */
      int32_t k1 = 0;
      int64_t acc = 0;
      while (k1 < k && acc < excess) { acc += list[k1].bs; k1++; }
      int32_t k2 = 0;
      acc = 0;
      while (k2 < k && acc + list[k2].b <= budget) { acc += list[k2].b; k2++; }
      int32_t take = k1 < k2 ? k1 : k2;
      for (int32_t j = 0; j < take; j++) {
        part[list[j].v] = (int8_t)d;
        pw[s] -= list[j].bs;
        pw[d] += list[j].b;
      }
      moves += take;
      z = 0;
    } else {
      int s = i & 1, d = 1 - s;
      int32_t k = 0;
      for (int32_t v = 0; v < n; v++)
        if (part[v] == s && gain[v] > 0) {
          list[k].v = v; list[k].gain = gain[v]; list[k].b = b[d][v]; list[k].bs = b[s][v];
          k++;
        }
      qsort(list, (size_t)k, sizeof(Cand), cand_cmp);
      int64_t budget = maxw[d] - pw[d];
      int32_t take = 0;
      int64_t acc = 0;
      while (take < k && acc + list[take].b <= budget) { acc += list[take].b; take++; }
      for (int32_t j = 0; j < take; j++) {
        part[list[j].v] = (int8_t)d;
        pw[s] -= list[j].bs;
        pw[d] += list[j].b;
      }
      moves += take;
      z = take == 0 ? z + 1 : 0;
      if (z == 2) break;
    }
  }
  free(gain);
  free(list);
  if (moves_out) *moves_out = moves;
  return passes;
}

static int refine_og(const OG* g, const int64_t* b, int8_t* part, int64_t* pw,
                     const int64_t* maxw, int P, int64_t* moves_out) {
  const int64_t* const bb[2] = {b, b};
  return refine_og2(g, bb, part, pw, maxw, P, moves_out);
}

/* ------------------------------------------------------------------------ */
/* Communication volume (a reading of "count a tile once per memory node"):  */
/* the graph's ids are a topological order, so the successors of u are its  */
/* neighbours with larger ids; u's output is as large as its largest edge to */
/* a successor, out(u), and crosses to the other part once when any          */
/* successor lies there.  vol = sum over u of out(u) [a successor of u is on  */
/* the other side].                                                          */
/* ------------------------------------------------------------------------ */
static OG og_view(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                  const int64_t* vc, const int64_t* vg);

static void vol_out(const OG* g, int64_t* out) {
  for (int32_t u = 0; u < g->n; u++) {
    out[u] = 0;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (g->adj[e] > u && g->w[e] > out[u]) out[u] = g->w[e];
  }
}

/* successors of u on the other side of u */
static void vol_ext_succ(const OG* g, const int8_t* part, int32_t* cnt) {
  for (int32_t u = 0; u < g->n; u++) {
    cnt[u] = 0;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (g->adj[e] > u && part[g->adj[e]] != part[u]) cnt[u]++;
  }
}

int64_t or_volume(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                  const int8_t* part) {
  OG g = og_view(n, xadj, adj, w, NULL, NULL);
  int64_t* out = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!out || !cnt) { free(out); free(cnt); return -1; }
  vol_out(&g, out);
  vol_ext_succ(&g, part, cnt);
  int64_t vol = 0;
  for (int32_t u = 0; u < n; u++)
    if (cnt[u] > 0) vol += out[u];
  free(out);
  free(cnt);
  return vol;
}

/* The volume gain of moving v from its side s to d, at the pass's start:
   v's own output stops crossing when no successor is left on d and starts
   crossing when one is on s; a predecessor u on d whose only successor on
   the other side was v stops crossing; a predecessor u on s with no
   successor on the other side starts crossing. */
static int64_t vol_gain(const OG* g, const int8_t* part, const int64_t* out, const int32_t* cnt,
                        int32_t v) {
  const int s = part[v], d = 1 - s;
  int32_t succ_s = 0, succ_d = 0;
  int64_t gain = 0;
  for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
    const int32_t x = g->adj[e];
    if (x > v) {
      if (part[x] == s) succ_s++;
      else succ_d++;
    } else if (x < v) {
      if (part[x] == d && cnt[x] == 1) gain += out[x];
      if (part[x] == s && cnt[x] == 0) gain -= out[x];
    }
  }
  gain += out[v] * ((succ_d > 0) - (succ_s > 0));
  return gain;
}

/* At most P passes of the refinement rules with the volume gain in place of
   the edge-cut gain (same pass plan, candidate order and admission). */
static int refine_vol(const OG* g, const int64_t* b, int8_t* part, int64_t* pw,
                      const int64_t* maxw, int P) {
  int32_t n = g->n;
  int64_t* out = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  Cand* list = (Cand*)malloc(sizeof(Cand) * (size_t)(n > 0 ? n : 1));
  if (!out || !cnt || !list) { free(out); free(cnt); free(list); return -1; }
  vol_out(g, out);
  int z = 0;
  for (int i = 0; i < P; i++) {
    vol_ext_succ(g, part, cnt);
    int over = pw[0] > maxw[0] ? 0 : (pw[1] > maxw[1] ? 1 : -1);
    int s = over >= 0 ? over : (i & 1), d = 1 - s;
    int32_t k = 0;
    for (int32_t v = 0; v < n; v++) {
      if (part[v] != s) continue;
      const int64_t gn = vol_gain(g, part, out, cnt, v);
      if (over >= 0 || gn > 0) {
        list[k].v = v; list[k].gain = gn; list[k].b = b[v]; list[k].bs = b[v];
        k++;
      }
    }
    qsort(list, (size_t)k, sizeof(Cand), cand_cmp);
    int64_t budget = maxw[d] - pw[d];
    int32_t take = 0;
    int64_t acc = 0;
    if (over >= 0) {
      int64_t excess = pw[s] - maxw[s];
      int32_t k1 = 0;
      while (k1 < k && acc < excess) { acc += list[k1].b; k1++; }
      int32_t k2 = 0;
      acc = 0;
      while (k2 < k && acc + list[k2].b <= budget) { acc += list[k2].b; k2++; }
      take = k1 < k2 ? k1 : k2;
    } else {
      while (take < k && acc + list[take].b <= budget) { acc += list[take].b; take++; }
    }
    for (int32_t j = 0; j < take; j++) {
      part[list[j].v] = (int8_t)d;
      pw[s] -= list[j].b;
      pw[d] += list[j].b;
    }
    if (over >= 0) z = 0;
    else {
      z = take == 0 ? z + 1 : 0;
      if (z == 2) break;
    }
  }
  free(out);
  free(cnt);
  free(list);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial bisection at the coarsest level by greedy graph growing.          */
/* The grown side g is the part with the smaller ratio (part 0 on a tie);    */
/* the other side is gb.  K = min(trials, n) trials; trial t starts with all */
/* vertices in gb and seed s_t = floor(t n / K), and adds one vertex at a    */
/* time while pw_g < tgt_g:                                                  */
/*   - the first addition is s_t if it fits (pw_g + b <= maxw_g);           */
/*   - otherwise, and for every later addition, among the vertices of gb     */
/*     that fit, those with a neighbour in g come first; among them the     */
/*     largest gain_g(v) = w(v, g) - w(v, gb) wins, then the smaller id;     */
/*   - growing stops when nothing fits.                                      */
/* Each trial is then refined (refine_og) and the kept trial is the first    */
/* one minimal in (infeasible, cut).                                         */
/* ------------------------------------------------------------------------ */
static int init_bisect_og(const OG* g, const int64_t* b, int64_t r0, int64_t r1,
                          const int64_t* tgt, const int64_t* maxw, int K, int P, int8_t* best,
                          int64_t* best_pw) {
  int32_t n = g->n;
  int gs = r0 <= r1 ? 0 : 1, gb = 1 - gs;
  int64_t W = 0;
  for (int32_t v = 0; v < n; v++) W += b[v];
  best_pw[gs] = 0;
  best_pw[gb] = W;
  for (int32_t v = 0; v < n; v++) best[v] = (int8_t)gb;
  if (n == 0) return OR_OK;
  if (K > n) K = n;
  int8_t* part = (int8_t*)malloc((size_t)n);
  int64_t* conn = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* tot = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int32_t* adjc = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!part || !conn || !tot || !adjc) {
    free(part); free(conn); free(tot); free(adjc);
    return OR_ENOMEM;
  }
  for (int32_t v = 0; v < n; v++) {
    tot[v] = 0;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) tot[v] += g->w[e];
  }
  int best_inf = 0;
  int64_t best_cut = 0;
  for (int t = 0; t < K; t++) {
    int64_t pw[2];
    pw[gs] = 0;
    pw[gb] = W;
    for (int32_t v = 0; v < n; v++) { part[v] = (int8_t)gb; conn[v] = 0; adjc[v] = 0; }
    int32_t seedv = (int32_t)(((int64_t)t * n) / K);
    int first = 1;
    while (pw[gs] < tgt[gs]) {
      int32_t pick = -1;
      if (first && pw[gs] + b[seedv] <= maxw[gs]) {
        pick = seedv;
      } else {
        int pa = 0;
        int64_t pg = 0;
        for (int32_t v = 0; v < n; v++) {
          if (part[v] != gb || pw[gs] + b[v] > maxw[gs]) continue;
          int a = adjc[v] > 0;
          int64_t gv = 2 * conn[v] - tot[v];
          if (pick < 0 || a > pa || (a == pa && gv > pg)) { pick = v; pa = a; pg = gv; }
        }
      }
      first = 0;
      if (pick < 0) break;
      part[pick] = (int8_t)gs;
      pw[gs] += b[pick];
      pw[gb] -= b[pick];
      for (int32_t e = g->xadj[pick]; e < g->xadj[pick + 1]; e++) {
        conn[g->adj[e]] += g->w[e];
        adjc[g->adj[e]] += 1;
      }
    }
    if (refine_og(g, b, part, pw, maxw, P, NULL) < 0) {
      free(part); free(conn); free(tot); free(adjc);
      return OR_ENOMEM;
    }
    int64_t cut = or_cut(n, g->xadj, g->adj, g->w, part);
    int inf = pw[0] > maxw[0] || pw[1] > maxw[1];
    if (t == 0 || inf < best_inf || (inf == best_inf && cut < best_cut)) {
      best_inf = inf;
      best_cut = cut;
      memcpy(best, part, (size_t)n);
      best_pw[0] = pw[0];
      best_pw[1] = pw[1];
    }
  }
  free(part); free(conn); free(tot); free(adjc);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exported single steps (for tests).                                        */
/* ------------------------------------------------------------------------ */
static OG og_view(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                  const int64_t* vc, const int64_t* vg) {
  OG g;
  g.n = n;
  g.xadj = (int32_t*)xadj;
  g.adj = (int32_t*)adj;
  g.w = (int64_t*)w;
  g.vc = (int64_t*)vc;
  g.vg = (int64_t*)vg;
  return g;
}

/* Contract; returns the coarse vertex count, or -1.  Output arrays must hold */
/* n (cmap, vc, vg), n+1 (xadj) and nnz (adj, w) entries; *cnnz gets the      */
/* coarse entry count.                                                        */
int32_t or_contract(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                    const int64_t* vc, const int64_t* vg, const int32_t* match, int32_t* cmap,
                    int32_t* cxadj, int32_t* cadj, int64_t* cw, int64_t* cvc, int64_t* cvg,
                    int64_t* cnnz) {
  OG g = og_view(n, xadj, adj, w, vc, vg), cg;
  if (or_contract_og(&g, match, cmap, &cg) != OR_OK) return -1;
  int64_t m = cg.xadj[cg.n];
  memcpy(cxadj, cg.xadj, sizeof(int32_t) * ((size_t)cg.n + 1));
  memcpy(cadj, cg.adj, sizeof(int32_t) * (size_t)m);
  memcpy(cw, cg.w, sizeof(int64_t) * (size_t)m);
  memcpy(cvc, cg.vc, sizeof(int64_t) * (size_t)cg.n);
  memcpy(cvg, cg.vg, sizeof(int64_t) * (size_t)cg.n);
  *cnnz = m;
  int32_t nc = cg.n;
  og_free(&cg);
  return nc;
}

/* Refine an assignment in place; pw holds the part weights on entry and on */
/* exit.  Returns passes run, or -1.                                         */
int or_refine(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
              const int64_t* b, int8_t* part, int64_t* pw, const int64_t* maxw, int P,
              int64_t* moves) {
  OG g = og_view(n, xadj, adj, w, b, b);
  return refine_og(&g, b, part, pw, maxw, P, moves);
}

int or_init_bisect(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                   const int64_t* b, int64_t r0, int64_t r1, const int64_t* tgt,
                   const int64_t* maxw, int K, int P, int8_t* part, int64_t* pw) {
  OG g = og_view(n, xadj, adj, w, b, b);
  return init_bisect_og(&g, b, r0, r1, tgt, maxw, K, P, part, pw);
}

/* ------------------------------------------------------------------------ */
/* Learned proposal hook: defined in mpnn.c.                                 */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Whole multilevel partition.                                               */
/* opts: [0] r0 (CPU share)  [1] r1 (GPU share)  [2] eps_ppm                 */
/*       [3] balance_on (0: cpu cost column, 1: gpu cost column)             */
/*       [4] seed  [5] coarsen_to C  [6] match rounds R  [7] refine passes P */
/*       [8] init trials K  [9] flags (bit 1: learned proposal)              */
/* res:  [0] cut  [1..2] part weights (balance column)  [3] CPU time of part */
/*       0 (cpu costs)  [4] GPU time of part 1 (gpu costs)  [5] feasible     */
/*       [6] levels  [7] learned result kept (judged on the input graph)    */
/*       [8] communication volume (with the volume objective, else 0)        */
/* trace (optional, 8 int64 per level, level 0 first): n, nnz, passes,       */
/*       moves, cut after refinement, pw0, pw1, pairs matched on this level  */
/* Coarsening runs while n > C, and stops after a level that removed less   */
/* than 5 % of the vertices (20 n' > 19 n) or after 48 levels; a stalled     */
/* level is kept.  The matching weight cap is ceil(3W / (2C)).              */
/* ------------------------------------------------------------------------ */
/* Uncoarsening from the coarsest level L to level 0: project the bisection
   to the finer level through cmap, then refine it there.  *partp holds the
   coarsest level's bisection on entry (pw its part weights) and the level-0
   bisection on return.  Writes the coarsest level's and every finer level's
   trace row. */
static int uncoarsen(OG* lv, int32_t* const* cmap, int L, int bal, int time_mode,
                     const int64_t* pairs, const int64_t* maxw, int P, int8_t** partp,
                     int64_t* pw, int64_t* trace, int32_t trace_cap) {
  int8_t* part = *partp;
  if (trace && L < trace_cap) {
    OG* g = &lv[L];
    int64_t* t = trace + 8 * L;
    t[0] = g->n; t[1] = g->xadj[g->n]; t[2] = 0; t[3] = 0;
    t[4] = or_cut(g->n, g->xadj, g->adj, g->w, part);
    t[5] = pw[0]; t[6] = pw[1]; t[7] = pairs[L];
  }
  for (int l = L - 1; l >= 0; l--) {
    OG* g = &lv[l];
    const int64_t* b = bal ? g->vg : g->vc;
    int8_t* next = (int8_t*)malloc((size_t)(g->n > 0 ? g->n : 1));
    if (!next) { *partp = part; return OR_ENOMEM; }
    for (int32_t u = 0; u < g->n; u++) next[u] = part[cmap[l][u]];
    free(part);
    part = next;
    int64_t moves = 0;
    const int64_t* const bt[2] = {g->vc, g->vg};
    int passes = time_mode ? refine_og2(g, bt, part, pw, maxw, P, &moves)
                           : refine_og(g, b, part, pw, maxw, P, &moves);
    if (passes < 0) { *partp = part; return OR_ENOMEM; }
    if (trace && l < trace_cap) {
      int64_t* t = trace + 8 * l;
      t[0] = g->n; t[1] = g->xadj[g->n]; t[2] = passes; t[3] = moves;
      t[4] = or_cut(g->n, g->xadj, g->adj, g->w, part);
      t[5] = pw[0]; t[6] = pw[1]; t[7] = pairs[l];
    }
  }
  *partp = part;
  return OR_OK;
}

#define OR_FLAG_LEARNED 2
/* Time balance (a reading of the paper's remark that the method assumes one
   CPU/GPU performance ratio for all kernels, Section IV-D): part 0 is
   measured by its CPU cost and part 1 by its GPU cost, each against its own
   bound tgt_p = floor(W_p r_p / R), maxw_p = ceil(W_p r_p (10^6 + eps) /
   (R 10^6)) with W_0 the CPU-cost total and W_1 the GPU-cost total (with
   r = (W_1, W_0), Eq. (1) on the totals, both bounds are the same time).
   The coarsening and the initial bisection use the balance column as
   usual; from the coarsest level on, the refinement works with the two
   columns, its rebalance passes bringing each side under its own bound. */
#define OR_FLAG_TIME 8
/* Communication-volume objective: after the edge-cut refinement of the input
   graph, at most P more passes with the volume gain (vol_gain); the result
   then also reports the volume. */
#define OR_FLAG_VOLUME 16

int or_partition(int32_t n, const int32_t* xadj, const int32_t* adj, const int64_t* w,
                 const int64_t* vwgt, const int64_t* opts, const void* model, int8_t* part_out,
                 int64_t* res, int64_t* trace, int32_t trace_cap) {
  int64_t r0 = opts[0], r1 = opts[1];
  int64_t eps = opts[2], bal = opts[3];
  uint64_t seed = (uint64_t)opts[4];
  int64_t C = opts[5], R = opts[6], P = opts[7], K = opts[8], flags = opts[9];
  if (r0 < 0 || r1 < 0 || r0 >= OR_RATIO_LIM || r1 >= OR_RATIO_LIM || r0 + r1 == 0)
    return OR_EINVAL;
  if (eps < 0 || eps > 1000000 || (bal != 0 && bal != 1)) return OR_EINVAL;
  if (C < 1 || R < 0 || R > 64 || P < 0 || P > 64 || K < 1 || K > 64) return OR_EINVAL;
  if ((flags & OR_FLAG_LEARNED) && !model) return OR_EMODEL;
  if ((flags & OR_FLAG_LEARNED) && (flags & OR_FLAG_TIME)) return OR_EINVAL;
  if ((flags & OR_FLAG_VOLUME) && (flags & (OR_FLAG_LEARNED | OR_FLAG_TIME))) return OR_EINVAL;
  const int time_mode = (flags & OR_FLAG_TIME) != 0;
  if (n < 0) return OR_EINVAL;

  OG lv[OR_MAX_LEVELS + 1];
  int32_t* cmap[OR_MAX_LEVELS];
  int64_t pairs[OR_MAX_LEVELS + 1];
  memset(lv, 0, sizeof(lv));
  memset(cmap, 0, sizeof(cmap));
  memset(pairs, 0, sizeof(pairs));
  int64_t nnz0 = n > 0 ? xadj[n] : 0;
  if (n > 0 && xadj[0] == 0 && nnz0 < 0) return OR_EINVAL;
  if (og_alloc(&lv[0], n, nnz0 > 0 ? nnz0 : 0) != OR_OK) return OR_ENOMEM;
  int rc = or_canonicalize(n, xadj, adj, w, vwgt, lv[0].xadj, lv[0].adj, lv[0].w);
  if (rc != OR_OK) { og_free(&lv[0]); return rc; }
  for (int32_t v = 0; v < n; v++) { lv[0].vc[v] = vwgt[2 * v]; lv[0].vg[v] = vwgt[2 * v + 1]; }

  int64_t W = 0;
  for (int32_t v = 0; v < n; v++) W += bal ? lv[0].vg[v] : lv[0].vc[v];
  int64_t tgt[2], maxw[2];
  or_balance(W, r0, r1, (int32_t)eps, tgt, maxw);
  int64_t cap = (int64_t)((((__int128)3 * W) + 2 * (__int128)C - 1) / (2 * (__int128)C));

  int L = 0;
  rc = OR_OK;
  while (lv[L].n > C) {
    OG* g = &lv[L];
    const int64_t* b = bal ? g->vg : g->vc;
    int32_t* match = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n);
    cmap[L] = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n);
    if (!match || !cmap[L]) { free(match); rc = OR_ENOMEM; break; }
    pairs[L] = or_match(g->n, g->xadj, g->adj, g->w, b, cap, seed, L, (int32_t)R, 1, match);
    if (pairs[L] < 0 || or_contract_og(g, match, cmap[L], &lv[L + 1]) != OR_OK) {
      free(match); rc = OR_ENOMEM; break;
    }
    free(match);
    L++;
    if (20 * (int64_t)lv[L].n > 19 * (int64_t)lv[L - 1].n || L == OR_MAX_LEVELS) break;
  }
  int8_t* part = NULL;
  int8_t* lp = NULL;
  int64_t pw[2] = {0, 0};
  int64_t lpw[2] = {0, 0};
  int used_learned = 0;
  int64_t* ltrace = NULL;
  if (rc == OR_OK) {
    OG* g = &lv[L];
    const int64_t* b = bal ? g->vg : g->vc;
    part = (int8_t*)malloc((size_t)(g->n > 0 ? g->n : 1));
    if (!part) rc = OR_ENOMEM;
    if (rc == OR_OK) rc = init_bisect_og(g, b, r0, r1, tgt, maxw, (int)K, (int)P, part, pw);
    /* the learned proposal runs on coarsest graphs of at most 3,072 vertices;
       its refined bisection is carried through the uncoarsening beside the
       plain one (below) */
    if (rc == OR_OK && (flags & OR_FLAG_LEARNED) && g->n > 0 && g->n <= 3072) {
      int gs = r0 <= r1 ? 0 : 1;
      lp = (int8_t*)malloc((size_t)g->n);
      if (!lp) rc = OR_ENOMEM;
      if (rc == OR_OK) rc = or_learned_proposal(g, b, model, gs, tgt, maxw, lp, lpw);
      if (rc == OR_OK && refine_og(g, b, lp, lpw, maxw, (int)P, NULL) < 0) rc = OR_ENOMEM;
      if (rc == OR_OK && trace && trace_cap > 0) {
        ltrace = (int64_t*)calloc((size_t)trace_cap * 8, sizeof(int64_t));
        if (!ltrace) rc = OR_ENOMEM;
      }
    }
  }
  if (rc == OR_OK && time_mode) {
    /* each side in its own column from here on */
    int64_t Wt[2] = {0, 0}, tt[2], mt[2];
    for (int32_t v = 0; v < n; v++) { Wt[0] += lv[0].vc[v]; Wt[1] += lv[0].vg[v]; }
    or_balance(Wt[0], r0, r1, (int32_t)eps, tt, mt);
    maxw[0] = mt[0];
    tgt[0] = tt[0];
    or_balance(Wt[1], r0, r1, (int32_t)eps, tt, mt);
    maxw[1] = mt[1];
    tgt[1] = tt[1];
    OG* g = &lv[L];
    pw[0] = pw[1] = 0;
    for (int32_t v = 0; v < g->n; v++) {
      if (part[v] == 0) pw[0] += g->vc[v];
      else pw[1] += g->vg[v];
    }
    /* the coarsest bisection is refined once more under the two bounds */
    const int64_t* const bt[2] = {g->vc, g->vg};
    if (refine_og2(g, bt, part, pw, maxw, (int)P, NULL) < 0) rc = OR_ENOMEM;
  }
  if (rc == OR_OK) rc = uncoarsen(lv, cmap, L, (int)bal, time_mode, pairs, maxw, (int)P, &part,
                                  pw, trace, trace_cap);
  if (rc == OR_OK && lp) {
    rc = uncoarsen(lv, cmap, L, (int)bal, 0, pairs, maxw, (int)P, &lp, lpw, ltrace, trace_cap);
    if (rc == OR_OK) {
      /* the plain bisection judges the learned one on the input graph: the
         learned result is kept only when it is strictly better in
         (infeasible, cut) after projection and refinement */
      OG* g = &lv[0];
      int inf_p = pw[0] > maxw[0] || pw[1] > maxw[1];
      int inf_l = lpw[0] > maxw[0] || lpw[1] > maxw[1];
      int64_t cut_p = or_cut(g->n, g->xadj, g->adj, g->w, part);
      int64_t cut_l = or_cut(g->n, g->xadj, g->adj, g->w, lp);
      if (inf_l < inf_p || (inf_l == inf_p && cut_l < cut_p)) {
        int8_t* t = part;
        part = lp;
        lp = t;
        pw[0] = lpw[0];
        pw[1] = lpw[1];
        used_learned = 1;
        if (ltrace) memcpy(trace, ltrace, sizeof(int64_t) * 8 * (size_t)trace_cap);
      }
    }
  }
  free(lp);
  free(ltrace);
  int64_t volume = 0;
  if (rc == OR_OK && (flags & OR_FLAG_VOLUME) && n > 0) {
    OG* g = &lv[0];
    if (refine_vol(g, bal ? g->vg : g->vc, part, pw, maxw, (int)P) < 0) rc = OR_ENOMEM;
    if (rc == OR_OK) volume = or_volume(n, g->xadj, g->adj, g->w, part);
    if (volume < 0) rc = OR_ENOMEM;
  }
  if (rc == OR_OK) {
    OG* g = &lv[0];
    int64_t tc = 0, tg = 0;
    for (int32_t v = 0; v < n; v++) {
      part_out[v] = part[v];
      if (part[v] == 0) tc += g->vc[v]; else tg += g->vg[v];
    }
    res[0] = n > 0 ? or_cut(n, g->xadj, g->adj, g->w, part) : 0;
    res[1] = pw[0];
    res[2] = pw[1];
    res[3] = tc;
    res[4] = tg;
    res[5] = pw[0] <= maxw[0] && pw[1] <= maxw[1];
    res[6] = L;
    res[7] = used_learned;
    res[8] = volume;
  }
  free(part);
  for (int l = 0; l <= L; l++) og_free(&lv[l]);
  for (int l = 0; l < OR_MAX_LEVELS; l++) free(cmap[l]);
  return rc;
}
