/*
 * gp.h - C ABI of the MI355X (gfx950) two-way task-DAG partitioner.
 *
 * Splits the kernels of a weighted data-flow task graph between a CPU memory
 * node (part 0) and a GPU memory node (part 1), the graph-partition
 * scheduling policy of Wu, Lohmann and Schroeder-Preikschat (Section III-B):
 *   - vertex weight = cost of a kernel on a processor (two costs per vertex:
 *     CPU and GPU), edge weight = cost (bytes) of the transfer a dependency
 *     implies; a transfer costs the same in both directions, so the graph is
 *     undirected;
 *   - the target share of each processor follows Eq. (1)-(2),
 *     R_CPU = T_GPU / (T_GPU + T_CPU), R_GPU = 1 - R_CPU, given here as an
 *     integer ratio r0:r1 with an imbalance tolerance eps;
 *   - k = 2 parts; every kernel is pinned to exactly one processor;
 *   - the objective keeps the load balanced while cutting as little edge
 *     weight as possible (Section IV-C).
 * The partition itself is a deterministic multilevel method (heavy-edge
 * matching, contraction, greedy-growing initial bisection, prefix-admission
 * boundary refinement).  All of its arithmetic is integer, so the result is
 * one exact assignment per (graph, options); it does not depend on the GPU's
 * scheduling of threads.
 *
 * Graph layout (CSR, the adjacency form the paper hands its partitioner):
 *   xadj   int32[n+1]  row offsets, xadj[0] = 0, non-decreasing, 2m = xadj[n] < 2^31
 *   adjncy int32[2m]   neighbour ids in [0, n); every edge appears in both rows
 *   adjwgt int64[2m]   edge weights >= 0, equal in both directions
 *   vwgt   int64[n][2] per vertex (cpu cost, gpu cost) >= 0
 * Sums of adjwgt and of each vwgt column must stay below 2^62.
 *
 * Threads: a gp_graph handle is used by one host thread at a time.
 * Errors: no call throws; on error nothing is written to the outputs.
 */
#ifndef GP_H
#define GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_graph gp_graph;

typedef enum {
  GP_OK = 0,
  GP_EINVAL = 1,     /* bad argument, bad option or malformed xadj */
  GP_EASYM = 2,      /* an edge u-v without v-u of equal weight */
  GP_EDUP = 3,       /* a neighbour listed twice in one row */
  GP_ESELF = 4,      /* a self loop */
  GP_ERANGE = 5,     /* a neighbour id outside [0, n) or a negative weight */
  GP_EOVERFLOW = 6,  /* sum of edge weights or of a cost column >= 2^62 */
  GP_ENOMEM = 7,     /* device or host allocation failed */
  GP_EDEVICE = 8,    /* a HIP runtime call failed */
  GP_EMODEL = 9      /* GP_LEARNED without a usable model */
} gp_status;

/* flags for gp_create (GP_HOST_PTRS) and gp_options.flags (the others) */
enum {
  GP_HOST_PTRS = 1,  /* input / output pointers are host memory (else device memory) */
  GP_LEARNED = 2,    /* run the learned coarsest-level proposal beside the plain one */
  GP_TRACE = 4,      /* record per-level statistics (costs one extra pass per level) */
  GP_TIME_BALANCE = 8, /* balance each side in its own cost column (below) */
  GP_VOLUME = 16       /* communication-volume passes on the input graph (below) */
};
/* GP_VOLUME: the objective counts each task's output once per memory node
 * that needs it (Section IV-C's transfer counts; a tile cached on a node is
 * not sent again) instead of once per cut edge.  The ids must be a
 * topological order (every dependency points from the smaller id to the
 * larger); task u's output is as large as its largest edge to a successor,
 * out(u), and the volume is the sum of out(u) over the tasks with a successor
 * on the other side.  After the edge-cut refinement of the input graph, up to
 * refine_passes more passes use the volume gain of a move in place of its
 * edge-cut gain (same pass plan, order and admission).  res->volume reports
 * the volume.  Not with GP_LEARNED or GP_TIME_BALANCE, the batched calls or
 * gp_partition_kway (GP_EINVAL).  gp_level_read's and the trace's level 0
 * show the bisection before these passes. */
/* GP_TIME_BALANCE lifts the assumption that every kernel has the same
 * CPU/GPU performance ratio (Section IV-D): side 0 is measured by its CPU
 * cost and side 1 by its GPU cost, each against its own bound tgt_p =
 * floor(W_p r_p / R), maxw_p = ceil(W_p r_p (10^6 + eps) / (R 10^6)) with W_0
 * the CPU-cost total and W_1 the GPU-cost total (ratio = {W_1, W_0}, Eq. (1)
 * on the totals, makes both bounds the same time).  Coarsening and the
 * initial bisection use the balance column as usual; the coarsest bisection
 * is then refined under the two bounds, and so is every level on the way
 * up.  res->load holds the two times; feasible refers to these bounds.
 * Not with GP_LEARNED, the batched calls or gp_partition_kway (GP_EINVAL). */

typedef struct {
  int64_t ratio[2];      /* CPU : GPU target shares, Eq. (1)-(2); each in [0, 2^40), sum > 0 */
  int32_t eps_ppm;       /* imbalance tolerance in parts per million, [0, 10^6]; 30000 = 3 % */
  int32_t balance_on;    /* 0: balance the CPU-cost column (default), 1: the GPU-cost column */
  uint64_t seed;         /* seed of the matching tie-break hash */
  int32_t coarsen_to;    /* coarsen while n > coarsen_to (>= 1; default 2048) */
  int32_t match_rounds;  /* proposal rounds per level, [0, 64] (default 8) */
  int32_t refine_passes; /* refinement passes per level, [0, 64] (default 8) */
  int32_t init_trials;   /* greedy-growing trials, [1, 64] (default 16) */
  int32_t flags;         /* GP_LEARNED | GP_TRACE | GP_HOST_PTRS (for part/res of batch calls) */
  int32_t reserved;
  const void* model;     /* from gp_model_create / gp_model_load; required iff GP_LEARNED */
} gp_options;

typedef struct {
  int64_t cut;           /* sum of w over edges whose ends lie in different parts */
  int64_t load[2];       /* balance-column weight of part 0 and part 1 */
  int64_t time[2];       /* sum of cpu costs of part 0, sum of gpu costs of part 1 */
  int32_t feasible;      /* load[p] <= maxw[p] for both parts */
  int32_t levels;        /* number of coarse graphs built */
  int32_t used_learned;  /* 1 when the learned proposal beat the plain one */
  int32_t status;        /* gp_status of this graph (batched calls); GP_OK otherwise */
  int64_t volume;        /* communication volume (GP_VOLUME; 0 otherwise) */
} gp_result;

/* Fill *o with the defaults: ratio 1:4, eps 3 %, CPU column, seed 0, 2048, 8, 8, 16. */
void gp_options_default(gp_options* o);

/* Eq. (1)-(2) as an integer ratio: R_CPU = T_GPU/(T_GPU+T_CPU), so
 * ratio = {t_gpu, t_cpu} divided by their gcd.  t >= 0, not both 0. */
gp_status gp_ratio_from_times(int64_t t_cpu, int64_t t_gpu, int64_t ratio[2]);

/* Check the graph and copy it into library-owned device memory in canonical
 * form (rows sorted by neighbour).  The inputs are read only during the call
 * and may be freed afterwards.  flags: GP_HOST_PTRS when the arrays are host
 * memory.  stream: the hipStream_t all work of this handle runs on (NULL =
 * the default stream).  Returns GP_EINVAL, GP_ERANGE, GP_ESELF, GP_EDUP,
 * GP_EASYM or GP_EOVERFLOW, checked in that order of precedence, for a
 * malformed graph; *g is then left NULL. */
gp_status gp_create(gp_graph** g, int32_t n, const int32_t* xadj, const int32_t* adjncy,
                    const int64_t* adjwgt, const int64_t* vwgt, int32_t flags, void* stream);

/* Change the stream of a handle. */
gp_status gp_set_stream(gp_graph* g, void* stream);

/* Partition.  part: caller-owned int8[n] receiving 0 (CPU) or 1 (GPU) per
 * vertex, in the caller's vertex order; device memory unless the handle was
 * created with GP_HOST_PTRS.  res: host memory.  The call returns after the
 * result is complete.  An infeasible balance is not an error: the call
 * returns GP_OK with res->feasible = 0 and the best assignment found. */
gp_status gp_partition(gp_graph* g, const gp_options* o, int8_t* part, gp_result* res);

/* As gp_partition, also writing 8 int64 per level (level 0 first, at most
 * trace_cap levels, host memory): n, 2m, refinement passes, vertices moved,
 * cut after refinement, load[0], load[1], pairs matched on that level. */
gp_status gp_partition_trace(gp_graph* g, const gp_options* o, int8_t* part, gp_result* res,
                             int64_t* trace, int32_t trace_cap);

/* Copies level `level` (0 = the input graph) of the last gp_partition /
 * gp_partition_trace on g to host memory: its vertex count and entry count,
 * CSR (xadj n+1, adjncy and adjwgt nnz), vertex weights (n x 2: cpu, gpu),
 * the matching that built the next level (n; only below the coarsest level)
 * and the final bisection of that level (n).  Every output may be NULL.
 * Blocks until the copies are done.  GP_EINVAL when no partition has run or
 * the level was not built by it.  For inspecting the multilevel hierarchy
 * that the partition builds (the paper delegates partitioning to a
 * multilevel library, Section III-A; the coarsening rules are this
 * library's own); not needed to partition. */
gp_status gp_level_read(gp_graph* g, int32_t level, int32_t* n, int64_t* nnz, int32_t* xadj,
                        int32_t* adjncy, int64_t* adjwgt, int64_t* vwgt, int32_t* match,
                        int8_t* part);

void gp_destroy(gp_graph* g);

/* Device-memory budget of a handle, for callers that share one GPU among
 * several handles or other work.  A handle holds its copy of the graph and
 * scratch buffers sized to the levels it builds (a fixed control block of a
 * few hundred bytes aside); buffers grow on demand and are kept for the next
 * call.  bytes = -1 (the default) sets no limit; bytes >= 0 makes a call
 * that would grow the handle's buffers past it return GP_ENOMEM before it
 * grows them.  A call refused this way may have launched part of its work
 * and leaves gp_level_read nothing to read; the buffers already held stay
 * valid, so the same call with a larger limit then succeeds with the same
 * result.  A k-way partition charges its subgraphs' buffers to the handle.
 * The limit never frees memory already held.  bytes < -1: GP_EINVAL. */
gp_status gp_set_workspace_limit(gp_graph* g, int64_t bytes);

/* Device bytes the handle's buffers hold now (-1 for a null handle). */
int64_t gp_workspace_bytes(const gp_graph* g);

/* ---------------------------------------------------------------------
 * k-way partition (CPU + GPU + further processors).  The paper leaves more
 * than two processors to future work (Section VI) and gives each processor
 * a share inversely proportional to its execution time (Eq. (1)
 * generalised: R_i = (1/T_i) / sum_j (1/T_j)); here the shares come as
 * integers ratio[0..k-1].  The partition is built by recursive bisection:
 * the vertices of part range [lo, hi) (first [0, k)) are split with the
 * two-way partition into [lo, mid) and [mid, hi), mid = lo + (hi - lo) / 2,
 * at target ratio (sum of ratio[lo..mid), sum of ratio[mid..hi)) and the
 * caller's eps and other options, on the subgraph they induce (vertices in
 * ascending id order).  Each part's imbalance bound therefore compounds over
 * the log2 k bisections above it.
 * --------------------------------------------------------------------- */
typedef struct {
  int64_t cut;           /* sum of w over edges whose ends lie in different parts */
  int32_t feasible;      /* every bisection met its balance bound */
  int32_t bisections;    /* two-way partitions run (ranges whose subgraph was not empty) */
} gp_kway_result;

/* k in [1, 1024]; ratio: host int64[k], each in [0, 2^40), sum in (0, 2^40);
 * o: as for gp_partition (o->ratio is ignored, GP_LEARNED gives GP_EMODEL);
 * part: caller-owned int32[n] receiving the part 0..k-1 of every vertex,
 * device memory unless the handle was created with GP_HOST_PTRS; load: host
 * int64[k] (may be NULL) receiving each part's weight in the balance column;
 * res: host.  A range with a zero share receives no vertex unless its
 * sibling's share is zero too. */
gp_status gp_partition_kway(gp_graph* g, int32_t k, const int64_t* ratio, const gp_options* o,
                            int32_t* part, int64_t* load, gp_kway_result* res);

/* Learned coarsest-level proposal (GP_LEARNED): a 3-layer message-passing
 * network, hidden size 64, whose 25,153 BF16 parameters (uint16 bits, host
 * memory) are laid out as Win[64][4], b_in[64], 3 x (Ws[64][64], Wn[64][64],
 * b[64]), wo[64], bo (matrices [output][input]).  It scores the coarsest
 * vertices; the best fill the grown side; refinement follows.  Both that
 * bisection and the plain one are projected and refined down to the input
 * graph, and the plain result is kept unless the learned one ends strictly
 * better there in (infeasible, cut), so the learned form never returns a
 * larger cut than the plain one.  It runs when the coarsest graph has at
 * most 3,072 vertices.  After such a call gp_level_read shows the levels of
 * the learned run.  *model is device state owned by the library. */
gp_status gp_model_create(const uint16_t* params, int32_t count, const void** model);
/* As gp_model_create, with the blob read from a file holding exactly the
 * 25,153 little-endian BF16 values in the order above (50,306 bytes, no
 * header; what the training driver writes).  GP_EINVAL when the file cannot
 * be opened, GP_EMODEL when its size differs; *model is then NULL. */
gp_status gp_model_load(const char* path, const void** model);
void gp_model_free(const void* model);
/* The network's FP32 score of every vertex of g's graph (its canonical rows):
 * scores is float[n], device memory unless g was created with GP_HOST_PTRS. */
gp_status gp_model_scores(const void* model, gp_graph* g, float* scores);

/* Per-kernel profile of the calls made while profiling is on (HIP events
 * around every launch; adds a host wait per level).  One row per kernel (and
 * team width): */
typedef struct {
  char name[40];        /* kernel, e.g. "k_refine_gain<8>" */
  int64_t launches;     /* launches recorded */
  int64_t executed;     /* launches that did their work; the others exited on a device flag */
  double ms;            /* summed event time of all launches, milliseconds */
  double bytes;         /* algorithmic bytes moved by the executed launches (0: not defined) */
} gp_prof_row;

/* on != 0 starts recording on this handle; on == 0 stops. */
gp_status gp_profile_enable(gp_graph* g, int32_t on);
/* Copies at most cap rows (host memory) and returns the row count (or -1);
 * reset != 0 clears the accumulated rows afterwards. */
int32_t gp_profile_read(gp_graph* g, gp_prof_row* rows, int32_t cap, int32_t reset);

/* ---------------------------------------------------------------------
 * Batched partition: many independent graphs in one persistent kernel
 * (one workgroup per graph, largest graphs first), launched as a captured
 * hipGraph.  Each graph's result equals gp_create + gp_partition on that
 * graph alone with the same options.
 *
 * Layout (device memory): graph g owns vertices voff[g]..voff[g+1] and CSR
 * entries eoff[g]..eoff[g+1] (int64[G+1] each, voff[0] = eoff[0] = 0); its
 * xadj has n_g+1 local offsets starting at 0 and sits at
 * xadj[voff[g]+g .. voff[g+1]+g]; adjncy holds local vertex ids; vwgt is
 * int64[voff[G]][2]; part receives int8[voff[G]].  res: host array of G
 * results, res[g].status holds that graph's check result (GP_ERANGE, ...).
 * GP_LEARNED is not available here (GP_EMODEL).
 * --------------------------------------------------------------------- */
typedef struct gp_batch gp_batch;

/* A batch context owning the device scratch (reused by later calls). */
gp_status gp_batch_create(gp_batch** b, void* stream);
/* workgroups: persistent workgroups (0 = two per compute unit); chunk:
 * graphs taken per queue pop; order_mode: 0 largest first, 1 input order,
 * 2 the graphs that took longest in the previous call of the same batch
 * size on b first (largest first without one).  None of them changes any
 * result. */
gp_status gp_batch_config(gp_batch* b, int32_t workgroups, int32_t chunk, int32_t order_mode);
/* Lanes per row of the batched kernels: the degree-based choice (4 to 64)
 * scaled by 2^shift and kept within [4, 64], shift in [-4, 1] (default 0).
 * No result depends on it; it is a tuning knob of the autotuner. */
gp_status gp_batch_team_width(gp_batch* b, int32_t shift);
gp_status gp_partition_batch(gp_batch* b, int32_t G, const int64_t* voff, const int64_t* eoff,
                             const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                             const int64_t* vwgt, const gp_options* o, int8_t* part,
                             gp_result* res);
void gp_batch_destroy(gp_batch* b);
/* Timeline of the last successful gp_partition_batch call on b, to see what
 * sets its time (a long graph at the end, or every workgroup busy to the
 * end): ticks (host int64[2G]) receives, for graph g, the device wall clock
 * when a workgroup took it (2g) and when it finished it (2g + 1); *hz (may
 * be NULL) the clock's rate.  A graph redone after running out of arena
 * shows its last run.  G above the last call's count: GP_EINVAL. */
gp_status gp_batch_timeline(gp_batch* b, int32_t G, int64_t* ticks, int64_t* hz);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gp_partition_batch with
 * no allocation of any kind.  Its scratch is one fixed 64 MiB device array
 * per GPU, held from the first call on that GPU until the process ends.
 * All pointers are device memory, res included (G records); the call only
 * queues two kernels on `stream` and returns without waiting.  Graphs are
 * taken in input order.  nmax / nnzmax bound every graph's vertex and entry
 * count (a graph beyond them gets status GP_EINVAL); ntot / nnztot are the
 * totals voff[G] and eoff[G].  When the per-workgroup scratch for these
 * bounds plus the level arena estimate (3 x (57 ntot + 12 nnztot) +
 * 8192 G + 1 MiB bytes) exceed the 64 MiB, the call returns GP_ENOMEM and
 * queues nothing; a graph whose levels still overrun the arena gets status
 * GP_ENOMEM (no retry).  Calls that overlap on one GPU share its array and
 * race: run them on one stream.  GP_LEARNED is not available (GP_EMODEL). */
gp_status gp_partition_batch_noalloc(int32_t G, const int64_t* voff, const int64_t* eoff,
                                     const int32_t* xadj, const int32_t* adjncy,
                                     const int64_t* adjwgt, const int64_t* vwgt,
                                     const gp_options* o, int32_t nmax, int32_t nnzmax,
                                     int64_t ntot, int64_t nnztot, int8_t* part,
                                     gp_result* res, void* stream);
/* Autotuner of the batched path: runs gp_partition_batch with each of 18
 * configurations (1 or 2 persistent workgroups per compute unit x 1, 2 or 4
 * graphs per queue pop x largest-first, input or previous-longest-first
 * order), then the fastest of them with the team width divided by 16, 8, 4
 * and 2, and doubled (gp_batch_team_width); checks that every configuration
 * returns byte-identical part and res, times `reps` calls of each (host wall
 * clock, whole calls), and keeps the fastest in b for later calls.  chosen (host
 * int32[4], may be NULL) receives workgroups, chunk, order_mode and the team
 * width shift; ms (may be NULL) its mean time per call.  part and res hold
 * the result on return.  GP_EDEVICE if two configurations disagree (the
 * previous configuration is then restored). */
gp_status gp_batch_autotune(gp_batch* b, int32_t G, const int64_t* voff, const int64_t* eoff,
                            const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                            const int64_t* vwgt, const gp_options* o, int8_t* part,
                            gp_result* res, int32_t reps, int32_t* chosen, double* ms);

/* Export, during later gp_partition_batch calls, every graph's coarsest
 * graph and its plain (greedy-growing + refinement) bisection - the training
 * data of the learned proposal.  All pointers device memory.  rec: int64[4G]
 * per graph = n, 2m, vertex slot, entry slot (-1 when the buffers are full);
 * the graph's xadj (n+1 local offsets), vwgt (n x 2) and part (n) start at its
 * vertex slot of xadj / vwgt / part (cap_vertices slots), its adjncy and
 * adjwgt at its entry slot (cap_entries slots).  rec == NULL turns it off. */
gp_status gp_batch_export(gp_batch* b, int64_t* rec, int32_t* xadj, int64_t* vwgt, int8_t* part,
                          int64_t cap_vertices, int32_t* adjncy, int64_t* adjwgt,
                          int64_t cap_entries);

/* ---------------------------------------------------------------------
 * Training of the learned proposal (GPU; MFMA BF16 -> FP32 dense layers,
 * CSR message passing and its transpose, BCE-with-logits loss weighted by
 * b_v / W_g and averaged over the graphs of a mini-batch, Adam on FP32
 * master weights).  Not bit-exact; gradients are checked against an FP64
 * reference within a tolerance.
 * --------------------------------------------------------------------- */
typedef struct gp_trainer gp_trainer;
/* init_params: host float[25153] in the blob order of gp_model_create */
gp_status gp_train_create(gp_trainer** t, const float* init_params, int32_t count, void* stream);
/* The training set, device memory, in the batched layout (see
 * gp_partition_batch); labels: int8 per vertex, 1 = on the grown side. */
gp_status gp_train_set_data(gp_trainer* t, int32_t G, const int64_t* voff, const int64_t* eoff,
                            const int32_t* xadj, const int32_t* adjncy, const int64_t* adjwgt,
                            const int64_t* vwgt, const int8_t* labels, int32_t balance_on);
/* one Adam step on graphs [g0, g1); *loss (host, may be NULL) gets the batch loss */
gp_status gp_train_step(gp_trainer* t, int32_t g0, int32_t g1, float lr, float* loss);
/* the gradient (host float[25153]) and loss on graphs [g0, g1), no update */
gp_status gp_train_grad(gp_trainer* t, int32_t g0, int32_t g1, float* grad, float* loss);
/* FP32 master weights and/or their BF16 copy (host arrays, may be NULL) */
gp_status gp_train_params(gp_trainer* t, float* f32, uint16_t* bf16);
void gp_train_destroy(gp_trainer* t);

/* ---------------------------------------------------------------------
 * Schedule simulator (host code): replays a task DAG on ncpu CPU workers
 * (memory node 0) and ngpu GPU workers (node 1) under one of the runtime
 * policies the paper compares (Section IV-C): eager (the worker free first),
 * dmda-like (the worker where the task would finish first, transfers
 * included) or gp (the node part[v] names, e.g. a gp_partition result).
 * Tasks are placed in id order, which must be a topological order (every
 * dependency u-v points from the smaller id to the larger).  vwgt[v] =
 * (cpu cost, gpu cost) in time units; a dependency between nodes costs one
 * transfer of the producer's output (as large as its largest edge to a
 * successor) over a single link (latency + ceil(bytes / bw) time units,
 * transfers in request order), made once per producer and destination
 * node.  All pointers are host memory; task_node (int8[n]) and
 * task_finish (int64[n]) may be NULL.
 * --------------------------------------------------------------------- */
enum { GP_SIM_EAGER = 0, GP_SIM_DMDA = 1, GP_SIM_GP = 2 };
typedef struct {
  int64_t makespan;      /* finish time of the last task */
  int64_t transfers;     /* transfers between the memory nodes */
  int64_t bytes;         /* bytes they moved */
  int64_t busy[2];       /* summed task time on the CPU workers, on the GPU workers */
  int64_t tasks[2];      /* tasks placed on the CPU, on the GPU */
} gp_sim_result;
gp_status gp_simulate(int32_t n, const int32_t* xadj, const int32_t* adjncy,
                      const int64_t* adjwgt, const int64_t* vwgt, const int8_t* part,
                      int32_t policy, int32_t ncpu, int32_t ngpu, int64_t latency, int64_t bw,
                      gp_sim_result* res, int8_t* task_node, int64_t* task_finish);

const char* gp_strerror(gp_status s);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
