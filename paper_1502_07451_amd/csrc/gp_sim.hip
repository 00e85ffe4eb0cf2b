// gp_sim.hip - schedule simulator of a task DAG on a CPU + GPU machine.
//
// The paper compares three runtime policies on one CPU-GPU node (Section
// IV-C, Figs. 5-6): eager (any idle processor takes the next task), a
// data-aware policy that places each task where it would finish first
// (StarPU's dmda), and the graph-partition policy (every task pinned to the
// processor its part names).  This host routine replays a DAG under one of
// them and reports the makespan and the transfers, so the partition can be
// judged the way the paper judges it (fewest transfers, all work on the GPU
// when the gap between the processors is large).
//
// Model (all integer time units):
//   * tasks 0..n-1 in a topological order: every dependency u-v of the
//     undirected graph points from the smaller id to the larger one (the
//     generators number tasks in program order);
//   * ncpu CPU workers on memory node 0, ngpu GPU workers on node 1; task v
//     costs vwgt[v][0] on a CPU worker and vwgt[v][1] on a GPU worker;
//   * tasks are placed one by one in id order (list scheduling); a task
//     starts when its worker is free and all its inputs are on its node;
//   * the output of task u sits on u's node when u finishes; a consumer on
//     the other node needs a transfer over one link (one copy engine: the
//     transfers queue in the order they are requested), which takes
//     latency + ceil(bytes / bw) and starts once the link is free and u has
//     finished; u's output is as large as u's largest edge to a successor,
//     and its first transfer to a node serves every later consumer there;
//   * eager: the worker that is free first (ties: GPU workers before CPU
//     workers, lower index first); dmda: the worker on which the task would
//     finish first, counting the transfers it would need (same ties); gp:
//     the earliest-free worker of the node part[v] names.
#include <stdint.h>
#include <string.h>

#include <unordered_map>
#include <vector>

#include "../../include/gp.h"

namespace {

struct SimState {
  int32_t n;
  const int32_t* xadj;
  const int32_t* adj;
  const int64_t* w;
  int64_t latency, bw;
  std::vector<int64_t> fin;
  std::vector<int64_t> out;  // size of each task's output: its largest successor edge
  std::vector<int8_t> node;
  // (producer, node) -> arrival time of its output on that node
  std::unordered_map<int64_t, int64_t> arrived;
  int64_t link_free = 0;
  int64_t transfers = 0, bytes = 0;

  int64_t xfer_time(int64_t b) const { return latency + (b + bw - 1) / bw; }

  // earliest time all inputs of v are on node p; commit = record the
  // transfers it takes (else only what they would cost)
  int64_t ready_on(int32_t v, int p, bool commit) {
    int64_t t = 0, link = link_free;
    for (int32_t e = xadj[v]; e < xadj[v + 1]; e++) {
      const int32_t u = adj[e];
      if (u >= v) continue;  // a consumer, not a producer
      int64_t at;
      if (node[u] == p) {
        at = fin[u];
      } else {
        const int64_t key = (int64_t)u * 2 + p;
        auto it = arrived.find(key);
        if (it != arrived.end()) {
          at = it->second;
        } else {
          const int64_t start = link > fin[u] ? link : fin[u];
          at = start + xfer_time(out[u]);
          link = at;
          if (commit) {
            arrived.emplace(key, at);
            transfers++;
            bytes += out[u];
          }
        }
      }
      t = at > t ? at : t;
    }
    if (commit) link_free = link;
    return t;
  }
};

}  // namespace

extern "C" {

gp_status gp_simulate(int32_t n, const int32_t* xadj, const int32_t* adjncy,
                      const int64_t* adjwgt, const int64_t* vwgt, const int8_t* part,
                      int32_t policy, int32_t ncpu, int32_t ngpu, int64_t latency, int64_t bw,
                      gp_sim_result* res, int8_t* task_node, int64_t* task_finish) {
  if (n < 0 || !res || ncpu < 0 || ngpu < 0 || ncpu + ngpu == 0 || latency < 0 || bw < 1 ||
      policy < GP_SIM_EAGER || policy > GP_SIM_GP || (n > 0 && (!xadj || !vwgt)) ||
      (policy == GP_SIM_GP && n > 0 && !part))
    return GP_EINVAL;
  if (n > 0 && xadj[n] > 0 && (!adjncy || !adjwgt)) return GP_EINVAL;
  for (int32_t v = 0; v < n; v++)
    if (vwgt[2 * v] < 0 || vwgt[2 * v + 1] < 0 ||
        (policy == GP_SIM_GP && (part[v] < 0 || part[v] > 1)) ||
        (policy == GP_SIM_GP && part[v] == 0 && ncpu == 0) ||
        (policy == GP_SIM_GP && part[v] == 1 && ngpu == 0))
      return GP_EINVAL;
  SimState S;
  S.n = n;
  S.xadj = xadj;
  S.adj = adjncy;
  S.w = adjwgt;
  S.latency = latency;
  S.bw = bw;
  S.fin.assign((size_t)n, 0);
  S.node.assign((size_t)n, 0);
  S.out.assign((size_t)n, 0);
  for (int32_t u = 0; u < n; u++)
    for (int32_t e = xadj[u]; e < xadj[u + 1]; e++)
      if (adjncy[e] > u && adjwgt[e] > S.out[u]) S.out[u] = adjwgt[e];
  // workers: GPU workers first (the tie order), then CPU workers
  const int nw = ngpu + ncpu;
  std::vector<int64_t> avail((size_t)nw, 0);
  auto wnode = [&](int i) { return i < ngpu ? 1 : 0; };
  int64_t busy[2] = {0, 0}, count[2] = {0, 0}, makespan = 0;
  for (int32_t v = 0; v < n; v++) {
    int best = -1;
    int64_t best_key = 0;
    for (int i = 0; i < nw; i++) {
      const int p = wnode(i);
      if (policy == GP_SIM_GP && p != part[v]) continue;
      int64_t key;
      if (policy == GP_SIM_DMDA) {
        const int64_t r = S.ready_on(v, p, false);
        key = (avail[i] > r ? avail[i] : r) + vwgt[2 * v + p];
      } else {
        key = avail[i];
      }
      if (best < 0 || key < best_key) {
        best = i;
        best_key = key;
      }
    }
    const int p = wnode(best);
    S.node[v] = (int8_t)p;
    const int64_t r = S.ready_on(v, p, true);
    const int64_t start = avail[best] > r ? avail[best] : r;
    const int64_t c = vwgt[2 * v + p];
    S.fin[v] = start + c;
    avail[best] = S.fin[v];
    busy[p] += c;
    count[p]++;
    makespan = S.fin[v] > makespan ? S.fin[v] : makespan;
    if (task_node) task_node[v] = (int8_t)p;
    if (task_finish) task_finish[v] = S.fin[v];
  }
  gp_sim_result r;
  memset(&r, 0, sizeof(r));
  r.makespan = makespan;
  r.transfers = S.transfers;
  r.bytes = S.bytes;
  r.busy[0] = busy[0];
  r.busy[1] = busy[1];
  r.tasks[0] = count[0];
  r.tasks[1] = count[1];
  *res = r;
  return GP_OK;
}

}  // extern "C"
