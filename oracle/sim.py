"""CPU oracle of the schedule simulator (test infrastructure).

Replays a task DAG on CPU and GPU workers under the three runtime policies
the paper compares (Section IV-C, Figs. 5-6): eager, a data-aware policy that
places each task where it would finish first (dmda), and the graph-partition
policy (the node the partition names).  Reading taken here: tasks are placed
one by one in id order (a topological order: dependencies point from the
smaller id to the larger); a task starts when its worker is free and its
inputs are on its node; a dependency across nodes costs one transfer of the
producer's output over a single link (latency + ceil(bytes / bw), transfers in the
order they are asked for, each starting when the link is free and the
producer has finished); the data a task produces is as large as its largest
edge to a successor, and its first transfer to a node serves every later
consumer there.  Ties go to GPU workers first, then to
the lower worker index.  Plain Python.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

EAGER, DMDA, GP = 0, 1, 2


@dataclass
class SimResult:
    makespan: int
    transfers: int
    bytes: int
    busy: tuple
    tasks: tuple
    node: list
    finish: list


def simulate(graph, policy: int, part=None, ncpu: int = 3, ngpu: int = 1, latency: int = 0,
             bw: int = 1) -> SimResult:
    n = graph.n
    xadj = [int(x) for x in graph.xadj]
    adj = [int(x) for x in graph.adjncy]
    w = [int(x) for x in graph.adjwgt]
    cost = [(int(a), int(b)) for a, b in np.asarray(graph.vwgt).reshape(n, 2)]
    workers = [1] * ngpu + [0] * ncpu          # node of each worker, GPU workers first
    avail = [0] * len(workers)
    fin = [0] * n
    node = [0] * n
    arrived = {}                              # (producer, node) -> arrival time
    state = {"link": 0, "transfers": 0, "bytes": 0}
    # size of each task's output: its largest edge to a successor
    out = [max([w[e] for e in range(xadj[u], xadj[u + 1]) if adj[e] > u], default=0)
           for u in range(n)]

    def ready_on(v, p, commit):
        t, link = 0, state["link"]
        for e in range(xadj[v], xadj[v + 1]):
            u = adj[e]
            if u >= v:
                continue                      # a consumer, not a producer
            if node[u] == p:
                at = fin[u]
            elif (u, p) in arrived:
                at = arrived[(u, p)]
            else:
                at = max(link, fin[u]) + latency + -(-out[u] // bw)
                link = at
                if commit:
                    arrived[(u, p)] = at
                    state["transfers"] += 1
                    state["bytes"] += out[u]
            t = max(t, at)
        if commit:
            state["link"] = link
        return t

    busy, count = [0, 0], [0, 0]
    for v in range(n):
        best, best_key = None, None
        for i, p in enumerate(workers):
            if policy == GP and p != int(part[v]):
                continue
            if policy == DMDA:
                key = max(avail[i], ready_on(v, p, False)) + cost[v][p]
            else:
                key = avail[i]
            if best is None or key < best_key:
                best, best_key = i, key
        p = workers[best]
        node[v] = p
        start = max(avail[best], ready_on(v, p, True))
        fin[v] = start + cost[v][p]
        avail[best] = fin[v]
        busy[p] += cost[v][p]
        count[p] += 1
    return SimResult(max(fin) if n else 0, state["transfers"], state["bytes"], tuple(busy),
                     tuple(count), node, fin)
