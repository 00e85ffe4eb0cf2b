"""CPU oracle of the k-way partition by recursive bisection (test infrastructure).

The paper leaves more than two processors to future work (Section VI), each
with a share inversely proportional to its execution time (Eq. (1)
generalised).  Reading taken here: the vertices of part range [lo, hi)
(first [0, k)) are split by the oracle's two-way partition into [lo, mid)
and [mid, hi), mid = lo + (hi - lo) // 2, with target ratio (sum of the
shares of [lo, mid), sum of the shares of [mid, hi)) and the same options
otherwise, on the subgraph they induce, its vertices in ascending id order.
Written with numpy and the two-way oracle only.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import OK, EINVAL, EMODEL, FLAG_LEARNED, Options, partition


@dataclass
class KwayResult:
    status: int
    part: np.ndarray      # int32 part id of every vertex
    cut: int
    load: tuple           # balance-column weight of each part
    feasible: int         # every bisection met its balance bound
    bisections: int


def induced(n, xadj, adjncy, adjwgt, vwgt, keep):
    """Subgraph induced by the vertices with keep[v], renumbered in ascending
    id order; rows keep their order, so they stay sorted."""
    keep = np.asarray(keep, bool)
    newid = np.cumsum(keep) - 1
    deg = np.diff(np.asarray(xadj, np.int64))
    rows = np.repeat(np.arange(n), deg)
    adjncy = np.asarray(adjncy, np.int64)
    e = keep[rows] & keep[adjncy] if len(adjncy) else np.zeros(0, bool)
    src = newid[rows[e]]
    ns = int(keep.sum())
    cnt = np.bincount(src, minlength=ns) if ns else np.zeros(0, np.int64)
    sx = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    sa = newid[adjncy[e]].astype(np.int32)
    sw = np.asarray(adjwgt, np.int64)[e]
    sv = np.asarray(vwgt, np.int64).reshape(n, 2)[keep]
    return ns, sx, sa, sw, sv


def partition_kway(graph, k: int, ratio, opts: Options | None = None) -> KwayResult:
    opts = opts or Options()
    n = graph.n
    ratio = [int(x) for x in ratio]
    if k < 1 or len(ratio) != k or any(r < 0 or r >= 1 << 40 for r in ratio) \
            or not 0 < sum(ratio) < 1 << 40:
        return KwayResult(EINVAL, np.zeros(n, np.int32), 0, (), 0, 0)
    if opts.flags & FLAG_LEARNED:
        return KwayResult(EMODEL, np.zeros(n, np.int32), 0, (), 0, 0)
    label = np.zeros(n, np.int32)
    feasible, bis = 1, 0
    todo = [(0, k)]
    while todo:
        lo, hi = todo.pop()
        if hi - lo < 2:
            continue
        mid = lo + (hi - lo) // 2
        r0, r1 = sum(ratio[lo:mid]), sum(ratio[mid:hi])
        members = label == lo
        if not members.any():
            continue
        if r0 + r1 > 0:
            ns, sx, sa, sw, sv = induced(n, graph.xadj, graph.adjncy, graph.adjwgt, graph.vwgt,
                                         members)
            res = partition(n=ns, xadj=sx, adjncy=sa, adjwgt=sw, vwgt=sv,
                            opts=replace(opts, ratio=(r0, r1)))
            if res.status != OK:
                return KwayResult(res.status, np.zeros(n, np.int32), 0, (), 0, 0)
            feasible &= res.feasible
            bis += 1
            idx = np.nonzero(members)[0]
            label[idx[res.part == 1]] = mid
        todo.append((mid, hi))
        todo.append((lo, mid))
    b = np.asarray(graph.vwgt, np.int64).reshape(n, 2)[:, opts.balance_on]
    load = tuple(int(b[label == p].sum()) for p in range(k))
    deg = np.diff(np.asarray(graph.xadj, np.int64))
    rows = np.repeat(np.arange(n), deg)
    diff = label[rows] != label[np.asarray(graph.adjncy, np.int64)] if n else np.zeros(0, bool)
    cut = int(np.asarray(graph.adjwgt, np.int64)[diff].sum()) // 2
    return KwayResult(OK, label, cut, load, feasible, bis)
