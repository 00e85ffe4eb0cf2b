"""Shared test helpers: tiny random graphs, exhaustive search, CSR checks."""
from __future__ import annotations

import numpy as np

import dagen


def random_graph(n: int, p: float, rng: np.random.Generator, wmax: int = 10, vmax: int = 10,
                 const_w: bool = False, name: str = "rand") -> dagen.Graph:
    """Erdos-Renyi-like undirected graph with integer weights (test input only)."""
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    src, dst = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    if const_w:
        w = np.full(len(src), wmax, np.int64)
    else:
        w = rng.integers(1, wmax + 1, len(src)).astype(np.int64)
    vw = np.stack([rng.integers(1, vmax + 1, n), rng.integers(1, vmax + 1, n)], 1).astype(np.int64)
    return dagen.to_csr(n, src, dst, w, vw, name)


def edges_of(g) -> tuple:
    """Unique undirected edges (u < v) with weights."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj.astype(np.int64)))
    cols = g.adjncy.astype(np.int64)
    keep = rows < cols
    return rows[keep], cols[keep], g.adjwgt[keep]


def cut_of(g, part) -> int:
    u, v, w = edges_of(g)
    part = np.asarray(part)
    return int(w[part[u] != part[v]].sum())


def brute_force(g, b: np.ndarray, maxw) -> tuple:
    """Exhaustive minimum cut over all 2^n assignments with pw_p <= maxw_p.

    Returns (cut, part) with part the lexicographically smallest optimum
    (vertex 0 most significant, 0 < 1), or (None, None) when nothing is
    feasible.
    """
    n = g.n
    assert n <= 20
    masks = np.arange(1 << n, dtype=np.int64)
    # vertex v's side is bit (n-1-v), so ascending masks are lexicographic order
    bits = [(masks >> (n - 1 - v)) & 1 for v in range(n)]
    pw1 = np.zeros(1 << n, np.int64)
    for v in range(n):
        pw1 += bits[v] * int(b[v])
    pw0 = int(np.sum(b)) - pw1
    ok = (pw0 <= int(maxw[0])) & (pw1 <= int(maxw[1]))
    if not ok.any():
        return None, None
    u, vv, w = edges_of(g)
    cut = np.zeros(1 << n, np.int64)
    for a, c, wt in zip(u, vv, w):
        cut += (bits[a] ^ bits[c]) * int(wt)
    cut = np.where(ok, cut, np.iinfo(np.int64).max)
    best = int(np.argmin(cut))
    part = np.array([(best >> (n - 1 - v)) & 1 for v in range(n)], np.int8)
    return int(cut[best]), part


def assert_canonical(xadj, adjncy, adjwgt, n):
    """Rows sorted strictly ascending, no self loops, symmetric weights."""
    xadj = np.asarray(xadj)
    assert xadj[0] == 0 and np.all(np.diff(xadj) >= 0)
    d = {}
    for u in range(n):
        row = adjncy[xadj[u]:xadj[u + 1]]
        assert np.all(np.diff(row) > 0), f"row {u} not strictly sorted"
        assert not np.any(row == u), f"self loop at {u}"
        for v, w in zip(row, adjwgt[xadj[u]:xadj[u + 1]]):
            d[(u, int(v))] = int(w)
    for (u, v), w in d.items():
        assert d.get((v, u)) == w, f"asymmetric {u}-{v}"


def dense_adj(n, xadj, adjncy, adjwgt) -> np.ndarray:
    a = np.zeros((n, n), np.int64)
    for u in range(n):
        for e in range(xadj[u], xadj[u + 1]):
            a[u, adjncy[e]] += adjwgt[e]
    return a


def path_graph(n: int, w: int = 1, vw: int = 1) -> dagen.Graph:
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    return dagen.to_csr(n, src, dst, np.full(n - 1, w, np.int64),
                        np.full((n, 2), vw, np.int64), f"path{n}")


def complete_graph(n: int, w: int = 1, vw: int = 1) -> dagen.Graph:
    iu, ju = np.triu_indices(n, 1)
    return dagen.to_csr(n, iu.astype(np.int32), ju.astype(np.int32),
                        np.full(len(iu), w, np.int64), np.full((n, 2), vw, np.int64), f"K{n}")


def edgeless_graph(n: int, vw) -> dagen.Graph:
    vw = np.asarray(vw, np.int64)
    if vw.ndim == 1:
        vw = np.stack([vw, vw], 1)
    return dagen.to_csr(n, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64),
                        vw, f"empty{n}")
