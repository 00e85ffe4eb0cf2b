"""Seeded synthetic task-DAG generators (input side only).

Vertices are kernels and arrows are data dependencies; a vertex carries two
costs (CPU, GPU) and an edge carries the bytes a dependency transfers, the
weighted-graph model of Section III-B.  Every graph is rebuilt from a seed, so
the CPU oracle and the HIP path can be handed identical inputs.  Nothing here
partitions anything.

The arrays follow the partitioner's input layout: int32 ``xadj[n+1]``, int32
``adjncy[2m]``, int64 ``adjwgt[2m]`` (symmetric, rows sorted by neighbour) and
int64 ``vwgt[n][2]`` = (cpu cost, gpu cost).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdagen.so")
_lib = None

TILE_512_BYTES = 512 * 512 * 8        # one 512x512 fp64 tile: 2 MiB
TILE_1024_BYTES = 1024 * 1024 * 8     # one 1024x1024 fp64 tile: 8 MiB


def build() -> str:
    """Compile the generator library in place with gcc."""
    src = os.path.join(_HERE, "dagen.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.dg_rand.restype = u64
    lib.dg_rand.argtypes = [u64, u64, u64]
    lib.dg_cholesky_size.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.dg_lu_size.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.dg_cholesky.argtypes = [i32, i64, i32, i64, i64, u64, vp, vp, vp, vp]
    lib.dg_lu.argtypes = [i32, i64, i32, i64, i64, u64, vp, vp, vp, vp]
    lib.dg_layered_edges.restype = i64
    lib.dg_layered_edges.argtypes = [i64, i32, dbl, u64]
    lib.dg_layered.argtypes = [i64, i32, dbl, dbl, dbl, dbl, dbl, i64, u64, vp, vp, vp, vp]
    lib.dg_to_csr.restype = i64
    lib.dg_to_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
    lib.dg_batch_plan.argtypes = [i32, dbl, dbl, u64, vp, vp, vp, vp]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    """Host pointer of a; the pointer object keeps a alive until the call returns."""
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """A symmetric weighted CSR graph plus per-vertex (cpu, gpu) costs."""
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray
    vwgt: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.xadj[-1]) if self.n > 0 else 0

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2


@dataclass
class Dag:
    """A directed task DAG before symmetrisation."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    bytes: np.ndarray
    vwgt: np.ndarray


def rand_u64(seed: int, stream: int, idx: int) -> int:
    return int(_load().dg_rand(seed, stream, idx))


def to_csr(n: int, src: np.ndarray, dst: np.ndarray, nbytes: np.ndarray, vwgt: np.ndarray,
           name: str = "") -> Graph:
    """Drop arrow direction, merge parallel arrows by summing bytes, sort rows."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    nbytes = np.ascontiguousarray(nbytes, dtype=np.int64)
    ne = len(src)
    xadj = np.zeros(n + 1, dtype=np.int32)
    adj = np.empty(max(2 * ne, 1), dtype=np.int32)
    w = np.empty(max(2 * ne, 1), dtype=np.int64)
    nnz = lib.dg_to_csr(n, ne, _p(src), _p(dst), _p(nbytes), _p(xadj), _p(adj), _p(w))
    if nnz < 0:
        raise MemoryError("dg_to_csr failed")
    return Graph(n, xadj, adj[:nnz].copy(), w[:nnz].copy(),
                 np.ascontiguousarray(vwgt, dtype=np.int64).reshape(n, 2), name)


def cholesky_dag(T: int, b: int, jitter_pm: int = 0, rate: int = 4,
                 edge_bytes: int = TILE_512_BYTES, seed: int = 0) -> Dag:
    lib = _load()
    n, ne = ctypes.c_int64(), ctypes.c_int64()
    lib.dg_cholesky_size(T, ctypes.byref(n), ctypes.byref(ne))
    n, ne = n.value, ne.value
    vw = np.zeros((n, 2), dtype=np.int64)
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    by = np.zeros(ne, dtype=np.int64)
    rc = lib.dg_cholesky(T, b, jitter_pm, rate, edge_bytes, seed, _p(vw), _p(src), _p(dst), _p(by))
    if rc != 0:
        raise MemoryError("dg_cholesky failed")
    return Dag(n, src, dst, by, vw)


def lu_dag(T: int, b: int, jitter_pm: int = 0, rate: int = 4,
           edge_bytes: int = TILE_512_BYTES, seed: int = 0) -> Dag:
    lib = _load()
    n, ne = ctypes.c_int64(), ctypes.c_int64()
    lib.dg_lu_size(T, ctypes.byref(n), ctypes.byref(ne))
    n, ne = n.value, ne.value
    vw = np.zeros((n, 2), dtype=np.int64)
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    by = np.zeros(ne, dtype=np.int64)
    rc = lib.dg_lu(T, b, jitter_pm, rate, edge_bytes, seed, _p(vw), _p(src), _p(dst), _p(by))
    if rc != 0:
        raise MemoryError("dg_lu failed")
    return Dag(n, src, dst, by, vw)


def layered_dag(n: int, L: int, lam: float = 4.0, mu_v: float = 8.0, sig_v: float = 1.0,
                mu_e: float = 16.0, sig_e: float = 1.5, rate: int = 3, seed: int = 0) -> Dag:
    lib = _load()
    ne = lib.dg_layered_edges(n, L, lam, seed)
    vw = np.zeros((n, 2), dtype=np.int64)
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    by = np.zeros(ne, dtype=np.int64)
    lib.dg_layered(n, L, lam, mu_v, sig_v, mu_e, sig_e, rate, seed, _p(vw), _p(src), _p(dst),
                   _p(by))
    return Dag(n, src, dst, by, vw)


def dag_to_graph(d: Dag, name: str = "") -> Graph:
    return to_csr(d.n, d.src, d.dst, d.bytes, d.vwgt, name)


def cholesky(T: int, b: int, jitter_pm: int = 0, rate: int = 4,
             edge_bytes: int = TILE_512_BYTES, seed: int = 0) -> Graph:
    g = dag_to_graph(cholesky_dag(T, b, jitter_pm, rate, edge_bytes, seed), f"cholesky_T{T}")
    g.meta.update(kind="cholesky", T=T, b=b, jitter_pm=jitter_pm, rate=rate, seed=seed)
    return g


def lu(T: int, b: int, jitter_pm: int = 0, rate: int = 4,
       edge_bytes: int = TILE_512_BYTES, seed: int = 0) -> Graph:
    g = dag_to_graph(lu_dag(T, b, jitter_pm, rate, edge_bytes, seed), f"lu_T{T}")
    g.meta.update(kind="lu", T=T, b=b, jitter_pm=jitter_pm, rate=rate, seed=seed)
    return g


def layered(n: int, L: int, lam: float = 4.0, mu_v: float = 8.0, sig_v: float = 1.0,
            mu_e: float = 16.0, sig_e: float = 1.5, rate: int = 3, seed: int = 0) -> Graph:
    g = dag_to_graph(layered_dag(n, L, lam, mu_v, sig_v, mu_e, sig_e, rate, seed),
                     f"layered_n{n}_L{L}")
    g.meta.update(kind="layered", L=L, rate=rate, seed=seed)
    return g


def batch_plan(G: int, lo: float = 100.0, hi: float = 50000.0, seed: int = 0):
    lib = _load()
    size = np.zeros(G, dtype=np.int64)
    kind = np.zeros(G, dtype=np.int32)
    param = np.zeros(G, dtype=np.int32)
    gseed = np.zeros(G, dtype=np.uint64)
    lib.dg_batch_plan(G, lo, hi, seed, _p(size), _p(kind), _p(param), _p(gseed))
    return size, kind, param, gseed


def batch(G: int = 4096, lo: float = 100.0, hi: float = 50000.0, seed: int = 0):
    """Uneven batch: even index -> tiled Cholesky (b=512, 2 MiB edges, rate 4),
    odd index -> random layered (lognormal costs/bytes, rate 4)."""
    size, kind, param, gseed = batch_plan(G, lo, hi, seed)
    out = []
    for g in range(G):
        s = int(gseed[g])
        if kind[g] == 0:
            out.append(cholesky(int(param[g]), 512, 0, 4, TILE_512_BYTES, s))
        else:
            out.append(layered(int(size[g]), int(param[g]), rate=4, seed=s))
    return out


@dataclass
class Batch:
    """Concatenated graphs: graph g owns vertices voff[g]..voff[g+1] and CSR
    entries eoff[g]..eoff[g+1]; its local xadj (n_g+1 entries, starting at 0)
    sits at xadj[voff[g]+g : voff[g+1]+g+1]."""
    G: int
    voff: np.ndarray
    eoff: np.ndarray
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray
    vwgt: np.ndarray


def concat(graphs) -> Batch:
    G = len(graphs)
    voff = np.zeros(G + 1, dtype=np.int64)
    eoff = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        voff[i + 1] = voff[i] + g.n
        eoff[i + 1] = eoff[i] + g.nnz
    xadj = np.concatenate([g.xadj for g in graphs]) if G else np.zeros(0, np.int32)
    adj = np.concatenate([g.adjncy for g in graphs]) if G else np.zeros(0, np.int32)
    w = np.concatenate([g.adjwgt for g in graphs]) if G else np.zeros(0, np.int64)
    vw = np.concatenate([g.vwgt for g in graphs]) if G else np.zeros((0, 2), np.int64)
    return Batch(G, voff, eoff, xadj.astype(np.int32), adj.astype(np.int32),
                 w.astype(np.int64), vw.astype(np.int64).reshape(-1, 2))


# ---------------------------------------------------------------- workloads
def config_cholesky8() -> Graph:
    """Tiled Cholesky, T=8 tiles of 512x512: 120 tasks, 252 dependencies."""
    return cholesky(8, 512, 0, 4, TILE_512_BYTES, 0)


def config_cholesky64_lu48():
    """Tiled Cholesky T=64 and tiled LU T=48, 1024x1024 tiles, +-10 % jitter."""
    return [cholesky(64, 1024, 100, 4, TILE_1024_BYTES, 0),
            lu(48, 1024, 100, 4, TILE_1024_BYTES, 0)]


def config_layered4m(seed: int = 0) -> Graph:
    """Random layered DAG, 4,000,000 vertices in 64 layers, Poisson(4) out-edges."""
    return layered(4_000_000, 64, rate=3, seed=seed)


def config_layered1m(seed: int = 0) -> Graph:
    """Random layered DAG, 1,000,000 vertices in 64 layers (learned-proposal eval)."""
    return layered(1_000_000, 64, rate=3, seed=seed)
