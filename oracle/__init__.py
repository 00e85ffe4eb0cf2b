"""CPU oracle of the two-way multilevel task-DAG partition (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this package.  It wraps ``liboracle.so`` (plain serial C, built with
gcc from ``oracle.c`` and ``mpnn.c``) and shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GP_ORACLE_LIB names another build of the same sources (the sanitizer test)
_LIB_PATH = os.environ.get("GP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EASYM, EDUP, ESELF, ERANGE, EOVERFLOW, ENOMEM, EDEVICE, EMODEL = range(10)
FLAG_LEARNED = 2
FLAG_TIME = 8
FLAG_VOLUME = 16


def build(extra_flags=()) -> str:
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "mpnn.c")]
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", *extra_flags, "-o", tmp, *srcs, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.or_ratio_from_times.argtypes = [i64, i64, vp]
    lib.or_balance.argtypes = [i64, i64, i64, i32, vp, vp]
    lib.or_balance.restype = None
    lib.or_canonicalize.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
    lib.or_mix64.restype = u64
    lib.or_mix64.argtypes = [u64]
    lib.or_edge_hash.restype = u64
    lib.or_edge_hash.argtypes = [u64, i32, i32, i32]
    lib.or_match.restype = i64
    lib.or_match.argtypes = [i32, vp, vp, vp, vp, i64, u64, i32, i32, i32, vp]
    lib.or_match_twohop.restype = i64
    lib.or_match_twohop.argtypes = [i32, vp, vp, vp, vp, i64, u64, i32, vp]
    lib.or_contract.restype = i32
    lib.or_contract.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.or_volume.restype = i64
    lib.or_volume.argtypes = [i32, vp, vp, vp, vp]
    lib.or_cut.restype = i64
    lib.or_cut.argtypes = [i32, vp, vp, vp, vp]
    lib.or_refine.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
    lib.or_init_bisect.argtypes = [i32, vp, vp, vp, vp, i64, i64, vp, vp, ctypes.c_int,
                                   ctypes.c_int, vp, vp]
    lib.or_partition.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
    lib.or_mpnn_nparam.restype = i32
    lib.or_phi.restype = ctypes.c_float
    lib.or_phi.argtypes = [i64]
    lib.or_mpnn_scores.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
    lib.or_bf16_round.restype = ctypes.c_uint16
    lib.or_bf16_round.argtypes = [ctypes.c_float]
    lib.or_learned_fill.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.or_mpnn_loss_grad_f64.restype = ctypes.c_double
    lib.or_mpnn_loss_grad_f64.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _p(a):
    """Host pointer of a; the pointer object keeps a alive until the call returns."""
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class Options:
    ratio: tuple = (1, 4)       # CPU : GPU target shares (Eq. (1)-(2) in integer form)
    eps_ppm: int = 30000        # imbalance tolerance, parts per million
    balance_on: int = 0         # 0: balance the CPU-cost column, 1: the GPU-cost column
    seed: int = 0               # matching hash seed
    coarsen_to: int = 2048      # coarsen while n > coarsen_to
    match_rounds: int = 8
    refine_passes: int = 8
    init_trials: int = 16
    flags: int = 0

    def as_array(self) -> np.ndarray:
        return np.array([self.ratio[0], self.ratio[1], self.eps_ppm, self.balance_on,
                         np.int64(np.uint64(self.seed).view(np.int64)), self.coarsen_to,
                         self.match_rounds, self.refine_passes, self.init_trials, self.flags],
                        dtype=np.int64)


@dataclass
class Result:
    status: int
    part: np.ndarray
    cut: int
    load: tuple
    time: tuple
    feasible: int
    levels: int
    used_learned: int
    trace: np.ndarray
    volume: int = 0


def ratio_from_times(t_cpu: int, t_gpu: int):
    out = np.zeros(2, dtype=np.int64)
    rc = _load().or_ratio_from_times(t_cpu, t_gpu, _p(out))
    return rc, (int(out[0]), int(out[1]))


def balance(W: int, r0: int, r1: int, eps_ppm: int):
    tgt = np.zeros(2, dtype=np.int64)
    maxw = np.zeros(2, dtype=np.int64)
    _load().or_balance(W, r0, r1, eps_ppm, _p(tgt), _p(maxw))
    return tgt, maxw


def canonicalize(n, xadj, adjncy, adjwgt, vwgt):
    xadj, adjncy = _c(xadj, np.int32), _c(adjncy, np.int32)
    adjwgt, vwgt = _c(adjwgt, np.int64), _c(vwgt, np.int64)
    nnz = int(xadj[n]) if n > 0 and len(xadj) > n and xadj[n] > 0 else 0
    ox = np.zeros(n + 1, np.int32)
    oa = np.zeros(max(nnz, 1), np.int32)
    ow = np.zeros(max(nnz, 1), np.int64)
    rc = _load().or_canonicalize(n, _p(xadj), _p(adjncy), _p(adjwgt), _p(vwgt), _p(ox), _p(oa),
                                 _p(ow))
    return rc, ox, oa[:nnz], ow[:nnz]


def mix64(z: int) -> int:
    """The SplitMix64 output finaliser the matching hash is built from."""
    return int(_load().or_mix64(z & (2**64 - 1)))


def edge_hash(seed: int, level: int, a: int, b: int) -> int:
    return int(_load().or_edge_hash(seed, level, a, b))


def match(n, xadj, adjncy, adjwgt, b, cap, seed, level, rounds, twohop=True):
    """R proposal rounds, then (twohop) the two-hop pairing pass."""
    xadj, adjncy, adjwgt, b = (_c(xadj, np.int32), _c(adjncy, np.int32), _c(adjwgt, np.int64),
                               _c(b, np.int64))
    m = np.zeros(max(n, 1), np.int32)
    pairs = _load().or_match(n, _p(xadj), _p(adjncy), _p(adjwgt), _p(b), cap, seed, level,
                             rounds, int(bool(twohop)), _p(m))
    return int(pairs), m[:n]


def match_twohop(n, xadj, adjncy, adjwgt, b, cap, seed, level, matchv):
    """The two-hop pairing pass alone, applied to a given matching."""
    m = _c(matchv, np.int32).copy()
    pairs = _load().or_match_twohop(n, _p(_c(xadj, np.int32)), _p(_c(adjncy, np.int32)),
                                    _p(_c(adjwgt, np.int64)), _p(_c(b, np.int64)), cap, seed,
                                    level, _p(m))
    return int(pairs), m[:n]


def contract(n, xadj, adjncy, adjwgt, vc, vg, matchv):
    xadj, adjncy, adjwgt = _c(xadj, np.int32), _c(adjncy, np.int32), _c(adjwgt, np.int64)
    vc, vg, matchv = _c(vc, np.int64), _c(vg, np.int64), _c(matchv, np.int32)
    nnz = int(xadj[n]) if n > 0 else 0
    cmap = np.zeros(max(n, 1), np.int32)
    cx = np.zeros(n + 1, np.int32)
    ca = np.zeros(max(nnz, 1), np.int32)
    cw = np.zeros(max(nnz, 1), np.int64)
    cvc = np.zeros(max(n, 1), np.int64)
    cvg = np.zeros(max(n, 1), np.int64)
    cnnz = ctypes.c_int64(0)
    nc = _load().or_contract(n, _p(xadj), _p(adjncy), _p(adjwgt), _p(vc), _p(vg), _p(matchv),
                             _p(cmap), _p(cx), _p(ca), _p(cw), _p(cvc), _p(cvg),
                             ctypes.byref(cnnz))
    if nc < 0:
        raise MemoryError("or_contract")
    m = cnnz.value
    return nc, cmap[:n], cx[:nc + 1], ca[:m], cw[:m], cvc[:nc], cvg[:nc]


def cut(n, xadj, adjncy, adjwgt, part) -> int:
    return int(_load().or_cut(n, _p(_c(xadj, np.int32)), _p(_c(adjncy, np.int32)),
                              _p(_c(adjwgt, np.int64)), _p(_c(part, np.int8))))


def volume(graph, part) -> int:
    """Communication volume of a two-way part vector: every task's output (as
    large as its largest edge to a successor) counted once when a successor
    lies on the other side."""
    adj = _c(graph.adjncy if len(graph.adjncy) else np.zeros(1), np.int32)
    w = _c(graph.adjwgt if len(graph.adjwgt) else np.zeros(1), np.int64)
    return int(_load().or_volume(graph.n, _p(_c(graph.xadj, np.int32)), _p(adj), _p(w),
                                 _p(_c(part, np.int8))))


def refine(n, xadj, adjncy, adjwgt, b, part, pw, maxw, passes):
    part = _c(part, np.int8).copy()
    pw = _c(pw, np.int64).copy()
    maxw = _c(maxw, np.int64)
    moves = ctypes.c_int64(0)
    p = _load().or_refine(n, _p(_c(xadj, np.int32)), _p(_c(adjncy, np.int32)),
                          _p(_c(adjwgt, np.int64)), _p(_c(b, np.int64)), _p(part), _p(pw),
                          _p(maxw), passes, ctypes.byref(moves))
    return p, part, pw, moves.value


def init_bisect(n, xadj, adjncy, adjwgt, b, ratio, tgt, maxw, trials, passes):
    part = np.zeros(max(n, 1), np.int8)
    pw = np.zeros(2, np.int64)
    rc = _load().or_init_bisect(n, _p(_c(xadj, np.int32)), _p(_c(adjncy, np.int32)),
                                _p(_c(adjwgt, np.int64)), _p(_c(b, np.int64)), ratio[0],
                                ratio[1], _p(_c(tgt, np.int64)), _p(_c(maxw, np.int64)), trials,
                                passes, _p(part), _p(pw))
    return rc, part[:n], pw


def partition(graph=None, opts: Options | None = None, *, n=None, xadj=None, adjncy=None,
              adjwgt=None, vwgt=None, model=None, trace_cap: int = 64) -> Result:
    """Run the whole oracle pipeline on one graph (a ``dagen.Graph`` or raw arrays)."""
    if graph is not None:
        n, xadj, adjncy, adjwgt, vwgt = graph.n, graph.xadj, graph.adjncy, graph.adjwgt, graph.vwgt
    opts = opts or Options()
    xadj, adjncy = _c(xadj, np.int32), _c(adjncy, np.int32)
    adjwgt, vwgt = _c(adjwgt, np.int64), _c(vwgt, np.int64)
    if len(adjncy) == 0:
        adjncy = np.zeros(1, np.int32)
        adjwgt = np.zeros(1, np.int64)
    if vwgt.size == 0:
        vwgt = np.zeros(2, np.int64)
    part = np.zeros(max(n, 1), np.int8)
    res = np.zeros(9, np.int64)
    trace = np.zeros(8 * trace_cap, np.int64)
    mp = None
    if model is not None:
        mp = ctypes.c_void_p(model.ctypes.data)
    rc = _load().or_partition(n, _p(xadj), _p(adjncy), _p(adjwgt), _p(vwgt), _p(opts.as_array()),
                              mp, _p(part), _p(res), _p(trace), trace_cap)
    levels = int(res[6])
    tr = trace.reshape(trace_cap, 8)[:levels + 1].copy() if rc == OK and n > 0 else trace[:0]
    return Result(rc, part[:n].copy(), int(res[0]), (int(res[1]), int(res[2])),
                  (int(res[3]), int(res[4])), int(res[5]), levels, int(res[7]), tr, int(res[8]))


# ------------------------------------------------------------ learned part
def mpnn_nparam() -> int:
    return int(_load().or_mpnn_nparam())


def phi(x: int) -> float:
    return float(_load().or_phi(int(x)))


def mpnn_scores(g, params_bf16: np.ndarray) -> np.ndarray:
    """Exact FP32/BF16 emulation of the network's inference (float32[n])."""
    P = _c(params_bf16, np.uint16)
    assert P.size == mpnn_nparam()
    out = np.zeros(max(g.n, 1), np.float32)
    vc = _c(g.vwgt[:, 0], np.int64)
    vg = _c(g.vwgt[:, 1], np.int64)
    rc = _load().or_mpnn_scores(g.n, _p(_c(g.xadj, np.int32)), _p(_c(g.adjncy, np.int32)),
                                _p(_c(g.adjwgt, np.int64)), _p(vc), _p(vg), _p(P), _p(out))
    assert rc == 0
    return out[:g.n]


def learned_fill(g, params_bf16: np.ndarray, b, gs: int, tgt, maxw):
    """The learned proposal before refinement: (part, pw)."""
    P = _c(params_bf16, np.uint16)
    assert P.size == mpnn_nparam()
    part = np.zeros(max(g.n, 1), np.int8)
    pw = np.zeros(2, np.int64)
    rc = _load().or_learned_fill(g.n, _p(_c(g.xadj, np.int32)), _p(_c(g.adjncy, np.int32)),
                                 _p(_c(g.adjwgt, np.int64)), _p(_c(g.vwgt[:, 0], np.int64)),
                                 _p(_c(g.vwgt[:, 1], np.int64)), _p(_c(b, np.int64)), _p(P), gs,
                                 _p(_c(tgt, np.int64)), _p(_c(maxw, np.int64)), _p(part), _p(pw))
    assert rc == 0
    return part[:g.n], pw


def mpnn_loss_grad_f64(g, bw: np.ndarray, labels: np.ndarray, params: np.ndarray):
    """FP64 training objective and gradient (no rounding anywhere)."""
    P = _c(params, np.float64)
    grad = np.zeros(mpnn_nparam(), np.float64)
    vc = _c(g.vwgt[:, 0], np.int64)
    vg = _c(g.vwgt[:, 1], np.int64)
    loss = _load().or_mpnn_loss_grad_f64(g.n, _p(_c(g.xadj, np.int32)), _p(_c(g.adjncy, np.int32)),
                                         _p(_c(g.adjwgt, np.int64)), _p(vc), _p(vg),
                                         _p(_c(bw, np.int64)), _p(_c(labels, np.int8)), _p(P),
                                         _p(grad))
    return float(loss), grad


def bf16_round(f: float) -> int:
    return int(_load().or_bf16_round(float(f)))
