"""Runs the library's host-side schedule simulator (gp_simulate), loaded from
the shared object named on the command line, over a fixed set of DAGs and
policies, and prints the results as one JSON object."""
import ctypes
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import dagen  # noqa: E402


class SimRes(ctypes.Structure):
    _fields_ = [("makespan", ctypes.c_int64), ("transfers", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("busy", ctypes.c_int64 * 2),
                ("tasks", ctypes.c_int64 * 2)]


def cases():
    """(graph, policy, part, ncpu, ngpu, latency, bw) - shared with the test."""
    out = []
    graphs = [dagen.cholesky(8, 512, jitter_pm=100, seed=1), dagen.lu(6, 512, seed=2),
              dagen.layered(3000, 10, rate=3, seed=3)]
    for gi, g in enumerate(graphs):
        rng = np.random.default_rng(gi)
        part = rng.integers(0, 2, g.n).astype(np.int8)
        for pol in (0, 1, 2):
            out.append((g, pol, part if pol == 2 else None, 3, 1, 5, 1000))
            out.append((g, pol, part if pol == 2 else None, 1, 2, 0, 1))
    return out


def main(lib_path):
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.gp_simulate.argtypes = [i32, vp, vp, vp, vp, vp, i32, i32, i32, i64, i64,
                                ctypes.POINTER(SimRes), vp, vp]
    lib.gp_simulate.restype = ctypes.c_int
    res = []
    for g, pol, part, ncpu, ngpu, lat, bw in cases():
        xadj = np.ascontiguousarray(g.xadj, np.int32)
        adj = np.ascontiguousarray(g.adjncy, np.int32)
        w = np.ascontiguousarray(g.adjwgt, np.int64)
        vw = np.ascontiguousarray(g.vwgt, np.int64)
        node = np.zeros(g.n, np.int8)
        fin = np.zeros(g.n, np.int64)
        r = SimRes()
        pp = None if part is None else np.ascontiguousarray(part, np.int8)
        st = lib.gp_simulate(g.n, xadj.ctypes.data, adj.ctypes.data, w.ctypes.data,
                             vw.ctypes.data, None if pp is None else pp.ctypes.data, pol, ncpu,
                             ngpu, lat, bw, ctypes.byref(r), node.ctypes.data, fin.ctypes.data)
        res.append([st, r.makespan, r.transfers, r.bytes, list(r.busy), list(r.tasks),
                    node.tolist(), fin.tolist()])
    print(json.dumps(res))


if __name__ == "__main__":
    main(sys.argv[1])
