"""A mixed oracle workload whose results are printed as one JSON object; the
sanitizer test runs it against the plain and the sanitized oracle build."""
import hashlib
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import dagen  # noqa: E402
import oracle  # noqa: E402
from helpers import edgeless_graph, path_graph, random_graph  # noqa: E402
from oracle.kway import partition_kway  # noqa: E402


def dig(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def main():
    rng = np.random.default_rng(11)
    params = (rng.standard_normal(oracle.mpnn_nparam()) * 0.2).astype(np.float32)
    model = np.array([oracle.bf16_round(float(x)) for x in params], np.uint16)
    graphs = [dagen.cholesky(10, 512, jitter_pm=100, seed=1), dagen.lu(8, 512, seed=2),
              dagen.layered(6000, 12, rate=3, seed=3),
              random_graph(300, 0.05, rng, wmax=1000, vmax=50),
              random_graph(40, 0.3, rng, wmax=10**9, vmax=10**6), path_graph(7),
              edgeless_graph(5, np.ones((5, 2), np.int64))]
    out = {}
    for i, g in enumerate(graphs):
        W = (int(g.vwgt[:, 1].sum()), int(g.vwgt[:, 0].sum()))
        while max(W) >= 1 << 40:
            W = (W[0] // 2, W[1] // 2)
        runs = [("plain", oracle.Options(ratio=(1, 3)), None),
                ("coarse16", oracle.Options(ratio=(2, 3), coarsen_to=16, eps_ppm=0), None),
                ("volume", oracle.Options(flags=oracle.FLAG_VOLUME, coarsen_to=64), None),
                ("time", oracle.Options(ratio=W, flags=oracle.FLAG_TIME, coarsen_to=64), None),
                ("learned", oracle.Options(flags=oracle.FLAG_LEARNED, coarsen_to=128), model)]
        for name, o, m in runs:
            r = oracle.partition(g, o, model=m)
            out[f"{i}-{name}"] = [r.status, r.cut, r.volume, list(r.load), r.levels,
                                  r.used_learned, dig(r.part), dig(np.asarray(r.trace))]
        k = partition_kway(g, 3, (1, 2, 3), oracle.Options(coarsen_to=64))
        out[f"{i}-kway"] = [k.status, k.cut, list(k.load), dig(k.part)]
        if g.n:
            out[f"{i}-scores"] = dig(oracle.mpnn_scores(g, model))
            y = (rng.random(g.n) < 0.5).astype(np.int8)
            bw = np.ones(g.n, np.int64)
            loss, grad = oracle.mpnn_loss_grad_f64(g, bw, y, params.astype(np.float64))
            out[f"{i}-loss"] = [round(float(loss), 9), dig(np.round(grad, 9))]
    print(json.dumps(out, sort_keys=True))


if __name__ == "__main__":
    main()
