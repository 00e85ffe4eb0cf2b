"""Writes the stored expected values under tests/golden/.

Inputs come from the seeded generators (dagen); expected partition results come
from the CPU oracle only.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import dagen  # noqa: E402
import oracle  # noqa: E402


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    g = dagen.config_cholesky8()
    with open(os.path.join(HERE, "cholesky8.sha256"), "w") as f:
        f.write(digest(g.xadj, g.adjncy, g.adjwgt, g.vwgt)
                + "  Cholesky T=8, b=512, rate 4, 2 MiB edges: xadj|adjncy|adjwgt|vwgt"
                  " (written by tests/golden/make_golden.py)\n")

    # 4,000,000-vertex layered DAG, CPU:GPU 1:3, eps 5 %, default options
    g = dagen.config_layered4m()
    r = oracle.partition(g, oracle.Options(ratio=(1, 3), eps_ppm=50000))
    assert r.status == 0
    with open(os.path.join(HERE, "layered4m_1to3_eps5.txt"), "w") as f:
        f.write("# oracle result for dagen.config_layered4m(), ratio 1:3, eps_ppm 50000,\n"
                "# seed 0, coarsen_to 2048, 8 rounds, 8 passes, 16 trials\n"
                "# (written by tests/golden/make_golden.py from the CPU oracle)\n")
        f.write(f"part_sha256={hashlib.sha256(r.part.tobytes()).hexdigest()}\n")
        f.write(f"cut={r.cut}\nload0={r.load[0]}\nload1={r.load[1]}\n")
        f.write(f"time0={r.time[0]}\ntime1={r.time[1]}\nfeasible={r.feasible}\n")
        f.write(f"levels={r.levels}\n")


if __name__ == "__main__":
    main()
