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


if __name__ == "__main__":
    main()
