"""Communication volume (GP_VOLUME): every task's output counted once per
memory node that needs it.  Pinned by hand-worked cases and by the schedule
simulator, which moves exactly the volume's bytes under the partition."""
import numpy as np
import pytest

import dagen
import oracle
from oracle.sim import GP, simulate
from helpers import random_graph


def dag(n, edges):
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    w = np.array([e[2] for e in edges], np.int64)
    return dagen.to_csr(n, src, dst, w, np.ones((n, 2), np.int64), "dag")


def test_volume_counts_an_output_once_per_node():
    """Task 0 feeds 1, 2 and 3 (edges 5, 7, 3 bytes): its output is 7 bytes;
    with 0 on the CPU and 1-3 on the GPU it crosses once (7), not three
    times (the cut, 15).  Task 1 feeds 4 (2 bytes) on the CPU: 2 more."""
    g = dag(5, [(0, 1, 5), (0, 2, 7), (0, 3, 3), (1, 4, 2)])
    part = np.array([0, 1, 1, 1, 0], np.int8)
    assert oracle.volume(g, part) == 7 + 2
    assert oracle.cut(g.n, g.xadj, g.adjncy, g.adjwgt, part) == 15 + 2
    assert oracle.volume(g, np.zeros(5, np.int8)) == 0


def test_volume_pass_trades_cut_for_volume():
    """Edges 0->3 (2 bytes), 1->2 (8), 1->3 (1); unit weights, ratio 1:1,
    eps 20 % (bounds 3 and 3).  The edge-cut partition is parts (0, 1, 1, 0):
    cut 1 (edge 1-3), but task 1's 8-byte output crosses for task 3: volume
    8.  First volume pass (side 0): task 3's gain is +8 (task 1 on the other
    side has 3 as its only successor there) - 2 (task 0 on its side would
    start to cross) = 6 > 0, task 0's is -2: task 3 moves (side 1 has room
    1).  The next passes find no positive gain that fits: parts (0, 1, 1, 1),
    cut 2, volume 2."""
    g = dag(4, [(0, 3, 2), (1, 2, 8), (1, 3, 1)])
    kw = dict(ratio=(1, 1), eps_ppm=200000)
    plain = oracle.partition(g, oracle.Options(**kw))
    assert plain.part.tolist() == [0, 1, 1, 0] and plain.cut == 1
    assert oracle.volume(g, plain.part) == 8 and plain.volume == 0
    r = oracle.partition(g, oracle.Options(**kw, flags=oracle.FLAG_VOLUME))
    assert r.part.tolist() == [0, 1, 1, 1]
    assert r.cut == 2 and r.volume == 2 and r.load == (1, 3) and r.feasible == 1


@pytest.mark.parametrize("seed", range(6))
def test_volume_equals_simulated_transfers(seed):
    """The simulator, written separately, moves each producer's output once to
    the other node: under the partition's placement its byte count is the
    volume."""
    rng = np.random.default_rng(seed)
    if seed % 2:
        g = dagen.layered(int(rng.integers(200, 4000)), int(rng.integers(3, 12)), rate=3,
                          seed=seed)
    else:
        g = random_graph(int(rng.integers(5, 300)), 0.05, rng, wmax=1000, vmax=20)
    r = oracle.partition(g, oracle.Options(ratio=(1, 2), flags=oracle.FLAG_VOLUME,
                                           coarsen_to=int(rng.choice([16, 2048]))))
    assert r.status == 0 and r.volume == oracle.volume(g, r.part)
    s = simulate(g, GP, part=r.part, ncpu=2, ngpu=1)
    assert s.bytes == r.volume


def test_volume_rejects_other_modes():
    g = dagen.config_cholesky8()
    model = np.zeros(oracle.mpnn_nparam(), np.uint16)
    for f in (oracle.FLAG_TIME, oracle.FLAG_LEARNED):
        r = oracle.partition(g, oracle.Options(flags=oracle.FLAG_VOLUME | f), model=model)
        assert r.status == oracle.EINVAL
