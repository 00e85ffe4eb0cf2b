"""Schedule simulator: the oracle pinned by hand-worked schedules, and the
library's host routine (gp_simulate) against the oracle, task by task."""
import numpy as np
import pytest

import dagen
import oracle
from oracle.sim import DMDA, EAGER, GP, simulate


def chain3():
    """a -> b -> c, CPU cost 10 and GPU cost 2 each, 8 bytes per dependency."""
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    vw = np.array([[10, 2]] * 3, np.int64)
    return dagen.to_csr(3, src, dst, np.array([8, 8], np.int64), vw, "chain3")


def test_chain_by_hand():
    """One CPU and one GPU worker, transfers of 8 bytes at 8 bytes per unit
    plus latency 1 = 2 units.
    eager: a -> GPU (tie, GPU first) [0, 2]; b -> CPU (free at 0), a's output
    crosses at 2, arrives 4, b runs [4, 14]; c -> GPU (free at 2), b's output
    crosses at 14, arrives 16, c runs [16, 18]: makespan 18, 2 transfers.
    dmda: a finishes at 2 on the GPU (10 on the CPU); b at 4 on the GPU (14
    on the CPU after the transfer); c at 6: makespan 6, no transfer.
    gp with parts (CPU, GPU, CPU): a [0, 10]; a's output arrives on the GPU
    at 12, b [12, 14]; b's output arrives on the CPU at 16, c [16, 26]."""
    g = chain3()
    r = simulate(g, EAGER, ncpu=1, ngpu=1, latency=1, bw=8)
    assert (r.makespan, r.transfers, r.bytes) == (18, 2, 16)
    assert r.node == [1, 0, 1] and r.finish == [2, 14, 18]
    r = simulate(g, DMDA, ncpu=1, ngpu=1, latency=1, bw=8)
    assert (r.makespan, r.transfers) == (6, 0) and r.node == [1, 1, 1]
    r = simulate(g, GP, part=[1, 1, 1], ncpu=1, ngpu=1, latency=1, bw=8)
    assert (r.makespan, r.transfers) == (6, 0)
    r = simulate(g, GP, part=[0, 1, 0], ncpu=1, ngpu=1, latency=1, bw=8)
    assert (r.makespan, r.transfers, r.finish) == (26, 2, [10, 14, 26])
    assert r.busy == (20, 2) and r.tasks == (2, 1)


def test_shared_output_crosses_once():
    """a feeds b and c, both pinned to the GPU while a runs on the CPU: one
    transfer of a's output serves both (the second consumer reuses it)."""
    src = np.array([0, 0], np.int32)
    dst = np.array([1, 2], np.int32)
    vw = np.array([[4, 4], [3, 3], [5, 5]], np.int64)
    g = dagen.to_csr(3, src, dst, np.array([6, 6], np.int64), vw, "fan")
    r = simulate(g, GP, part=[0, 1, 1], ncpu=1, ngpu=1, latency=0, bw=2)
    # a [0, 4]; transfer [4, 7]; b [7, 10]; c waits for the GPU: [10, 15]
    assert (r.transfers, r.bytes, r.makespan) == (1, 6, 15)
    assert r.finish == [4, 10, 15]


def test_idle_cpu_when_the_gap_is_large():
    """Matrix-multiply-like costs (CPU 50 times slower): dmda places all but one
    task of a 56-task tiled Cholesky DAG on the GPU and ends within 1 % of
    putting everything there (R_CPU close to 0, the paper's observation for
    its MM kernels); eager hands tasks to idle CPU workers and ends 8 times
    later.  With a gap of 4 the CPU workers are worth using: dmda keeps a
    third of the tasks there and beats the all-GPU schedule."""
    g = dagen.cholesky(6, 64, rate=50)
    e = simulate(g, EAGER, ncpu=3, ngpu=1, latency=10, bw=1 << 20)
    d = simulate(g, DMDA, ncpu=3, ngpu=1, latency=10, bw=1 << 20)
    gp = simulate(g, GP, part=[1] * g.n, ncpu=3, ngpu=1, latency=10, bw=1 << 20)
    assert d.tasks[0] <= 1 and d.makespan <= gp.makespan * 1.01
    assert e.tasks[0] > 10 and e.makespan > 5 * d.makespan
    g4 = dagen.cholesky(6, 64, rate=4)
    d4 = simulate(g4, DMDA, ncpu=3, ngpu=1, latency=10, bw=1 << 20)
    gp4 = simulate(g4, GP, part=[1] * g4.n, ncpu=3, ngpu=1, latency=10, bw=1 << 20)
    assert d4.tasks[0] > 10 and d4.makespan < gp4.makespan


def lib():
    pytest.importorskip("torch")
    import paper_1502_07451_amd as gp
    return gp


@pytest.mark.parametrize("which", ["chol", "lu", "layered", "random"])
def test_library_matches_oracle(which):
    gpm = lib()
    rng = np.random.default_rng(len(which))
    if which == "chol":
        g = dagen.cholesky(10, 256, jitter_pm=100, seed=1)
    elif which == "lu":
        g = dagen.lu(9, 256, jitter_pm=100, seed=2)
    elif which == "layered":
        g = dagen.layered(3000, 20, rate=3, seed=3)
    else:
        from helpers import random_graph
        g = random_graph(300, 0.02, rng, wmax=10**6, vmax=1000)
    part = rng.integers(0, 2, g.n).astype(np.int8)
    for policy in (EAGER, DMDA, GP):
        for ncpu, ngpu, lat, bw in ((3, 1, 0, 1), (1, 2, 7, 1 << 20), (4, 1, 100, 3)):
            ref = simulate(g, policy, part=part, ncpu=ncpu, ngpu=ngpu, latency=lat, bw=bw)
            res, node, fin = gpm.simulate(g, policy, part=part, ncpu=ncpu, ngpu=ngpu,
                                          latency=lat, bw=bw)
            assert (res.makespan, res.transfers, res.bytes) == (ref.makespan, ref.transfers,
                                                                ref.bytes)
            assert tuple(res.busy) == ref.busy and tuple(res.tasks) == ref.tasks
            assert node.tolist() == ref.node and fin.tolist() == ref.finish


def test_library_rejects_bad_input():
    gpm = lib()
    g = chain3()
    with pytest.raises(gpm.GPError):
        gpm.simulate(g, GP)                       # gp needs a partition
    with pytest.raises(gpm.GPError):
        gpm.simulate(g, EAGER, ncpu=0, ngpu=0)    # no worker
    with pytest.raises(gpm.GPError):
        gpm.simulate(g, GP, part=[0, 0, 0], ncpu=0, ngpu=1)


@pytest.mark.parametrize("T,rate", [(10, 4), (12, 4), (10, 50), (12, 50)])
def test_partition_moves_least_data(T, rate):
    """The paper's runtime comparison (Section IV-C): the graph-partition
    policy moves the least data.  Tiled Cholesky on 3 CPU workers and one GPU
    worker, shares from Eq. (1) with the CPU node's time taken as its summed
    task time over its three workers; the oracle's partition pins the tasks."""
    g = dagen.cholesky(T, 512, rate=rate)
    tc, tg = int(g.vwgt[:, 0].sum()) // 3, int(g.vwgt[:, 1].sum())
    rc, ratio = oracle.ratio_from_times(tc, tg)
    assert rc == 0
    part = oracle.partition(g, oracle.Options(ratio=ratio, eps_ppm=30000)).part
    e, d, p = (simulate(g, pol, part=part, ncpu=3, ngpu=1, latency=0, bw=1)
               for pol in (EAGER, DMDA, GP))
    assert p.transfers < min(e.transfers, d.transfers)
    assert p.bytes < min(e.bytes, d.bytes)
