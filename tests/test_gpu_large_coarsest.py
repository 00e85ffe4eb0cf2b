"""Coarsest graphs above the LDS-resident size (3,072 vertices): the greedy
growing trials run in their global-memory form, in the single-graph path and
in the batched persistent kernel.  Reached by a large coarsening threshold,
by graphs that are never coarsened, and by a coarsening that stalls at
level 0 (no pair fits under the weight cap)."""
import sys

import numpy as np
import pytest

import dagen
import oracle
from helpers import random_graph

pytestmark = pytest.mark.gpu

LDS_MAX = 3072


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def coarsest_n(ref):
    return int(np.asarray(ref.trace)[-1][0]) if len(ref.trace) else None


def run_single(gp, g, **kw):
    say(f"case single {g.name} n={g.n} opts={kw}")
    ref = oracle.partition(g, oracle.Options(**kw))
    assert ref.status == 0
    h = gp.create(g)
    part, res = h.partition(gp.options(**kw))
    got = part.cpu().numpy()
    h.close()
    assert res.levels == ref.levels
    assert np.array_equal(got, ref.part), f"{int((got != ref.part).sum())} vertices differ"
    assert res.cut == ref.cut and (res.load[0], res.load[1]) == ref.load
    assert (res.time[0], res.time[1]) == ref.time and res.feasible == ref.feasible
    return ref


def stalled_graph(n, seed):
    """Balance weights 10, a few 20: with coarsen_to = 0.8 n the cap
    ceil(3W/(2C)) is 19, so no pair fits (every pair weighs >= 20), the
    matching stalls at level 0 and the kept level 1 equals level 0."""
    rng = np.random.default_rng(seed)
    g = random_graph(n, 6.0 / n, rng, wmax=1000, vmax=1, name=f"stall{n}")
    vw = np.full((n, 2), 10, np.int64)
    vw[rng.choice(n, n // 100, replace=False)] = 20
    g.vwgt = vw
    return g


@pytest.mark.parametrize("which,C", [(0, 6000), (0, 16000), (1, 6000), (1, 16000)],
                         ids=["chol64-6000", "chol64-16000", "lu48-6000", "lu48-16000"])
def test_large_coarsest_cholesky_lu(gp, which, C):
    g = dagen.config_cholesky64_lu48()[which]
    ref = run_single(gp, g, ratio=(1, 4), eps_ppm=30000, coarsen_to=C)
    assert coarsest_n(ref) > LDS_MAX


@pytest.mark.parametrize("kw", [dict(init_trials=3), dict(init_trials=16, balance_on=1,
                                                          ratio=(2, 5)),
                                dict(init_trials=7, eps_ppm=0, refine_passes=2)],
                         ids=["K3", "K16-gpu-col", "K7-eps0"])
def test_uncoarsened_layered(gp, kw):
    g = dagen.layered(5003, 12, rate=4, seed=17)
    ref = run_single(gp, g, coarsen_to=8192, **kw)
    assert ref.levels == 0


def test_stalled_coarsening(gp):
    g = stalled_graph(5000, 3)
    ref = run_single(gp, g, coarsen_to=4000)
    assert ref.levels == 1 and coarsest_n(ref) == 5000


@pytest.mark.parametrize("C,min_big", [(8192, 4), (2800, 1)], ids=["C8192", "C2800-stall"])
def test_batch_large_coarsest(gp, C, min_big):
    """The batched kernel on graphs whose coarsest level exceeds the LDS form
    (never coarsened, or stalled at level 0), mixed with small and coarsened
    ones, each against the oracle."""
    import torch
    graphs = [dagen.layered(4100, 10, rate=4, seed=1), dagen.cholesky(30, 512, jitter_pm=100,
                                                                       seed=2),
              dagen.layered(300, 4, rate=3, seed=3), dagen.lu(28, 512, jitter_pm=100, seed=4),
              stalled_graph(3500, 5), dagen.layered(6000, 20, rate=3, seed=6)]
    kw = dict(ratio=(1, 4), eps_ppm=30000, coarsen_to=C)
    b = dagen.concat(graphs)
    dev = gp.batch_to_device(b)
    bt = gp.Batch()
    say(f"case batch large coarsest C={C}")
    part, res = bt.partition(*dev, opts=gp.options(**kw))
    torch.cuda.synchronize()
    got = part.cpu().numpy()
    bt.close()
    big = 0
    for i, g in enumerate(graphs):
        ref = oracle.partition(g, oracle.Options(**kw))
        assert ref.status == 0 and res[i].status == 0
        big += coarsest_n(ref) > LDS_MAX
        p = got[b.voff[i]:b.voff[i + 1]]
        assert np.array_equal(p, ref.part), f"graph {i} ({g.name}): assignment differs"
        assert res[i].cut == ref.cut and (res[i].load[0], res[i].load[1]) == ref.load
        assert res[i].levels == ref.levels and res[i].feasible == ref.feasible
    assert big >= min_big
