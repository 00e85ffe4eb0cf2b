"""Batched persistent-kernel path vs the CPU oracle, graph by graph.

Each graph's result from gp_partition_batch must equal the oracle's result
for that graph alone (and so the single-graph path's), whatever the queue
order, chunking or number of workgroups.
"""
import sys

import numpy as np
import pytest

import dagen
import oracle
from helpers import complete_graph, edgeless_graph, path_graph, random_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_graphs(seed: int, count: int):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = i % 6
        if k == 0:
            g = random_graph(int(rng.integers(1, 300)), float(rng.uniform(0.01, 0.2)), rng,
                             wmax=int(rng.choice([1, 9, 1000])), vmax=9, const_w=bool(i % 4 == 0))
        elif k == 1:
            g = dagen.cholesky(int(rng.integers(2, 14)), 256, jitter_pm=100, seed=i)
        elif k == 2:
            g = dagen.layered(int(rng.integers(100, 6000)), int(rng.integers(2, 20)), rate=4,
                              seed=i)
        elif k == 3:
            g = dagen.lu(int(rng.integers(2, 12)), 256, jitter_pm=50, seed=i)
        elif k == 4:
            g = path_graph(int(rng.integers(1, 500)))
        else:
            m = int(rng.integers(0, 40))
            g = edgeless_graph(m, rng.integers(1, 5, m))
        out.append(g)
    return out


def run_batch(gp, graphs, opts_kw, config=None):
    import torch
    b = dagen.concat(graphs)
    dev = gp.batch_to_device(b)
    bt = gp.Batch()
    if config:
        bt.config(*config)
    part, res = bt.partition(*dev, opts=gp.options(**opts_kw))
    torch.cuda.synchronize()
    got = part.cpu().numpy()
    bt.close()
    return b, got, res


def check_against_oracle(b, graphs, got, res, opts_kw, which=None):
    oo = oracle.Options(**opts_kw)
    idx = range(len(graphs)) if which is None else which
    for g in idx:
        gr = graphs[g]
        ref = oracle.partition(gr, oo)
        r = res[g]
        assert r.status == ref.status, f"graph {g}: status {r.status} vs {ref.status}"
        if ref.status != 0:
            continue
        p = got[b.voff[g]:b.voff[g + 1]]
        assert np.array_equal(p, ref.part), f"graph {g} ({gr.name}, n={gr.n}): assignment differs"
        assert r.cut == ref.cut and (r.load[0], r.load[1]) == ref.load, f"graph {g}"
        assert (r.time[0], r.time[1]) == ref.time and r.feasible == ref.feasible, f"graph {g}"
        assert r.levels == ref.levels, f"graph {g}"


@pytest.mark.parametrize("kw", [dict(), dict(coarsen_to=16, ratio=(1, 1)),
                                dict(coarsen_to=64, balance_on=1, ratio=(2, 5), eps_ppm=0,
                                     match_rounds=2, refine_passes=3, init_trials=5)],
                         ids=["default", "deep", "odd"])
def test_batch_mixed_matches_oracle(gp, kw):
    graphs = mixed_graphs(11, 48)
    say(f"case batch mixed {kw}")
    b, got, res = run_batch(gp, graphs, kw)
    check_against_oracle(b, graphs, got, res, kw)


def test_batch_config_independent(gp):
    graphs = mixed_graphs(5, 40)
    kw = dict(coarsen_to=32)
    say("case batch config A")
    b, got1, res1 = run_batch(gp, graphs, kw)
    say("case batch config B")
    _, got2, res2 = run_batch(gp, graphs, kw, config=(7, 3, 1))
    say("case batch config C")
    _, got3, res3 = run_batch(gp, graphs, kw, config=(1, 64, 0))
    assert np.array_equal(got1, got2) and np.array_equal(got1, got3)
    for a, c, d in zip(res1, res2, res3):
        assert a.as_dict() == c.as_dict() == d.as_dict()


def test_batch_errors_per_graph(gp):
    good = path_graph(30)
    bad = path_graph(5)
    bad.adjncy = bad.adjncy.copy()
    bad.adjncy[1] = 1   # self loop in row 1
    asym = path_graph(6)
    asym.adjwgt = asym.adjwgt.copy()
    asym.adjwgt[0] = 7
    graphs = [good, bad, asym, complete_graph(12)]
    say("case batch errors")
    b, got, res = run_batch(gp, graphs, {})
    assert [r.status for r in res] == [0, oracle.ESELF, oracle.EASYM, 0]
    check_against_oracle(b, graphs, got, res, {}, which=[0, 3])


def test_batch_uneven_sizes(gp):
    # log-uniform sizes from the batch recipe, a reduced count
    size, kind, param, gseed = dagen.batch_plan(96, 100, 50000, 7)
    graphs = []
    for i in range(96):
        if kind[i] == 0:
            graphs.append(dagen.cholesky(int(param[i]), 512, 0, 4, dagen.TILE_512_BYTES,
                                         int(gseed[i])))
        else:
            graphs.append(dagen.layered(int(size[i]), int(param[i]), rate=4, seed=int(gseed[i])))
    kw = dict(ratio=(1, 4), eps_ppm=30000)
    say("case batch uneven 96")
    b, got, res = run_batch(gp, graphs, kw)
    check_against_oracle(b, graphs, got, res, kw)


def test_batch_full_4096(gp):
    """The 4,096-graph batch at full size (sizes 100..50,000, half Cholesky,
    half layered), as the benchmark runs it: every graph's assignment, cut,
    loads, times, feasibility and level count against the oracle (run over
    the graphs on a host thread pool), and the largest graphs also through
    the single-graph GPU path."""
    import concurrent.futures
    import os
    graphs = dagen.batch(4096, 100, 50000, 0)
    kw = dict(ratio=(1, 4), eps_ppm=30000)
    say("case batch full 4096")
    b, got, res = run_batch(gp, graphs, kw)
    assert all(r.status == 0 for r in res)
    oo = oracle.Options(**kw)
    with concurrent.futures.ThreadPoolExecutor(min(os.cpu_count() or 1, 16)) as ex:
        refs = list(ex.map(lambda g: oracle.partition(g, oo), graphs))
    bad = []
    for i, (ref, r) in enumerate(zip(refs, res)):
        p = got[b.voff[i]:b.voff[i + 1]]
        if not (ref.status == 0 and np.array_equal(p, ref.part) and r.cut == ref.cut and
                (r.load[0], r.load[1]) == ref.load and (r.time[0], r.time[1]) == ref.time and
                r.feasible == ref.feasible and r.levels == ref.levels):
            bad.append(i)
    assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:8]}"
    sizes = np.diff(b.voff)
    for g in np.argsort(-sizes)[:6].tolist():
        h = gp.create(graphs[g])
        p, r = h.partition(gp.options(**kw))
        h.close()
        assert np.array_equal(p.cpu().numpy(), got[b.voff[g]:b.voff[g + 1]])
        assert r.cut == res[g].cut


def test_batch_autotune_keeps_results(gp):
    """Every autotuner configuration must give the same bytes; the chosen
    one is then used by later calls and still matches the oracle."""
    graphs = mixed_graphs(23, 60)
    kw = dict(coarsen_to=64)
    bb = dagen.concat(graphs)
    dev = gp.batch_to_device(bb)
    bt = gp.Batch()
    say("case batch autotune")
    part, res, chosen, ms = bt.autotune(*dev, opts=gp.options(**kw), reps=1)
    say(f"chosen {chosen} {ms:.3f} ms")
    assert chosen[1] in (1, 2, 4) and chosen[2] in (0, 1, 2) and -4 <= chosen[3] <= 1
    assert chosen[0] > 0 and ms > 0
    got = part.cpu().numpy()
    check_against_oracle(bb, graphs, got, res, kw)
    part2, res2 = bt.partition(*dev, opts=gp.options(**kw))
    assert np.array_equal(part2.cpu().numpy(), got)
    assert [r.as_dict() for r in res2] == [r.as_dict() for r in res]
    bt.close()


def test_batch_timeline(gp):
    """gp_batch_timeline: every graph of the last call has a start and an end
    on the device clock, in order; asking for more graphs than it ran is
    refused."""
    graphs = [dagen.layered(int(n), 6, rate=3, seed=i)
              for i, n in enumerate(np.linspace(200, 5000, 24).astype(int))]
    bb = dagen.concat(graphs)
    say("case batch timeline 24")
    b = gp.Batch()
    _, res = b.partition(*gp.batch_to_device(bb))
    assert all(r.status == 0 for r in res)
    t, hz = b.timeline(len(graphs))
    assert hz > 0 and t.shape == (len(graphs), 2)
    assert (t[:, 0] > 0).all() and (t[:, 1] >= t[:, 0]).all()
    with pytest.raises(gp.GPError) as e:
        b.timeline(len(graphs) + 1)
    assert e.value.status == gp.EINVAL
    b.close()


def test_batch_order_by_previous_times(gp):
    """Order mode 2 (the previous call's slowest graphs first) on the same
    context: the same bytes as largest-first, on the first call (no timeline
    yet) and the second (ordered by the first call's times)."""
    import torch
    graphs = mixed_graphs(9, 48)
    kw = dict(coarsen_to=64)
    bb = dagen.concat(graphs)
    dev = gp.batch_to_device(bb)
    say("case batch order mode 2")
    ref = gp.Batch()
    p0, r0 = ref.partition(*dev, opts=gp.options(**kw))
    want = p0.cpu().numpy()
    ref.close()
    b = gp.Batch()
    b.config(0, 1, 2)
    for _ in range(2):
        p, r = b.partition(*dev, opts=gp.options(**kw))
        torch.cuda.synchronize()
        assert np.array_equal(p.cpu().numpy(), want)
        assert [x.as_dict() for x in r] == [x.as_dict() for x in r0]
    b.close()


@pytest.mark.parametrize("shift", [-4, -2, -1, 1])
def test_batch_team_width_keeps_results(gp, shift):
    """gp_batch_team_width changes the lanes per row, never a result."""
    import torch
    graphs = mixed_graphs(31, 40)
    kw = dict(coarsen_to=48)
    bb = dagen.concat(graphs)
    dev = gp.batch_to_device(bb)
    say(f"case batch team width {shift}")
    ref = gp.Batch()
    p0, r0 = ref.partition(*dev, opts=gp.options(**kw))
    want = p0.cpu().numpy()
    ref.close()
    b = gp.Batch()
    b.team_width(shift)
    p, r = b.partition(*dev, opts=gp.options(**kw))
    torch.cuda.synchronize()
    assert np.array_equal(p.cpu().numpy(), want)
    assert [x.as_dict() for x in r] == [x.as_dict() for x in r0]
    with pytest.raises(gp.GPError):
        b.team_width(2)
    b.close()
