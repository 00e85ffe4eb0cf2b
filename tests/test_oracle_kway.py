"""Pins of the k-way oracle (recursive bisection of part ranges).

The split rule, the recursion's labels and the shares per bisection are
worked out by hand on a path and on three cliques; k = 1 and k = 2 reduce
to the trivial partition and to the two-way oracle; brute force over all
3^n assignments of tiny graphs bounds the heuristic's cut from below.
"""
import itertools

import numpy as np
import pytest

import dagen
import oracle
from oracle.kway import induced, partition_kway
from helpers import path_graph, random_graph


def kcut(g, part):
    deg = np.diff(g.xadj.astype(np.int64))
    rows = np.repeat(np.arange(g.n), deg)
    return int(g.adjwgt[part[rows] != part[g.adjncy]].sum()) // 2


def test_path_split_rule():
    """Path of 9 unit vertices, shares 1:1:1.  The first bisection splits
    [0, 3) into [0, 1) and [1, 3) at ratio 1:2: side 0 is grown (the smaller
    share), trial 0 seeds vertex 0 and takes the prefix {0, 1, 2} (tgt_0 =
    3, cut 1); the rest, the path 3..8, is split 1:1 into {3, 4, 5} and
    {6, 7, 8}.  Splitting the other way round ([0, 2) and [2, 3)) would put
    the prefix in part 2."""
    r = partition_kway(path_graph(9), 3, (1, 1, 1))
    assert r.status == 0 and r.bisections == 2 and r.feasible == 1
    assert r.part.tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    assert r.cut == 2 and r.load == (3, 3, 3)


def three_cliques():
    """Cliques of 2, 4 and 6 unit vertices (ids 0-1, 2-5, 6-11), internal
    edges 100, one edge of weight 1 between each pair of cliques."""
    groups = [range(0, 2), range(2, 6), range(6, 12)]
    edges = [(a, b, 100) for grp in groups for a, b in itertools.combinations(grp, 2)]
    edges += [(1, 2, 1), (5, 6, 1), (0, 11, 1)]
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    w = np.array([e[2] for e in edges], np.int64)
    return dagen.to_csr(12, src, dst, w, np.ones((12, 2), np.int64), "cliques")


def test_three_cliques_follow_the_shares():
    """Shares 1:2:3 on the 2-, 4- and 6-cliques: the first bisection (1:5)
    grows side 0 from vertex 0 to tgt_0 = 2, the 2-clique; the second (2:3)
    grows the 4-clique from its first vertex.  Every part is one clique and
    the cut is the three bridges."""
    r = partition_kway(three_cliques(), 3, (1, 2, 3), oracle.Options(eps_ppm=0))
    assert r.part.tolist() == [0] * 2 + [1] * 4 + [2] * 6
    assert r.cut == 3 and r.load == (2, 4, 6) and r.feasible == 1


def test_k1_and_zero_shares():
    g = dagen.config_cholesky8()
    r = partition_kway(g, 1, (5,))
    assert r.status == 0 and not r.part.any() and r.cut == 0 and r.bisections == 0
    # [0] gets no share: the first bisection puts everything on [1, 3)
    r = partition_kway(g, 3, (0, 1, 1))
    assert (r.part != 0).all() and r.load[0] == 0
    # [1] gets no share inside [1, 3)
    r = partition_kway(g, 3, (1, 0, 1))
    assert (r.part != 1).all() and r.load[1] == 0
    assert partition_kway(g, 2, (0, 0)).status == oracle.EINVAL
    assert partition_kway(g, 2, (1, -1)).status == oracle.EINVAL


@pytest.mark.parametrize("seed", range(6))
def test_k2_is_the_two_way_partition(seed):
    rng = np.random.default_rng(seed)
    g = random_graph(int(rng.integers(2, 300)), 0.05, rng, wmax=50, vmax=9)
    ratio = (int(rng.integers(1, 5)), int(rng.integers(1, 5)))
    opts = oracle.Options(coarsen_to=int(rng.choice([8, 64, 2048])), balance_on=seed % 2)
    two = oracle.partition(g, oracle.Options(**{**opts.__dict__, "ratio": ratio}))
    r = partition_kway(g, 2, ratio, opts)
    assert np.array_equal(r.part, two.part.astype(np.int32))
    assert r.cut == two.cut and r.load == two.load and r.feasible == two.feasible


def test_induced_subgraph():
    """The subgraph of the odd vertices of a path is edgeless; of the first
    four, the path of four; renumbering keeps ascending ids."""
    g = path_graph(8)
    ns, sx, sa, sw, sv = induced(g.n, g.xadj, g.adjncy, g.adjwgt, g.vwgt, np.arange(8) % 2 == 1)
    assert ns == 4 and sx.tolist() == [0] * 5
    ns, sx, sa, sw, sv = induced(g.n, g.xadj, g.adjncy, g.adjwgt, g.vwgt, np.arange(8) < 4)
    assert ns == 4 and sx.tolist() == [0, 1, 3, 5, 6] and sa.tolist() == [1, 0, 2, 1, 3, 2]


@pytest.mark.parametrize("seed", range(10))
def test_invariants_random(seed):
    rng = np.random.default_rng(100 + seed)
    g = random_graph(int(rng.integers(20, 400)), float(rng.uniform(0.01, 0.1)), rng, wmax=100,
                     vmax=20)
    k = int(rng.integers(2, 9))
    ratio = rng.integers(0, 6, k)
    ratio[0] += 1
    opts = oracle.Options(coarsen_to=int(rng.choice([16, 2048])), balance_on=seed % 2)
    r = partition_kway(g, k, ratio, opts)
    assert r.status == 0
    assert r.part.min() >= 0 and r.part.max() < k
    b = g.vwgt[:, opts.balance_on]
    assert sum(r.load) == int(b.sum())
    assert r.cut == kcut(g, r.part)
    # a part with no share gets no vertex (its sibling ranges have shares)
    for p in range(k):
        if ratio[p] == 0:
            assert r.load[p] == 0 or b[r.part == p].sum() == 0


def brute_kway(g, k, maxw, b):
    best = None
    for assign in itertools.product(range(k), repeat=g.n):
        a = np.array(assign)
        if any(b[a == p].sum() > maxw[p] for p in range(k)):
            continue
        c = kcut(g, a)
        best = c if best is None or c < best else best
    return best


def test_brute_force_lower_bound_k3():
    """For 40 graphs of 6-9 vertices, k = 3: whenever every part of the
    heuristic's result lies within ceil(W r_p (10^6 + eps) / (R 10^6)), its
    cut is at least the exhaustive optimum under the same bounds; the share
    of optima found is recorded (quality is not pinned beyond that)."""
    rng = np.random.default_rng(7)
    checked = optimal = 0
    for i in range(40):
        g = random_graph(int(rng.integers(6, 10)), float(rng.uniform(0.2, 0.6)), rng, wmax=9,
                         vmax=5)
        ratio = tuple(int(x) for x in rng.integers(1, 4, 3))
        eps = 200000
        r = partition_kway(g, 3, ratio, oracle.Options(eps_ppm=eps))
        b = g.vwgt[:, 0]
        W, R = int(b.sum()), sum(ratio)
        maxw = [-(-W * ratio[p] * (10**6 + eps) // (R * 10**6)) for p in range(3)]
        if any(r.load[p] > maxw[p] for p in range(3)):
            continue
        opt = brute_kway(g, 3, maxw, b)
        assert opt is not None and r.cut >= opt, (i, r.cut, opt)
        checked += 1
        optimal += r.cut == opt
    assert checked >= 20
    assert optimal >= checked // 3
