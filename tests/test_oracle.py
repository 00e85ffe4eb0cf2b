"""Pins of the CPU oracle against things other than itself.

Closed forms (Eq. (1)-(2) and the balance bounds in exact rational
arithmetic), exhaustive search on graphs of at most 20 vertices, the
equivalence of converged mutual-proposal matching with sequential greedy
matching, contraction as the matrix product P^T A P, invariants of every
step, and special graphs whose optimum is known in closed form.
"""
from fractions import Fraction
from math import ceil, floor

import numpy as np
import pytest

import dagen
import oracle
from helpers import (assert_canonical, brute_force, complete_graph, cut_of, dense_adj,
                     edgeless_graph, edges_of, path_graph, random_graph)

# --------------------------------------------------------------- Eq. (1)-(2)


def test_ratio_from_times_eq1():
    # R_CPU = T_GPU / (T_GPU + T_CPU): a GPU 4x faster gives CPU:GPU = 1:4
    assert oracle.ratio_from_times(400, 100) == (0, (1, 4))
    assert oracle.ratio_from_times(7, 21) == (0, (3, 1))
    # the GPU so fast that the CPU share vanishes (Section IV-C, Fig. 6 discussion)
    assert oracle.ratio_from_times(5, 0) == (0, (0, 1))
    rc, (a, b) = oracle.ratio_from_times(123456789, 987654321)
    assert rc == 0 and Fraction(a, a + b) == Fraction(987654321, 987654321 + 123456789)
    assert oracle.ratio_from_times(0, 0)[0] == oracle.EINVAL
    assert oracle.ratio_from_times(-1, 3)[0] == oracle.EINVAL


@pytest.mark.parametrize("W,r0,r1,eps", [
    (22_906_492_240, 1, 4, 30000), (0, 1, 4, 30000), (17, 1, 1, 0), (10**18, 3, 7, 50000),
    ((1 << 62) - 1, (1 << 40) - 1, 1, 1_000_000), ((1 << 62) - 1, 1, (1 << 40) - 1, 999_999),
    (123_456_789_012, 0, 5, 30000)])
def test_balance_exact(W, r0, r1, eps):
    tgt, maxw = oracle.balance(W, r0, r1, eps)
    R = r0 + r1
    for p, r in enumerate((r0, r1)):
        assert tgt[p] == floor(Fraction(W * r, R))
        assert maxw[p] == ceil(Fraction(W * r * (10**6 + eps), R * 10**6))
    assert int(maxw[0]) + int(maxw[1]) >= W


def test_balance_cholesky8_values():
    W = 22_906_492_240
    tgt, maxw = oracle.balance(W, 1, 4, 30000)
    assert tgt.tolist() == [4_581_298_448, 18_325_193_792]
    assert maxw.tolist() == [4_718_737_402, 18_874_949_606]


# ----------------------------------------------------------- canonical input


def test_canonicalize_sorts_rows():
    rng = np.random.default_rng(1)
    g = random_graph(30, 0.3, rng)
    xadj, adj, w = g.xadj.copy(), g.adjncy.copy(), g.adjwgt.copy()
    for u in range(g.n):
        s, e = xadj[u], xadj[u + 1]
        perm = rng.permutation(e - s)
        adj[s:e], w[s:e] = adj[s:e][perm], w[s:e][perm]
    rc, ox, oa, ow = oracle.canonicalize(g.n, xadj, adj, w, g.vwgt)
    assert rc == 0
    assert np.array_equal(ox, g.xadj) and np.array_equal(oa, g.adjncy)
    assert np.array_equal(ow, g.adjwgt)


def _bad_inputs():
    g = path_graph(5)
    base = dict(n=5, xadj=g.xadj.copy(), adj=g.adjncy.copy(), w=g.adjwgt.copy(),
                vw=g.vwgt.copy())
    cases = []
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["xadj"][0] = 1
    cases.append(("xadj0", c, oracle.EINVAL))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["xadj"][2], c["xadj"][3] = c["xadj"][3], c["xadj"][2]
    cases.append(("xadj_dec", c, oracle.EINVAL))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["adj"][0] = 7
    cases.append(("range", c, oracle.ERANGE))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["w"][3] = -1
    cases.append(("negw", c, oracle.ERANGE))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["vw"][2, 1] = -5
    cases.append(("negv", c, oracle.ERANGE))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["adj"][1] = 1   # row 1 = [0, 2] -> [1, 2]
    cases.append(("self", c, oracle.ESELF))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["adj"][2] = 0   # row 1 = [0, 2] -> [0, 0]
    cases.append(("dup", c, oracle.EDUP))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["w"][0] = 2
    cases.append(("asym_w", c, oracle.EASYM))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["adj"][2] = 3   # row 1 = [0, 3]: 1-3 has no 3-1
    cases.append(("asym_e", c, oracle.EASYM))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["w"][:] = 1 << 60
    cases.append(("overflow_w", c, oracle.EOVERFLOW))
    c = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in base.items()}
    c["vw"][:, 0] = 1 << 60
    cases.append(("overflow_v", c, oracle.EOVERFLOW))
    return cases


@pytest.mark.parametrize("name,c,code", _bad_inputs(), ids=[x[0] for x in _bad_inputs()])
def test_canonicalize_errors(name, c, code):
    rc, *_ = oracle.canonicalize(c["n"], c["xadj"], c["adj"], c["w"], c["vw"])
    assert rc == code
    r = oracle.partition(n=c["n"], xadj=c["xadj"], adjncy=c["adj"], adjwgt=c["w"], vwgt=c["vw"])
    assert r.status == code


def test_option_errors():
    g = path_graph(10)
    for kw in (dict(ratio=(0, 0)), dict(ratio=(-1, 2)), dict(ratio=(1 << 40, 1)),
               dict(eps_ppm=-1), dict(eps_ppm=1_000_001), dict(balance_on=2),
               dict(coarsen_to=0), dict(init_trials=0), dict(match_rounds=65)):
        assert oracle.partition(g, oracle.Options(**kw)).status == oracle.EINVAL, kw
    assert oracle.partition(g, oracle.Options(flags=oracle.FLAG_LEARNED)).status == oracle.EMODEL


# ------------------------------------------------------------------ matching


def greedy_matching(g, b, cap, seed, level):
    """Sequential greedy over all edges sorted by the matching order."""
    u, v, w = edges_of(g)
    keys = []
    for a, c, wt in zip(u.tolist(), v.tolist(), w.tolist()):
        h = oracle.edge_hash(seed, level, a, c)
        keys.append((-wt, -h, a, c))
    order = sorted(range(len(keys)), key=lambda i: keys[i])
    match = -np.ones(g.n, np.int32)
    for i in order:
        a, c = int(u[i]), int(v[i])
        if match[a] < 0 and match[c] < 0 and b[a] + b[c] <= cap:
            match[a], match[c] = c, a
    return match


def check_matching_valid(g, match, b, cap):
    for x in range(g.n):
        y = match[x]
        if y >= 0:
            assert match[y] == x
            row = g.adjncy[g.xadj[x]:g.xadj[x + 1]]
            assert y in row
            assert b[x] + b[y] <= cap


@pytest.mark.parametrize("trial", range(40))
def test_matching_converged_equals_greedy(trial):
    rng = np.random.default_rng(100 + trial)
    n = int(rng.integers(2, 60))
    g = random_graph(n, float(rng.uniform(0.05, 0.5)), rng, wmax=int(rng.choice([1, 2, 5, 50])),
                     const_w=bool(trial % 3 == 0))
    b = g.vwgt[:, 0]
    cap = int(rng.choice([10**9, 12, 8]))
    seed, level = int(rng.integers(0, 2**63)), int(trial % 5)
    pairs, m = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, cap, seed, level, 10**6,
                            twohop=False)
    check_matching_valid(g, m, b, cap)
    ref = greedy_matching(g, b, cap, seed, level)
    assert np.array_equal(m, ref)
    assert pairs == int((m >= 0).sum()) // 2
    # a fixed round count yields a subset of the converged matching
    _, m8 = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, cap, seed, level, 2, twohop=False)
    check_matching_valid(g, m8, b, cap)
    sel = m8 >= 0
    assert np.array_equal(m8[sel], ref[sel])


def test_matching_is_maximal_when_converged():
    rng = np.random.default_rng(7)
    g = random_graph(200, 0.05, rng, wmax=1, const_w=True)
    b = g.vwgt[:, 0]
    _, m = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, 10**9, 3, 0, 10**6, twohop=False)
    u, v, _ = edges_of(g)
    assert not np.any((m[u] < 0) & (m[v] < 0))


def test_matching_heavy_edge_first():
    # a triangle 0-1 (5), 1-2 (9), 0-2 (1): the heaviest edge wins
    g = dagen.to_csr(3, np.array([0, 1, 0], np.int32), np.array([1, 2, 2], np.int32),
                     np.array([5, 9, 1], np.int64), np.ones((3, 2), np.int64))
    _, m = oracle.match(3, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], 10, 0, 0, 8, twohop=False)
    assert m.tolist() == [-1, 2, 1]
    # with the cap below b(1)+b(2) the next heaviest eligible edge is taken
    vw = np.array([[1, 1], [1, 1], [5, 5]], np.int64)
    _, m = oracle.match(3, g.xadj, g.adjncy, g.adjwgt, vw[:, 0], 3, 0, 0, 8, twohop=False)
    assert m.tolist() == [1, 0, -1]


def hubs_of(g, seed, level):
    """Best neighbour of every vertex under the matching edge order (-1: none)."""
    u, v, w = edges_of(g)
    best = {}
    for a, c, wt in zip(u.tolist(), v.tolist(), w.tolist()):
        key = (-wt, -oracle.edge_hash(seed, level, a, c), a, c)
        for x, y in ((a, c), (c, a)):
            if x not in best or key < best[x][0]:
                best[x] = (key, y)
    return [best[x][1] if x in best else -1 for x in range(g.n)]


@pytest.mark.parametrize("trial", range(30))
def test_twohop_pairs_leaves_of_one_hub(trial):
    rng = np.random.default_rng(900 + trial)
    n = int(rng.integers(3, 80))
    g = random_graph(n, float(rng.uniform(0.02, 0.3)), rng, wmax=int(rng.choice([1, 7, 90])))
    b = g.vwgt[:, 0]
    cap = int(rng.choice([10**9, 13, 9]))
    seed, level = int(rng.integers(0, 2**62)), trial % 3
    rounds = int(rng.integers(0, 3))
    _, m0 = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, cap, seed, level, rounds,
                         twohop=False)
    p2, m1 = oracle.match_twohop(g.n, g.xadj, g.adjncy, g.adjwgt, b, cap, seed, level, m0)
    _, mfull = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, cap, seed, level, rounds)
    assert np.array_equal(m1, mfull)
    # earlier pairs untouched, result still a matching within the cap
    assert np.all(m1[m0 >= 0] == m0[m0 >= 0])
    for x in range(n):
        if m1[x] >= 0:
            assert m1[m1[x]] == x and b[x] + b[m1[x]] <= cap
    hub = hubs_of(g, seed, level)
    free = [x for x in range(n) if m0[x] < 0]
    groups = {}
    for x in free:
        groups.setdefault(hub[x], []).append(x)
    expect = m0.copy()
    made = 0
    for h, members in groups.items():
        members.sort()
        for i in range(0, len(members) - 1, 2):
            x, y = members[i], members[i + 1]
            if b[x] + b[y] <= cap:
                expect[x], expect[y] = y, x
                made += 1
    assert np.array_equal(m1, expect) and p2 == made
    # a pair shares a neighbour, or both vertices have none
    for x in range(n):
        y = m1[x]
        if m0[x] < 0 and y >= 0:
            nx = set(g.adjncy[g.xadj[x]:g.xadj[x + 1]].tolist())
            ny = set(g.adjncy[g.xadj[y]:g.xadj[y + 1]].tolist())
            assert (nx & ny) or (not nx and not ny)


def test_twohop_star_collapses():
    # star with 9 leaves: plain matching pairs the centre once, two-hop pairs 4 leaf pairs
    n = 10
    g = dagen.to_csr(n, np.zeros(9, np.int32), np.arange(1, 10, dtype=np.int32),
                     np.arange(1, 10, dtype=np.int64), np.ones((n, 2), np.int64))
    pairs, m = oracle.match(n, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], 100, 0, 0, 8)
    assert m[0] == 9 and m[9] == 0          # heaviest edge 0-9
    assert m[1:9].tolist() == [2, 1, 4, 3, 6, 5, 8, 7]
    assert pairs == 5


# --------------------------------------------------------------- contraction


@pytest.mark.parametrize("trial", range(25))
def test_contraction_is_PtAP(trial):
    rng = np.random.default_rng(300 + trial)
    n = int(rng.integers(2, 50))
    g = random_graph(n, float(rng.uniform(0.05, 0.6)), rng, wmax=20)
    b = g.vwgt[:, 0]
    _, m = oracle.match(g.n, g.xadj, g.adjncy, g.adjwgt, b, 10**9, trial, 0,
                        int(rng.integers(1, 4)))
    nc, cmap, cx, ca, cw, cvc, cvg = oracle.contract(g.n, g.xadj, g.adjncy, g.adjwgt,
                                                     g.vwgt[:, 0], g.vwgt[:, 1], m)
    # coarse ids follow the pair leaders (single or smaller id) in ascending order
    leaders = [u for u in range(n) if m[u] < 0 or u < m[u]]
    assert nc == len(leaders)
    assert [int(cmap[u]) for u in leaders] == list(range(nc))
    for u in range(n):
        if m[u] >= 0:
            assert cmap[u] == cmap[m[u]]
    # P^T A P with the diagonal (internal edges) removed
    P = np.zeros((n, nc), np.int64)
    P[np.arange(n), cmap] = 1
    A = dense_adj(n, g.xadj, g.adjncy, g.adjwgt)
    Ac = P.T @ A @ P
    np.fill_diagonal(Ac, 0)
    assert np.array_equal(dense_adj(nc, cx, ca, cw), Ac)
    assert_canonical(cx, ca, cw, nc)
    # both cost columns conserved, coarse vertex = sum over its members
    assert np.array_equal(cvc, P.T @ g.vwgt[:, 0]) and np.array_equal(cvg, P.T @ g.vwgt[:, 1])
    # total edge weight drops by exactly the matched edges
    mw = sum(int(A[u, m[u]]) for u in range(n) if m[u] > u)
    assert int(cw.sum()) == int(g.adjwgt.sum()) - 2 * mw
    # the cut of a coarse assignment equals the cut of its projection
    pc = rng.integers(0, 2, nc).astype(np.int8)
    assert oracle.cut(nc, cx, ca, cw, pc) == cut_of(g, pc[cmap])


# ---------------------------------------------------------------- refinement


def _random_feasible_setup(trial):
    rng = np.random.default_rng(500 + trial)
    n = int(rng.integers(5, 80))
    g = random_graph(n, float(rng.uniform(0.05, 0.4)), rng, wmax=30, vmax=9)
    b = g.vwgt[:, trial % 2].copy()
    W = int(b.sum())
    ratio = [(1, 4), (1, 1), (3, 1), (2, 5)][trial % 4]
    tgt, maxw = oracle.balance(W, ratio[0], ratio[1], 50000)
    part = rng.integers(0, 2, n).astype(np.int8)
    pw = np.array([int(b[part == 0].sum()), int(b[part == 1].sum())], np.int64)
    return rng, g, b, part, pw, maxw


@pytest.mark.parametrize("trial", range(30))
def test_refine_invariants(trial):
    rng, g, b, part, pw, maxw = _random_feasible_setup(trial)
    cuts = [cut_of(g, part)]
    cur, cpw = part.copy(), pw.copy()
    for p in range(1, 12):
        passes, nxt, npw, moves = oracle.refine(g.n, g.xadj, g.adjncy, g.adjwgt, b, cur, cpw,
                                                maxw, 1)
        # tracked loads equal recomputed loads
        assert npw.tolist() == [int(b[nxt == 0].sum()), int(b[nxt == 1].sum())]
        was_feasible = cpw[0] <= maxw[0] and cpw[1] <= maxw[1]
        c = cut_of(g, nxt)
        if was_feasible:
            # an improvement pass never raises the cut and keeps feasibility
            assert c <= cuts[-1]
            assert npw[0] <= maxw[0] and npw[1] <= maxw[1]
            if moves > 0:
                assert c < cuts[-1]
        cuts.append(c)
        cur, cpw = nxt, npw


@pytest.mark.parametrize("trial", range(20))
def test_refine_converged_is_stable(trial):
    rng, g, b, part, pw, maxw = _random_feasible_setup(trial)
    passes, p1, pw1, moves = oracle.refine(g.n, g.xadj, g.adjncy, g.adjwgt, b, part, pw, maxw, 64)
    if pw1[0] <= maxw[0] and pw1[1] <= maxw[1] and passes < 64:
        _, p2, pw2, moves2 = oracle.refine(g.n, g.xadj, g.adjncy, g.adjwgt, b, p1, pw1, maxw, 64)
        assert moves2 == 0 and np.array_equal(p1, p2)


def test_refine_rebalances():
    g = path_graph(40)
    b = g.vwgt[:, 0]
    tgt, maxw = oracle.balance(40, 1, 1, 0)
    part = np.zeros(40, np.int8)
    part[35:] = 1
    pw = np.array([35, 5], np.int64)
    _, p, npw, _ = oracle.refine(40, g.xadj, g.adjncy, g.adjwgt, b, part, pw, maxw, 8)
    assert npw.tolist() == [20, 20]
    # side 0 in (gain desc, id asc) order: 34 (gain 0), 0 (gain -1), then 1, 2, ...
    # (gain -2); 15 of them cover the excess of 15, later passes find no gain
    expect = np.zeros(40, np.int8)
    expect[:14] = 1
    expect[34:] = 1
    assert np.array_equal(p, expect) and cut_of(g, p) == 2


# ----------------------------------------------------------- whole pipeline


def _check_result(g, r, opts):
    b = g.vwgt[:, opts.balance_on]
    assert r.status == 0
    assert set(np.unique(r.part)) <= {0, 1}
    assert r.cut == cut_of(g, r.part)
    assert r.load == (int(b[r.part == 0].sum()), int(b[r.part == 1].sum()))
    assert r.time == (int(g.vwgt[r.part == 0, 0].sum()), int(g.vwgt[r.part == 1, 1].sum()))
    tgt, maxw = oracle.balance(int(b.sum()), *opts.ratio, opts.eps_ppm)
    assert r.feasible == int(r.load[0] <= maxw[0] and r.load[1] <= maxw[1])
    return maxw


def test_bruteforce_bound_many():
    """Exhaustive optimum vs the oracle on thousands of tiny graphs."""
    rng = np.random.default_rng(2024)
    stats = dict(total=0, feasible_bf=0, feasible_or=0, optimal=0)
    for trial in range(1500):
        n = int(rng.integers(1, 13)) if trial < 1400 else int(rng.integers(13, 17))
        g = random_graph(n, float(rng.uniform(0.1, 0.7)), rng, wmax=int(rng.choice([1, 9, 100])),
                         vmax=int(rng.choice([1, 5, 50])), const_w=bool(trial % 4 == 0))
        opts = oracle.Options(ratio=[(1, 4), (1, 1), (1, 3), (4, 1), (2, 3)][trial % 5],
                              eps_ppm=int(rng.choice([0, 30000, 100000, 300000])),
                              balance_on=trial % 2, seed=trial,
                              coarsen_to=int(rng.choice([2, 3, 4, 2048])),
                              init_trials=int(rng.choice([1, 4, 16])))
        r = oracle.partition(g, opts)
        maxw = _check_result(g, r, opts)
        b = g.vwgt[:, opts.balance_on]
        opt, _ = brute_force(g, b, maxw)
        stats["total"] += 1
        if opt is not None:
            stats["feasible_bf"] += 1
            stats["feasible_or"] += r.feasible
            if r.feasible:
                assert r.cut >= opt
                stats["optimal"] += int(r.cut == opt)
        else:
            assert not r.feasible
    # Quality floor: a regression threshold recorded from the first run of the
    # heuristic (1234 of 1376 feasible, 962 of those optimal); not a pin.
    # Most misses are eps = 0 instances that need an exact subset sum.
    assert stats["feasible_or"] >= 1220 and stats["optimal"] >= 950


@pytest.mark.parametrize("n", [17, 20])
def test_bruteforce_bound_20(n):
    rng = np.random.default_rng(n)
    for trial in range(3):
        g = random_graph(n, 0.25, rng, wmax=10, vmax=6)
        opts = oracle.Options(coarsen_to=4, seed=trial)
        r = oracle.partition(g, opts)
        maxw = _check_result(g, r, opts)
        opt, _ = brute_force(g, g.vwgt[:, 0], maxw)
        if r.feasible:
            assert opt is not None and r.cut >= opt


@pytest.mark.parametrize("g", [dagen.cholesky(2, 512), dagen.cholesky(3, 512), dagen.lu(2, 512)],
                         ids=["chol2", "chol3", "lu2"])
def test_special_tiny_dags_optimal(g):
    """Tiled Cholesky T=2 (4 tasks), T=3 (10 tasks), LU T=2 (5 tasks): the
    oracle reaches the exhaustive optimum whenever one exists."""
    for ratio in ((1, 1), (1, 2), (1, 3), (1, 4)):
        for eps in (30000, 100000, 300000):
            opts = oracle.Options(ratio=ratio, eps_ppm=eps)
            r = oracle.partition(g, opts)
            maxw = _check_result(g, r, opts)
            opt, _ = brute_force(g, g.vwgt[:, 0], maxw)
            if opt is None:
                assert not r.feasible
            else:
                assert r.feasible and r.cut == opt, (ratio, eps)


@pytest.mark.parametrize("n", [100, 1000, 2048])
def test_special_path_cut_one(n):
    # unit path at 1:4: the CPU side must hold at least n - maxw_1 > 0 vertices
    g = path_graph(n)
    r = oracle.partition(g, oracle.Options())
    _check_result(g, r, oracle.Options())
    assert r.cut == 1 and r.feasible and r.levels == 0
    # trial 0 grows a prefix from vertex 0
    k = int(r.load[0])
    assert np.all(r.part[:k] == 0) and np.all(r.part[k:] == 1)


@pytest.mark.parametrize("g", [path_graph(50), complete_graph(30), dagen.config_cholesky8()],
                         ids=["path", "K30", "chol8"])
def test_special_zero_cpu_share(g):
    # ratio 0:1 - the CPU gets nothing and nothing is cut (Section IV-C, Fig. 6)
    r = oracle.partition(g, oracle.Options(ratio=(0, 1)))
    assert r.status == 0 and r.cut == 0 and np.all(r.part == 1) and r.feasible


def test_special_zero_gpu_share():
    g = dagen.config_cholesky8()
    r = oracle.partition(g, oracle.Options(ratio=(1, 0)))
    assert r.cut == 0 and np.all(r.part == 0)


def test_special_two_components():
    # component A (ids 16..31, a path, weight 16) and component B (the rest, a
    # path, weight 64); W = 80 and the CPU target is exactly 16 at 1:4
    n = 64
    src, dst = [], []
    for a in range(16, 31):
        src.append(a); dst.append(a + 1)
    rest = [v for v in range(n) if not 16 <= v < 32]
    for a, c in zip(rest[:-1], rest[1:]):
        src.append(a); dst.append(c)
    vw = np.ones((n, 2), np.int64)
    vw[rest[:16], :] = 2
    g = dagen.to_csr(n, np.array(src, np.int32), np.array(dst, np.int32),
                     np.full(len(src), 3, np.int64), vw)
    assert int(vw[:, 0].sum()) == 80
    r = oracle.partition(g, oracle.Options(eps_ppm=0))
    assert r.cut == 0 and r.load == (16, 64)
    assert np.all(r.part[16:32] == 0)


@pytest.mark.parametrize("n", [10, 30, 100])
def test_special_complete_graph(n):
    g = complete_graph(n)
    opts = oracle.Options()
    r = oracle.partition(g, opts)
    tgt, maxw = oracle.balance(n, 1, 4, 30000)
    a = max(0, n - int(maxw[1]))
    assert r.load[0] == a and r.cut == a * (n - a)


@pytest.mark.parametrize("seed", range(4))
def test_special_edgeless(seed):
    rng = np.random.default_rng(seed)
    n = 200
    w = rng.integers(1, 20, n) if seed else np.ones(n, np.int64)
    g = edgeless_graph(n, w)
    r = oracle.partition(g, oracle.Options())
    assert r.cut == 0
    tgt, maxw = oracle.balance(int(w.sum()), 1, 4, 30000)
    # trial 0: seed vertex 0, then the smallest ids that still fit
    expect = np.ones(n, np.int8)
    pw0 = 0
    for v in range(n):
        if pw0 >= tgt[0]:
            break
        if pw0 + w[v] <= maxw[0]:
            expect[v] = 0
            pw0 += w[v]
    assert np.array_equal(r.part, expect)


def test_balance_on_gpu_column():
    g = dagen.cholesky(6, 512, jitter_pm=100)
    for bal in (0, 1):
        opts = oracle.Options(balance_on=bal, ratio=(1, 3))
        r = oracle.partition(g, opts)
        _check_result(g, r, opts)
        assert r.feasible


def test_empty_and_single():
    r = oracle.partition(n=0, xadj=np.zeros(1, np.int32), adjncy=np.zeros(0, np.int32),
                         adjwgt=np.zeros(0, np.int64), vwgt=np.zeros((0, 2), np.int64))
    assert r.status == 0 and r.cut == 0 and r.feasible and len(r.part) == 0
    g = edgeless_graph(1, [7])
    r = oracle.partition(g, oracle.Options())
    # 1:4 with one vertex of weight 7: maxw = (2, 6), so neither side can take
    # it; growing finds nothing that fits and the vertex stays on the GPU side
    assert r.part.tolist() == [1] and not r.feasible


def test_levels_and_trace_consistent():
    g = dagen.layered(20000, 16, seed=3)
    opts = oracle.Options(coarsen_to=256)
    r = oracle.partition(g, opts)
    _check_result(g, r, opts)
    assert r.levels >= 3
    tr = r.trace
    assert tr[0, 0] == g.n and tr[0, 1] == g.nnz and tr[0, 4] == r.cut
    for l in range(1, r.levels + 1):
        # each level removes exactly its matched pairs
        assert tr[l, 0] == tr[l - 1, 0] - tr[l - 1, 7]
        assert tr[l, 5] + tr[l, 6] == tr[0, 5] + tr[0, 6]
    # stop rule: only the last level may have shrunk by less than 5 %
    for l in range(1, r.levels):
        assert 20 * tr[l, 0] <= 19 * tr[l - 1, 0]
    assert tr[r.levels - 1, 0] > 256
