"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every case prints its name before touching the GPU.  Sizes span one to many
tiles with ragged tails; the full-size 4M-vertex layered DAG is checked
against the oracle's stored digest (tests/golden/, written by
make_golden.py from the oracle only).
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import dagen
import oracle
from helpers import complete_graph, edgeless_graph, path_graph, random_graph

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def opts_pair(gp, **kw):
    return gp.options(**kw), oracle.Options(**{k: v for k, v in kw.items()})


def run_both(gp, g, trace=True, **kw):
    go, oo = opts_pair(gp, **kw)
    say(f"case {g.name} n={g.n} nnz={g.nnz} opts={kw}")
    ref = oracle.partition(g, oo)
    assert ref.status == 0
    h = gp.create(g)
    if trace:
        part, res, tr = h.partition(go, trace_cap=64)
    else:
        part, res = h.partition(go)
        tr = None
    got = part.cpu().numpy()
    h.close()
    return ref, got, res, tr


def assert_same(ref, got, res, tr=None):
    if tr is not None and len(ref.trace):
        gt, ot = np.asarray(tr), np.asarray(ref.trace)
        msg = f"gpu trace {gt.tolist()} vs oracle {ot.tolist()}"
        n = min(len(gt), len(ot))
        # coarsening columns (n, 2m, pairs) from the top level down, then the
        # refinement columns from the coarsest level up
        for l in range(n):
            assert np.array_equal(gt[l, [0, 1, 7]], ot[l, [0, 1, 7]]), f"level {l}: {msg}"
        for l in range(n - 1, -1, -1):
            assert np.array_equal(gt[l], ot[l]), f"level {l}: {msg}"
        assert len(gt) == len(ot), msg
    assert res.levels == ref.levels
    assert np.array_equal(got, ref.part), f"{int((got != ref.part).sum())} vertices differ"
    assert res.cut == ref.cut
    assert (res.load[0], res.load[1]) == ref.load
    assert (res.time[0], res.time[1]) == ref.time
    assert res.feasible == ref.feasible


def check_hierarchy(gp, g, **kw):
    """Every phase of the GPU run against the oracle applied to the GPU's own
    level graphs: matching (rounds + two-hop + isolated pairs), contraction,
    initial bisection, projection + refinement.  Names the first phase and
    level that differ."""
    go, oo = opts_pair(gp, **kw)
    say(f"hierarchy {g.name} n={g.n} nnz={g.nnz} opts={kw}")
    h = gp.create(g)
    try:
        _, res = h.partition(go)
        L = res.levels
        lv = [h.level(l) for l in range(L + 1)]
    finally:
        h.close()
    bal = oo.balance_on
    W = int(lv[0]["vwgt"][:, bal].sum())
    C = oo.coarsen_to
    cap = (3 * W + 2 * C - 1) // (2 * C)
    for l in range(L):
        a, c = lv[l], lv[l + 1]
        b = a["vwgt"][:, bal]
        _, m = oracle.match(a["n"], a["xadj"], a["adjncy"], a["adjwgt"], b, cap, oo.seed, l,
                            oo.match_rounds)
        bad = np.nonzero(m != a["match"])[0]
        assert len(bad) == 0, (f"matching differs at level {l} (n={a['n']}): {len(bad)} vertices,"
                               f" first {bad[:8].tolist()} gpu {a['match'][bad[:8]].tolist()} "
                               f"oracle {m[bad[:8]].tolist()}")
        nc, cmap, cx, ca, cw, cvc, cvg = oracle.contract(a["n"], a["xadj"], a["adjncy"],
                                                         a["adjwgt"], a["vwgt"][:, 0],
                                                         a["vwgt"][:, 1], m)
        assert nc == c["n"], f"contraction of level {l}: nc gpu {c['n']} oracle {nc}"
        assert np.array_equal(cx, c["xadj"]), f"contraction of level {l}: xadj"
        assert np.array_equal(ca, c["adjncy"]), f"contraction of level {l}: adjncy"
        assert np.array_equal(cw, c["adjwgt"]), f"contraction of level {l}: adjwgt"
        assert np.array_equal(cvc, c["vwgt"][:, 0]) and np.array_equal(cvg, c["vwgt"][:, 1]), (
            f"contraction of level {l}: vertex weights")
    tgt, maxw = oracle.balance(W, oo.ratio[0], oo.ratio[1], oo.eps_ppm)
    cl = lv[L]
    if not (oo.flags & oracle.FLAG_LEARNED):
        rc, p0, _ = oracle.init_bisect(cl["n"], cl["xadj"], cl["adjncy"], cl["adjwgt"],
                                       cl["vwgt"][:, bal], oo.ratio, tgt, maxw,
                                       min(oo.init_trials, cl["n"]), oo.refine_passes)
        assert rc == 0
        bad = np.nonzero(p0 != cl["part"])[0]
        assert len(bad) == 0, f"initial bisection (n={cl['n']}): {len(bad)} vertices differ"
    for l in range(L - 1, -1, -1):
        a, c = lv[l], lv[l + 1]
        m = a["match"]
        lead = (m < 0) | (np.arange(a["n"]) < m)
        cid = np.cumsum(lead) - 1
        cmap = np.where(lead, cid, cid[np.where(m < 0, 0, m)])
        proj = c["part"][cmap].astype(np.int8)
        b = a["vwgt"][:, bal]
        pw = np.array([b[proj == 0].sum(), b[proj == 1].sum()], np.int64)
        _, pr, _, _ = oracle.refine(a["n"], a["xadj"], a["adjncy"], a["adjwgt"], b, proj, pw,
                                    maxw, oo.refine_passes)
        bad = np.nonzero(pr[:a["n"]] != a["part"])[0]
        assert len(bad) == 0, f"refinement at level {l} (n={a['n']}): {len(bad)} vertices differ"


def test_cholesky8(gp):
    g = dagen.config_cholesky8()
    assert_same(*run_both(gp, g))


@pytest.mark.parametrize("which", [0, 1], ids=["cholesky64", "lu48"])
def test_hierarchy_cholesky64_lu48(gp, which):
    check_hierarchy(gp, dagen.config_cholesky64_lu48()[which], ratio=(1, 4), eps_ppm=30000)


@pytest.mark.parametrize("which", [0, 1], ids=["cholesky64", "lu48"])
def test_cholesky64_lu48(gp, which):
    g = dagen.config_cholesky64_lu48()[which]
    assert_same(*run_both(gp, g))


@pytest.mark.parametrize("seed", range(12))
def test_random_small_with_coarsening(gp, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    g = random_graph(n, float(rng.uniform(0.005, 0.2)), rng, wmax=int(rng.choice([1, 9, 1000])),
                     vmax=int(rng.choice([1, 9, 100])), const_w=bool(seed % 3 == 0),
                     name=f"rand{seed}")
    kw = dict(ratio=[(1, 4), (1, 1), (3, 1), (2, 7)][seed % 4],
              eps_ppm=int(rng.choice([0, 30000, 200000])), balance_on=seed % 2, seed=seed,
              coarsen_to=int(rng.choice([2, 8, 32, 2048])),
              match_rounds=int(rng.choice([0, 1, 8])), refine_passes=int(rng.choice([0, 1, 8])),
              init_trials=int(rng.choice([1, 5, 16])))
    assert_same(*run_both(gp, g, **kw))


@pytest.mark.parametrize("n,L,seed", [(5000, 8, 1), (77777, 16, 2), (262147, 64, 3)])
def test_layered_parity(gp, n, L, seed):
    g = dagen.layered(n, L, rate=3, seed=seed)
    assert_same(*run_both(gp, g, ratio=(1, 3), eps_ppm=50000))


@pytest.mark.parametrize("T", [12, 30])
def test_jittered_cholesky_lu(gp, T):
    for g in (dagen.cholesky(T, 256, jitter_pm=100, seed=T), dagen.lu(T, 256, jitter_pm=100,
                                                                          seed=T)):
        assert_same(*run_both(gp, g, coarsen_to=64))
        assert_same(*run_both(gp, g, balance_on=1, ratio=(2, 5), coarsen_to=256))


def test_special_graphs(gp):
    for g, kw in ((path_graph(3000), dict()), (complete_graph(200), dict(coarsen_to=16)),
                  (edgeless_graph(5000, np.arange(5000) % 17 + 1), dict(coarsen_to=64)),
                  (dagen.config_cholesky8(), dict(ratio=(0, 1))),
                  (dagen.config_cholesky8(), dict(ratio=(1, 0))),
                  (path_graph(1), dict()), (path_graph(2), dict())):
        g.name = g.name or "special"
        assert_same(*run_both(gp, g, **kw))


def test_unsorted_rows_canonicalised(gp):
    rng = np.random.default_rng(5)
    g = dagen.layered(20000, 16, rate=3, seed=9)
    ref = oracle.partition(g)
    adj, w = g.adjncy.copy(), g.adjwgt.copy()
    for u in range(g.n):
        s, e = g.xadj[u], g.xadj[u + 1]
        p = rng.permutation(e - s)
        adj[s:e], w[s:e] = adj[s:e][p], w[s:e][p]
    g2 = dagen.Graph(g.n, g.xadj, adj, w, g.vwgt, "shuffled")
    say("case shuffled rows")
    h = gp.create(g2)
    part, res = h.partition(gp.options())
    assert np.array_equal(part.cpu().numpy(), ref.part) and res.cut == ref.cut
    h.close()


def test_long_rows_and_hubs(gp):
    # a hub joined to every vertex (a long row at every level) plus a sparse rest
    n = 20000
    rng = np.random.default_rng(3)
    src = np.concatenate([np.zeros(n - 1, np.int32), rng.integers(1, n, 30000).astype(np.int32)])
    dst = np.concatenate([np.arange(1, n, dtype=np.int32), rng.integers(1, n, 30000).astype(
        np.int32)])
    keep = src != dst
    g = dagen.to_csr(n, src[keep], dst[keep], rng.integers(1, 50, keep.sum()).astype(np.int64),
                     rng.integers(1, 9, (n, 2)).astype(np.int64), "hub20k")
    assert_same(*run_both(gp, g, coarsen_to=100))


def test_determinism_repeat(gp):
    g = dagen.layered(100000, 32, rate=3, seed=4)
    h = gp.create(g)
    outs = []
    for i in range(3):
        say(f"case repeat {i}")
        part, res = h.partition(gp.options(ratio=(1, 3)))
        outs.append((part.cpu().numpy().copy(), res.cut, res.load[0]))
    h.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1:] == outs[0][1:]


def _bad_cases():
    g = path_graph(5)
    base = dict(xadj=g.xadj, adj=g.adjncy, w=g.adjwgt, vw=g.vwgt)
    out = []

    def mk(name, code, **mods):
        c = {k: v.copy() for k, v in base.items()}
        for k, f in mods.items():
            f(c[k])
        out.append((name, c, code))

    mk("xadj0", oracle.EINVAL, xadj=lambda a: a.__setitem__(0, 1))
    mk("range", oracle.ERANGE, adj=lambda a: a.__setitem__(0, 7))
    mk("negw", oracle.ERANGE, w=lambda a: a.__setitem__(3, -1))
    mk("negv", oracle.ERANGE, vw=lambda a: a.__setitem__((2, 1), -5))
    mk("self", oracle.ESELF, adj=lambda a: a.__setitem__(1, 1))
    mk("dup", oracle.EDUP, adj=lambda a: a.__setitem__(2, 0))
    mk("asym_w", oracle.EASYM, w=lambda a: a.__setitem__(0, 2))
    mk("asym_e", oracle.EASYM, adj=lambda a: a.__setitem__(2, 3))
    mk("overflow", oracle.EOVERFLOW, w=lambda a: a.__setitem__(slice(None), 1 << 60))
    return out


@pytest.mark.parametrize("name,c,code", _bad_cases(), ids=[x[0] for x in _bad_cases()])
def test_create_errors_match_oracle(gp, name, c, code):
    import torch
    say(f"case error {name}")
    r = oracle.partition(n=5, xadj=c["xadj"], adjncy=c["adj"], adjwgt=c["w"], vwgt=c["vw"])
    assert r.status == code
    dev = [torch.from_numpy(np.ascontiguousarray(c[k])).cuda() for k in ("xadj", "adj", "w")]
    vw = torch.from_numpy(np.ascontiguousarray(c["vw"]).reshape(-1)).cuda()
    assert gp.create_status(5, *dev, vw, host=False) == code
    assert gp.create_status(5, c["xadj"], c["adj"], c["w"], np.ascontiguousarray(c["vw"]),
                            host=True) == code


def test_host_pointer_path(gp):
    g = dagen.layered(30000, 16, rate=3, seed=8)
    ref = oracle.partition(g)
    say("case host pointers")
    h = gp.Graph(g.n, g.xadj, g.adjncy, g.adjwgt, np.ascontiguousarray(g.vwgt))
    part, res = h.partition(gp.options())
    h.close()
    assert np.array_equal(part, ref.part) and res.cut == ref.cut


def test_layered4m_full_size(gp):
    """The 4,000,000-vertex layered DAG at its full size, in the launch
    configuration the benchmark times, against the oracle's stored digest."""
    path = os.path.join(HERE, "golden", "layered4m_1to3_eps5.txt")
    exp = dict(l.split("=", 1) for l in open(path).read().split("\n") if "=" in l)
    g = dagen.config_layered4m()
    say("case layered4m full size")
    h = gp.create(g)
    part, res = h.partition(gp.options(ratio=(1, 3), eps_ppm=50000))
    got = part.cpu().numpy()
    h.close()
    assert hashlib.sha256(got.tobytes()).hexdigest() == exp["part_sha256"]
    assert res.cut == int(exp["cut"]) and res.levels == int(exp["levels"])
    assert (res.load[0], res.load[1]) == (int(exp["load0"]), int(exp["load1"]))
    assert (res.time[0], res.time[1]) == (int(exp["time0"]), int(exp["time1"]))


def test_concurrent_streams_match_serial(gp):
    """Two graphs partitioned at the same time from two host threads, each on
    its own stream, give the oracle's results (as the benchmark step runs)."""
    import concurrent.futures
    import ctypes

    import torch
    graphs = dagen.config_cholesky64_lu48()
    refs = [oracle.partition(g, oracle.Options(ratio=(1, 4), eps_ppm=30000)) for g in graphs]
    streams = [torch.cuda.Stream() for _ in graphs]
    arrays = [gp.to_device(g) for g in graphs]
    torch.cuda.synchronize()
    hs = [gp.Graph(*a, stream=ctypes.c_void_p(s.cuda_stream)) for a, s in zip(arrays, streams)]
    parts = [torch.empty(g.n, dtype=torch.int8, device="cuda") for g in graphs]
    torch.cuda.synchronize()
    o = gp.options(ratio=(1, 4), eps_ppm=30000)
    say("case concurrent streams")
    with concurrent.futures.ThreadPoolExecutor(2) as ex:
        for rep in range(3):
            res = list(ex.map(lambda i: hs[i].partition(o, part=parts[i])[1], range(2)))
            torch.cuda.synchronize()
            for p, r, ref in zip(parts, res, refs):
                assert np.array_equal(p.cpu().numpy(), ref.part), f"repeat {rep}"
                assert r.cut == ref.cut and (r.load[0], r.load[1]) == ref.load
    for h in hs:
        h.close()


def star_forest(sizes, rng, name):
    """Stars (centre + leaves) joined by a few random edges, random weights:
    matching stalls after the first rounds, the two-hop pass pairs the
    leftover leaves."""
    src, dst, n = [], [], 0
    for k in sizes:
        src += [n] * k
        dst += list(range(n + 1, n + 1 + k))
        n += k + 1
    # a few edges between random vertices keep the cut from being zero
    extra = rng.integers(0, n, (n // 6, 2))
    extra = extra[extra[:, 0] != extra[:, 1]]
    src = np.concatenate([np.asarray(src, np.int32), extra[:, 0].astype(np.int32)])
    dst = np.concatenate([np.asarray(dst, np.int32), extra[:, 1].astype(np.int32)])
    w = rng.integers(1, 100, len(src)).astype(np.int64)
    vw = rng.integers(1, 20, (n, 2)).astype(np.int64)
    return dagen.to_csr(n, src, dst, w, vw, name)


@pytest.mark.parametrize("rounds", [2, 3, 8])
def test_matching_stalls_match_oracle(gp, rounds):
    # rounds after a settle that matched nothing return at once; every level's
    # matching must still equal the oracle's
    rng = np.random.default_rng(40 + rounds)
    sizes = rng.integers(1, 60, 700).tolist() + [3000, 1]
    g = star_forest(sizes, rng, "stars")
    check_hierarchy(gp, g, coarsen_to=32, match_rounds=rounds)
    assert_same(*run_both(gp, g, coarsen_to=32, match_rounds=rounds))


@pytest.mark.parametrize("seed", range(4))
def test_random_mixed_sweep(gp, seed):
    """50 mixed graphs (random, layered, tiled Cholesky, tiled LU) with random
    options per seed: partition, cut, loads and level count as the oracle's."""
    rng = np.random.default_rng(1000 + seed)
    for case in range(50):
        kind = int(rng.integers(0, 4))
        if kind == 0:
            g = random_graph(int(rng.integers(2, 3000)), float(rng.uniform(0.0005, 0.02)), rng,
                             wmax=int(rng.choice([10, 10**6])), vmax=int(rng.choice([10, 10**4])))
        elif kind == 1:
            g = dagen.layered(int(rng.integers(500, 60000)), int(rng.integers(2, 40)),
                              rate=int(rng.integers(1, 5)), seed=int(rng.integers(0, 10**6)))
        elif kind == 2:
            g = dagen.cholesky(int(rng.integers(4, 24)), 512, jitter_pm=100,
                               seed=int(rng.integers(0, 10**6)))
        else:
            g = dagen.lu(int(rng.integers(4, 20)), 512, jitter_pm=100,
                         seed=int(rng.integers(0, 10**6)))
        kw = dict(ratio=(int(rng.integers(1, 6)), int(rng.integers(1, 6))),
                  eps_ppm=int(rng.choice([0, 10000, 30000, 100000])),
                  balance_on=int(rng.integers(0, 2)), coarsen_to=int(rng.choice([16, 64, 256, 2048])),
                  match_rounds=int(rng.choice([1, 2, 3, 8])),
                  refine_passes=int(rng.choice([1, 2, 8])),
                  init_trials=int(rng.choice([1, 4, 16])), seed=int(rng.integers(0, 1000)))
        ref, got, res, _ = run_both(gp, g, trace=False, **kw)
        assert_same(ref, got, res)


def dense_random(n, deg, seed, name):
    """Random graph with about deg neighbours per vertex, drawn as edge lists
    (the triangle form of random_graph is too large at this size)."""
    rng = np.random.default_rng(seed)
    m = n * deg // 2
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    keep = src != dst
    w = rng.integers(1, 10**6, keep.sum()).astype(np.int64)
    vw = rng.integers(1, 100, (n, 2)).astype(np.int64)
    return dagen.to_csr(n, src[keep], dst[keep], w, vw, name)


def test_long_rows_one_wave_each(gp):
    """Coarse rows of 513..4,096 candidates on levels with few coarse vertices:
    the one-wave packed-key sort.  Every level against the oracle."""
    g = dense_random(6000, 420, 21, "dense6000")
    check_hierarchy(gp, g, coarsen_to=64, ratio=(1, 3))
    assert_same(*run_both(gp, g, coarsen_to=64, ratio=(1, 3)))


@pytest.mark.parametrize("seed", range(6))
def test_dense_coarsest_block_rows(gp, seed):
    """Coarsest graphs whose rows hold more than 128 entries on average: the
    trial form that reads each pick's row with the whole block, on the input
    itself (coarsen_to above n) and on a coarsened dense graph."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(400, 3072))
    g = dense_random(n, int(rng.integers(300, min(n, 2000))), 900 + seed, f"dense{n}")
    assert g.nnz > 128 * g.n
    kw = dict(coarsen_to=4096, ratio=(1, int(rng.integers(1, 6))),
              eps_ppm=int(rng.choice([0, 30000, 100000])), init_trials=int(rng.choice([1, 16])),
              balance_on=seed % 2)
    assert_same(*run_both(gp, g, **kw))
    if seed < 2:
        g = dense_random(12000, 700, 950 + seed, "dense12000")
        check_hierarchy(gp, g, coarsen_to=2048, ratio=(1, 3))
        assert_same(*run_both(gp, g, coarsen_to=2048, ratio=(1, 3)))


def test_long_rows_beyond_packed_ids(gp):
    """Long coarse rows on a level with more than 2^19 - 1 coarse vertices,
    where the packed key does not fit: rows beyond one wave's LDS sort take
    the one-block form, rows of 65..512 candidates the (key, value) wave sort."""
    n = 1_100_000
    rng = np.random.default_rng(8)
    src = rng.integers(0, n, 3 * n).astype(np.int32)
    dst = rng.integers(0, n, 3 * n).astype(np.int32)
    hubs = rng.choice(n, 2300, replace=False).astype(np.int32)
    hs = np.concatenate([np.repeat(hubs[:300], 900), np.repeat(hubs[300:], 150)])
    hd = rng.integers(0, n, len(hs)).astype(np.int32)
    src, dst = np.concatenate([src, hs]), np.concatenate([dst, hd])
    keep = src != dst
    w = rng.integers(1, 1000, keep.sum()).astype(np.int64)
    vw = rng.integers(1, 50, (n, 2)).astype(np.int64)
    g = dagen.to_csr(n, src[keep], dst[keep], w, vw, "hubs1.1m")
    check_hierarchy(gp, g)
    assert_same(*run_both(gp, g))


@pytest.mark.parametrize("seed", range(4))
def test_time_balance_matches_oracle(gp, seed):
    """GP_TIME_BALANCE (each side in its own cost column) on graphs whose
    per-kernel CPU/GPU ratio varies, every level's trace included."""
    from test_oracle_time import mixed_cholesky
    rng = np.random.default_rng(500 + seed)
    graphs = [mixed_cholesky(int(rng.integers(8, 40)), seed),
              dagen.layered(int(rng.integers(2000, 80000)), int(rng.integers(4, 30)), rate=3,
                            seed=seed),
              random_graph(int(rng.integers(3, 400)), 0.03, rng, wmax=100, vmax=50)]
    g = graphs[1]
    g.vwgt = np.stack([g.vwgt[:, 0], rng.integers(1, 5000, g.n)], 1).astype(np.int64)
    for g in graphs:
        W0, W1 = int(g.vwgt[:, 0].sum()), int(g.vwgt[:, 1].sum())
        ratio = (W1, W0)
        while max(ratio) >= 1 << 40:
            ratio = (ratio[0] // 2, ratio[1] // 2)
        kw = dict(ratio=ratio, eps_ppm=int(rng.choice([0, 30000])), flags=oracle.FLAG_TIME,
                  coarsen_to=int(rng.choice([16, 256, 2048])), balance_on=seed % 2)
        assert_same(*run_both(gp, g, **kw))


@pytest.mark.parametrize("seed", range(4))
def test_volume_objective_matches_oracle(gp, seed):
    """GP_VOLUME: the volume passes on the input graph and the reported volume
    equal the oracle's."""
    rng = np.random.default_rng(700 + seed)
    graphs = [dagen.layered(int(rng.integers(2000, 120000)), int(rng.integers(4, 40)), rate=3,
                            seed=seed),
              dagen.cholesky(int(rng.integers(8, 30)), 512, jitter_pm=100, seed=seed),
              random_graph(int(rng.integers(3, 400)), 0.03, rng, wmax=1000, vmax=50)]
    for g in graphs:
        kw = dict(ratio=(1, int(rng.integers(1, 5))), eps_ppm=int(rng.choice([0, 30000, 100000])),
                  flags=oracle.FLAG_VOLUME, coarsen_to=int(rng.choice([16, 2048])),
                  balance_on=seed % 2)
        ref, got, res, tr = run_both(gp, g, **kw)
        assert_same(ref, got, res, tr)
        assert res.volume == ref.volume == oracle.volume(g, ref.part)
