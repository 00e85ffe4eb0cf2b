"""Hand-derived pins of oracle rules that the randomised pins cannot see.

Each case is small enough to work out on paper; the expected values below
come from that working, written next to them, not from running the oracle.
A plausible misreading of each rule (skipping a candidate that does not fit,
moving the whole covering prefix of a rebalance, filling the learned proposal
in another order or stopping at the first vertex that does not fit, other
finaliser constants, another coarsening stall threshold) changes at least
one expected value here.
"""
import numpy as np
import pytest

import dagen
import oracle
from helpers import edgeless_graph

# --------------------------------------------------------------- SplitMix64

GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def test_mix64_published_splitmix64_outputs():
    """The matching hash is built on the SplitMix64 output finaliser (Steele,
    Lea and Flood's SplitMix, in Vigna's public-domain splitmix64.c).  The
    generator adds the golden gamma to its state and finalises; its published
    first outputs from state 1234567 and the first output from state 0 pin
    both multipliers and all three shifts of the finaliser."""
    state = 1234567
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    got = []
    for _ in want:
        state = (state + GOLDEN_GAMMA) % 2**64
        got.append(oracle.mix64(state))
    assert got == want
    assert oracle.mix64(GOLDEN_GAMMA) == 0xE220A8397B1DCDAF


def test_edge_hash_is_the_finaliser_twice():
    # h = mix(mix(seed ^ level) ^ (lo << 32 | hi)), symmetric in its two ends
    s, lvl, a, b = 0x0123456789ABCDEF, 3, 17, 5
    inner = oracle.mix64(s ^ lvl)
    assert oracle.edge_hash(s, lvl, a, b) == oracle.mix64(inner ^ ((5 << 32) | 17))
    assert oracle.edge_hash(s, lvl, b, a) == oracle.edge_hash(s, lvl, a, b)


# ---------------------------------------------------------------- refinement


def _graph(n, edges, b):
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    w = np.array([e[2] for e in edges], np.int64)
    vw = np.stack([np.asarray(b, np.int64)] * 2, 1)
    return dagen.to_csr(n, src, dst, w, vw)


def test_improvement_pass_longest_prefix_no_skipping():
    """Side 0 holds 0, 1, 2 with gains 30, 20, 10 (each has one edge to its
    own partner 3, 4, 5 on side 1).  Weights 1, 10, 1; the GPU side can take
    5 more.  In order 0, 1, 2: vertex 0 fits (1 <= 5), vertex 1 does not
    (11 > 5), so the prefix ends there and vertex 2, which would fit, stays."""
    b = [1, 10, 1, 1, 1, 1]
    g = _graph(6, [(0, 3, 30), (1, 4, 20), (2, 5, 10)], b)
    part = np.array([0, 0, 0, 1, 1, 1], np.int8)
    pw = np.array([12, 3], np.int64)
    maxw = np.array([100, 8], np.int64)
    passes, p, npw, moves = oracle.refine(6, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], part, pw,
                                          maxw, 1)
    assert passes == 1 and moves == 1
    assert p.tolist() == [1, 0, 0, 1, 1, 1]
    assert npw.tolist() == [11, 4]
    # edge 0-3 is now internal: cut 20 + 10
    assert oracle.cut(6, g.xadj, g.adjncy, g.adjwgt, p) == 30


def test_improvement_pass_side_alternates_and_gain_must_be_positive():
    """Pass 0 moves from side 0, pass 1 from side 1.  Same graph, with the
    GPU side full: pass 0 admits nothing (every candidate's weight exceeds
    the room of 0); pass 1 moves from side 1, whose vertices 3, 4, 5 have
    gains 30, 20, 10, into the room of 88 on side 0, all three in one pass.
    Two empty improvement passes are needed to stop, so the first empty one
    does not end the loop."""
    b = [1, 10, 1, 1, 1, 1]
    g = _graph(6, [(0, 3, 30), (1, 4, 20), (2, 5, 10)], b)
    part = np.array([0, 0, 0, 1, 1, 1], np.int8)
    pw = np.array([12, 3], np.int64)
    maxw = np.array([100, 3], np.int64)
    passes, p, npw, moves = oracle.refine(6, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], part, pw,
                                          maxw, 2)
    assert passes == 2 and moves == 3
    assert p.tolist() == [0, 0, 0, 0, 0, 0] and npw.tolist() == [15, 0]
    # with every vertex on side 0 no gain is positive: two empty passes, stop
    passes, p2, npw2, moves2 = oracle.refine(6, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], p, npw,
                                             maxw, 8)
    assert passes == 2 and moves2 == 0 and np.array_equal(p2, p)


def test_rebalance_cut_back_to_what_the_other_side_absorbs():
    """Edgeless, so every gain is 0 and the order is by id.  Side 0 holds
    0, 1, 2 (weight 4 each), side 1 holds 3 (weight 1); maxw = (5, 6).
    Excess of side 0 = 12 - 5 = 7: the covering prefix is {0, 1} (8 >= 7).
    Room on side 1 = 6 - 1 = 5: only {0} fits (4 <= 5, 8 > 5).  One vertex
    moves; side 0 stays over its bound."""
    g = edgeless_graph(4, [4, 4, 4, 1])
    part = np.array([0, 0, 0, 1], np.int8)
    pw = np.array([12, 1], np.int64)
    maxw = np.array([5, 6], np.int64)
    passes, p, npw, moves = oracle.refine(4, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], part, pw,
                                          maxw, 1)
    assert (passes, moves) == (1, 1)
    assert p.tolist() == [1, 0, 0, 1] and npw.tolist() == [8, 5]


def test_rebalance_shortest_covering_prefix():
    """Same shape with a large room: excess 7 is covered by {0, 1} and the
    room of 95 would take all three; the shortest covering prefix wins."""
    g = edgeless_graph(4, [4, 4, 4, 1])
    part = np.array([0, 0, 0, 1], np.int8)
    pw = np.array([12, 1], np.int64)
    maxw = np.array([5, 96], np.int64)
    _, p, npw, moves = oracle.refine(4, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], part, pw,
                                     maxw, 1)
    assert moves == 2 and p.tolist() == [1, 1, 0, 1] and npw.tolist() == [4, 9]


def test_rebalance_orders_by_gain_then_id():
    """Path 0-1-2-3 with weights 5, 1, 7 on its edges; side 0 = {0, 1, 2},
    side 1 = {3}.  Gains on side 0: v0 = -5, v1 = -6, v2 = 7 - 1 = 6.  Order
    (gain desc, id asc): 2, 0, 1.  Unit vertex weights, maxw = (2, 10):
    excess 1, so only vertex 2 moves (cut 1 + 7 -> 1)."""
    g = _graph(4, [(0, 1, 5), (1, 2, 1), (2, 3, 7)], [1, 1, 1, 1])
    part = np.array([0, 0, 0, 1], np.int8)
    pw = np.array([3, 1], np.int64)
    maxw = np.array([2, 10], np.int64)
    _, p, npw, moves = oracle.refine(4, g.xadj, g.adjncy, g.adjwgt, g.vwgt[:, 0], part, pw,
                                     maxw, 1)
    assert moves == 1 and p.tolist() == [0, 0, 1, 1] and npw.tolist() == [2, 2]
    assert oracle.cut(4, g.xadj, g.adjncy, g.adjwgt, p) == 1


# ---------------------------------------------------------- coarsening stop


def _stall_graph(n_light):
    """n_light light vertices (weight 1) in disjoint edges 0-1, 2-3, ...,
    then 100 - n_light heavy isolated vertices (weight 1000)."""
    n = 100
    src = np.arange(0, n_light, 2, dtype=np.int32)
    dst = src + 1
    b = np.full(n, 1000, np.int64)
    b[:n_light] = 1
    return dagen.to_csr(n, src, dst, np.ones(len(src), np.int64), np.stack([b, b], 1))


@pytest.mark.parametrize("n_light,want_n", [(10, [100, 95, 92]), (14, [100, 93, 89])])
def test_coarsening_stall_threshold(n_light, want_n):
    """Coarsening goes on after a level that removed at least 5 % of the
    vertices and stops after one that removed less.  With C = 70 the cap is
    ceil(3W / 140): W = 90,010 gives 1,929 and W = 86,014 gives 1,844, so two
    heavy vertices (2,000) never pair but a light one pairs with anything.
      level 0: the light edges match (5 or 7 pairs); the isolated heavy
               vertices are grouped in id order and never fit the cap;
               100 -> 95 (exactly 5 %: 20*95 = 19*100, go on) or 100 -> 93;
      level 1: the coarse light vertices (ids 0..4 or 0..6) are isolated and
               come first in the isolated group, so pairs form up to the
               first light-heavy pair: 3 or 4 pairs; 95 -> 92 or 93 -> 89;
               both shrink by less than 5 %, so coarsening stops (L = 2)."""
    g = _stall_graph(n_light)
    r = oracle.partition(g, oracle.Options(coarsen_to=70))
    assert r.status == 0 and r.levels == 2
    assert r.trace[:, 0].tolist() == want_n
    assert r.trace[:2, 7].tolist() == [100 - want_n[1], want_n[1] - want_n[2]]


# ---------------------------------------------------- learned proposal fill

BF16_ONE, BF16_MINUS_ONE, BF16_HALF = 0x3F80, 0xBF80, 0x3F00
H = 64
OFF_BIN = H * 4
OFF_L = [OFF_BIN + H + l * (2 * H * H + H) for l in range(3)]
OFF_WO = OFF_BIN + H + 3 * (2 * H * H + H)
OFF_BO = OFF_WO + H


def cpu_cost_model(sign_bits, bias_bits):
    """A network whose score is sign * phi(cpu cost) + bias, exactly:
    hidden unit 0 copies phi(cpu) through the three layers (self weight 1),
    every other weight is 0."""
    P = np.zeros(oracle.mpnn_nparam(), np.uint16)
    P[0] = BF16_ONE                      # Win[0][0]
    for off in OFF_L:
        P[off] = BF16_ONE                # Ws[0][0] of each layer
    P[OFF_WO] = sign_bits
    P[OFF_BO] = bias_bits
    return P


# cpu costs 3, 8, 2, 8, 5, 1, 6, 4 -> phi = 1.5, 3, 1, 3, 2.25, 0, 2.5, 2
CPU = [3, 8, 2, 8, 5, 1, 6, 4]


def test_learned_scores_of_the_hand_model():
    g = edgeless_graph(8, CPU)
    s = oracle.mpnn_scores(g, cpu_cost_model(BF16_ONE, 0))
    assert s.tolist() == [1.5, 3.0, 1.0, 3.0, 2.25, 0.0, 2.5, 2.0]
    s = oracle.mpnn_scores(g, cpu_cost_model(BF16_MINUS_ONE, BF16_HALF))
    assert s.tolist() == [-1.0, -2.5, -0.5, -2.5, -1.75, 0.5, -2.0, -1.5]


def test_learned_fill_order_ties_and_skip():
    """Scores 1.5, 3, 1, 3, 2.25, 0, 2.5, 2: order (score desc, id asc) is
    1, 3, 6, 4, 7, 0, 2, 5.  Weights = cpu costs, tgt_0 = 12, maxw_0 = 14:
    1 joins (8); 3 does not fit (16 > 14) and is passed over; 6 joins (14);
    14 >= 12 ends the fill.  Side 0 = {1, 6}."""
    g = edgeless_graph(8, CPU)
    b = np.array(CPU, np.int64)
    part, pw = oracle.learned_fill(g, cpu_cost_model(BF16_ONE, 0), b, 0, [12, 25], [14, 30])
    assert part.tolist() == [1, 0, 1, 1, 1, 1, 0, 1]
    assert pw.tolist() == [14, 23]


def test_learned_fill_negative_scores():
    """Scores 0.5 - phi = -1, -2.5, -0.5, -2.5, -1.75, 0.5, -2, -1.5: order
    5, 2, 0, 7, 4, 6, 1, 3 (negative floats ordered by value).  Filling to
    tgt 12 under maxw 14: 5, 2, 0, 7 reach 10; 4 (15), 6 (16), 1 and 3 (18)
    do not fit; the fill ends below the target."""
    g = edgeless_graph(8, CPU)
    b = np.array(CPU, np.int64)
    part, pw = oracle.learned_fill(g, cpu_cost_model(BF16_MINUS_ONE, BF16_HALF), b, 0,
                                   [12, 25], [14, 30])
    assert part.tolist() == [0, 1, 0, 1, 1, 0, 1, 0]
    assert pw.tolist() == [10, 27]


def test_learned_fill_grows_part_one():
    """Grown side 1 (a ratio with the larger CPU share): the same order
    1, 3, 6, ... fills part 1 to tgt_1 = 9 under maxw_1 = 10: 1 joins (8),
    3 and 6 do not fit, 4 (13), 7 (12), 0 (11) do not fit, 2 joins (10)."""
    g = edgeless_graph(8, CPU)
    b = np.array(CPU, np.int64)
    part, pw = oracle.learned_fill(g, cpu_cost_model(BF16_ONE, 0), b, 1, [28, 9], [30, 10])
    assert part.tolist() == [0, 1, 1, 0, 0, 0, 0, 0]
    assert pw.tolist() == [27, 10]


def test_learned_proposal_kept_in_the_pipeline():
    """A whole learned partition that the judge keeps.  Cliques A = {1..4}
    and B = {5..8} (edge weight 100) and vertex 0 tied to 1 and 5 (weight 2
    each); unit balance weights (gpu column), ratio 4:5, eps 0, so side 0
    must hold exactly 4.  One greedy trial seeds vertex 0, then takes 1
    (gain -298, tie with 5 broken by id), 2 (-100) and 3 (+100): side 0 =
    {0, 1, 2, 3}, cut 3 x 100 + 2 = 302, and no positive gain fits either
    side afterwards.  The hand model scores phi(cpu) = 3 for B and 0 for the
    rest, so the proposal is side 0 = B with cut 2 (edge 0-5), which
    refinement cannot improve; 2 < 302, so the learned result is kept."""
    edges = [(a, c, 100) for a in range(1, 5) for c in range(a + 1, 5)]
    edges += [(a, c, 100) for a in range(5, 9) for c in range(a + 1, 9)]
    edges += [(0, 1, 2), (0, 5, 2)]
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    w = np.array([e[2] for e in edges], np.int64)
    cpu = np.array([1, 1, 1, 1, 1, 8, 8, 8, 8], np.int64)
    g = dagen.to_csr(9, src, dst, w, np.stack([cpu, np.ones(9, np.int64)], 1))
    model = cpu_cost_model(BF16_ONE, 0)
    opts = dict(ratio=(4, 5), eps_ppm=0, balance_on=1, init_trials=1)
    plain = oracle.partition(g, oracle.Options(**opts))
    assert plain.cut == 302 and plain.part.tolist() == [0, 0, 0, 0, 1, 1, 1, 1, 1]
    part, pw = oracle.learned_fill(g, model, g.vwgt[:, 1], 0, [4, 5], [4, 5])
    assert part.tolist() == [1, 1, 1, 1, 1, 0, 0, 0, 0] and pw.tolist() == [4, 5]
    r = oracle.partition(g, oracle.Options(**opts, flags=oracle.FLAG_LEARNED), model=model)
    assert r.status == 0 and r.used_learned == 1 and r.cut == 2 and r.feasible
    assert r.part.tolist() == [1, 1, 1, 1, 1, 0, 0, 0, 0]


# ------------------------------------------------- judge on the input graph

def _key(r):
    return (1 - int(r.feasible), int(r.cut))


def _judge_invariants(g, kw, model):
    plain = oracle.partition(g, oracle.Options(**kw))
    lr = oracle.partition(g, oracle.Options(**kw, flags=oracle.FLAG_LEARNED), model=model)
    assert plain.status == 0 and lr.status == 0
    assert lr.levels == plain.levels
    if lr.used_learned:
        # kept only when strictly better on the input graph
        assert _key(lr) < _key(plain)
    else:
        assert np.array_equal(lr.part, plain.part) and lr.cut == plain.cut
        assert lr.load == plain.load and lr.time == plain.time
    return plain, lr


def test_learned_never_worse_than_plain_random():
    """The plain bisection judges the learned one after both are projected and
    refined to the input graph: the learned form never ends worse than the
    plain one, and it equals the plain result whenever it is not kept.  A
    judge at the coarsest level breaks this on some of these graphs."""
    rng = np.random.default_rng(77)
    kept = 0
    for i in range(24):
        g = dagen.layered(int(rng.integers(600, 5000)), int(rng.integers(3, 16)), rate=3,
                          seed=int(rng.integers(0, 10**6)))
        P = (rng.standard_normal(oracle.mpnn_nparam()) * 0.3).astype(np.float32)
        bits = (P.view(np.uint32) >> 16).astype(np.uint16)   # truncation to BF16 is fine here
        kw = dict(ratio=(1, int(rng.integers(1, 5))), eps_ppm=30000,
                  coarsen_to=int(rng.choice([32, 128, 512])))
        _, lr = _judge_invariants(g, kw, bits)
        kept += lr.used_learned
    assert 0 < kept < 24


def test_learned_judged_after_uncoarsening_cholesky64():
    """The committed trained weights on the tiled Cholesky T=64 DAG (1:4, 3 %):
    the learned proposal beats the best greedy trial on the coarsest graph,
    but after projection and refinement it ends with a larger cut, so the
    judge on the input graph keeps the plain result.  On the tiled LU T=48
    DAG the learned run ends with a smaller cut and is kept."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1502_07451_amd", "mpnn_weights.bin")
    model = np.fromfile(path, dtype=np.uint16)
    chol, lu = dagen.config_cholesky64_lu48()
    kw = dict(ratio=(1, 4), eps_ppm=30000)
    plain, lr = _judge_invariants(chol, kw, model)
    assert lr.used_learned == 0 and lr.cut == plain.cut
    plain, lr = _judge_invariants(lu, kw, model)
    assert lr.used_learned == 1 and lr.cut < plain.cut
