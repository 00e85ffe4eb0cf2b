"""Time balance (GP_TIME_BALANCE): side 0 measured by CPU cost, side 1 by GPU
cost, each against its own bound; pinned by a hand-worked case and by
invariants of the result."""
import numpy as np
import pytest

import dagen
import oracle
from helpers import edgeless_graph, random_graph


def time_bounds(g, ratio, eps):
    W0, W1 = int(g.vwgt[:, 0].sum()), int(g.vwgt[:, 1].sum())
    _, m0 = oracle.balance(W0, ratio[0], ratio[1], eps)
    _, m1 = oracle.balance(W1, ratio[0], ratio[1], eps)
    return int(m0[0]), int(m1[1])


def test_hand_case_moves_the_gpu_friendly_kernel():
    """Four independent kernels, (CPU, GPU) costs (1, 7), (6, 3), (4, 6),
    (3, 2); totals 14 and 18, ratio (18, 14) from Eq. (1), eps 0.
    Plain (CPU column): side 1 grows (r1 < r0) from vertex 0: 0 (pw 1), then
    1 (pw 7 = tgt 6 reached): parts (1, 1, 0, 0), feasible in the CPU column
    (7 <= 8 and 7 <= 7), but the GPU would run 7 + 3 = 10 time units.
    Time balance: bounds ceil(14 * 18 / 32) = 8 and ceil(18 * 14 / 32) = 8;
    side 1 is 2 over, the rebalance orders its kernels 0, 1 (gains 0, ids),
    covers the excess with kernel 0 (GPU cost 7) and the CPU absorbs it (CPU
    cost 1 <= 8 - 7): parts (0, 1, 0, 0), times (8, 3)."""
    cpu, gpu = [1, 6, 4, 3], [7, 3, 6, 2]
    g = edgeless_graph(4, cpu)
    g.vwgt = np.array([cpu, gpu], np.int64).T.copy()
    plain = oracle.partition(g, oracle.Options(ratio=(18, 14), eps_ppm=0))
    assert plain.part.tolist() == [1, 1, 0, 0] and plain.feasible == 1
    assert plain.time == (7, 10)
    r = oracle.partition(g, oracle.Options(ratio=(18, 14), eps_ppm=0, flags=oracle.FLAG_TIME))
    assert r.status == 0 and r.part.tolist() == [0, 1, 0, 0]
    assert r.load == (8, 3) and r.time == (8, 3) and r.feasible == 1
    assert time_bounds(g, (18, 14), 0) == (8, 8)


def test_time_balance_with_learned_is_rejected():
    g = dagen.config_cholesky8()
    P = np.zeros(oracle.mpnn_nparam(), np.uint16)
    r = oracle.partition(g, oracle.Options(flags=oracle.FLAG_TIME | oracle.FLAG_LEARNED),
                         model=P)
    assert r.status == oracle.EINVAL


def mixed_cholesky(T, seed):
    """Tiled Cholesky whose GEMMs gain 8x on the GPU and the other kernels 2x
    (the per-kernel ratio is not uniform)."""
    g = dagen.cholesky(T, 256, jitter_pm=100, seed=seed)
    cpu = g.vwgt[:, 0].copy()
    gemm = cpu > 1.5 * 256 ** 3
    g.vwgt = np.stack([cpu, np.where(gemm, cpu // 8, cpu // 2)], 1).astype(np.int64)
    return g


@pytest.mark.parametrize("seed", range(8))
def test_invariants(seed):
    rng = np.random.default_rng(seed)
    if seed % 2:
        g = mixed_cholesky(int(rng.integers(4, 14)), seed)
    else:
        g = random_graph(int(rng.integers(5, 500)), float(rng.uniform(0.01, 0.1)), rng,
                         wmax=100, vmax=50)
    W0, W1 = int(g.vwgt[:, 0].sum()), int(g.vwgt[:, 1].sum())
    eps = int(rng.choice([0, 30000, 100000]))
    ratio = (W1, W0)
    while max(ratio) >= 1 << 40:
        ratio = (ratio[0] // 2, ratio[1] // 2)
    r = oracle.partition(g, oracle.Options(ratio=ratio, eps_ppm=eps, flags=oracle.FLAG_TIME,
                                           coarsen_to=int(rng.choice([8, 2048]))))
    assert r.status == 0
    t0 = int(g.vwgt[r.part == 0, 0].sum())
    t1 = int(g.vwgt[r.part == 1, 1].sum())
    assert r.load == (t0, t1) == r.time
    m0, m1 = time_bounds(g, ratio, eps)
    assert r.feasible == int(t0 <= m0 and t1 <= m1)
