"""k-way partition by recursive bisection on the GPU vs the k-way oracle:
the part of every vertex, the cut, the part loads, feasibility and the
number of bisections."""
import sys

import numpy as np
import pytest

import dagen
import oracle
from oracle.kway import partition_kway
from helpers import path_graph, random_graph
from test_oracle_kway import three_cliques

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_kway(gp, g, k, ratio, **kw):
    say(f"case kway {g.name} n={g.n} k={k} ratio={tuple(ratio)} opts={kw}")
    ref = partition_kway(g, k, ratio, oracle.Options(**kw))
    assert ref.status == 0
    h = gp.create(g)
    part, res, load = h.partition_kway(k, ratio, gp.options(**kw))
    got = part.cpu().numpy()
    h.close()
    assert np.array_equal(got, ref.part), f"{int((got != ref.part).sum())} vertices differ"
    assert res.cut == ref.cut and tuple(load) == ref.load
    assert res.feasible == ref.feasible and res.bisections == ref.bisections


def test_kway_small_cases(gp):
    run_kway(gp, path_graph(9), 3, (1, 1, 1))
    run_kway(gp, three_cliques(), 3, (1, 2, 3), eps_ppm=0)
    run_kway(gp, dagen.config_cholesky8(), 1, (3,))
    run_kway(gp, dagen.config_cholesky8(), 3, (0, 1, 1))
    run_kway(gp, dagen.config_cholesky8(), 3, (1, 0, 1))


@pytest.mark.parametrize("seed", range(6))
def test_kway_random(gp, seed):
    rng = np.random.default_rng(300 + seed)
    for case in range(4):
        kind = int(rng.integers(0, 3))
        if kind == 0:
            g = random_graph(int(rng.integers(2, 2000)), float(rng.uniform(0.002, 0.05)), rng,
                             wmax=1000, vmax=50)
        elif kind == 1:
            g = dagen.layered(int(rng.integers(500, 40000)), int(rng.integers(3, 30)),
                              rate=int(rng.integers(1, 5)), seed=int(rng.integers(0, 10**6)))
        else:
            g = dagen.cholesky(int(rng.integers(4, 20)), 512, jitter_pm=100,
                               seed=int(rng.integers(0, 10**6)))
        k = int(rng.integers(2, 9))
        ratio = rng.integers(0, 8, k)
        ratio[int(rng.integers(0, k))] += 1
        run_kway(gp, g, k, ratio.tolist(), eps_ppm=int(rng.choice([0, 30000, 100000])),
                 balance_on=int(rng.integers(0, 2)), coarsen_to=int(rng.choice([32, 2048])))


def test_kway_cholesky64_cpu_gpu_fpga(gp):
    """Three processors with times in ratio 4 : 1 : 2 (CPU, GPU, a third
    accelerator): shares inversely proportional, 1/4 : 1 : 1/2 = 1 : 4 : 2."""
    run_kway(gp, dagen.config_cholesky64_lu48()[0], 3, (1, 4, 2), eps_ppm=30000)


def test_kway_layered1m(gp):
    run_kway(gp, dagen.config_layered1m(), 4, (1, 3, 3, 2), eps_ppm=50000)
