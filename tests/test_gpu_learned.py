"""Learned coarsest-level proposal on the GPU vs the oracle: inference scores
bit for bit, and whole partitions with the proposal and its acceptance check."""
import sys

import numpy as np
import pytest
import torch

import dagen
import oracle
from helpers import random_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(oracle.mpnn_nparam()) * scale).astype(np.float32)
    return torch.from_numpy(p).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)


@pytest.mark.parametrize("seed", range(5))
def test_scores_bit_exact(gp, seed):
    rng = np.random.default_rng(seed)
    graphs = [random_graph(int(rng.integers(1, 400)), float(rng.uniform(0.01, 0.3)), rng,
                           wmax=10**7, vmax=10**6),
              dagen.layered(3000, 10, rate=3, seed=seed),
              dagen.cholesky(9, 512, jitter_pm=100, seed=seed)]
    P = rand_params(seed)
    model = gp.Model(P)
    for g in graphs:
        say(f"case scores seed={seed} {g.name} n={g.n}")
        ref = oracle.mpnn_scores(g, P)
        h = gp.create(g)
        got = h.scores(model).cpu().numpy()
        h.close()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (
            f"{int((got != ref).sum())} scores differ")
    model.close()


@pytest.mark.parametrize("seed", range(4))
def test_learned_partition_matches_oracle(gp, seed):
    P = rand_params(100 + seed)
    model = gp.Model(P)
    for g, ratio in ((dagen.layered(40000, 32, rate=3, seed=seed), (1, 3)),
                     (dagen.cholesky(24, 512, jitter_pm=100, seed=seed), (1, 4)),
                     (dagen.lu(20, 512, jitter_pm=100, seed=seed), (1, 4))):
        say(f"case learned seed={seed} {g.name}")
        ref = oracle.partition(g, oracle.Options(ratio=ratio, flags=oracle.FLAG_LEARNED),
                               model=P)
        h = gp.create(g)
        part, res = h.partition(gp.options(ratio=ratio, flags=gp.LEARNED, model=model.handle))
        h.close()
        assert ref.status == 0
        assert np.array_equal(part.cpu().numpy(), ref.part)
        assert res.cut == ref.cut and res.used_learned == ref.used_learned
        assert (res.load[0], res.load[1]) == ref.load and res.levels == ref.levels
    model.close()


def test_learned_requires_model(gp):
    g = dagen.config_cholesky8()
    h = gp.create(g)
    with pytest.raises(gp.GPError) as e:
        h.partition(gp.options(flags=gp.LEARNED))
    assert e.value.status == gp.EMODEL
    h.close()


def test_trained_weights_match_oracle(gp):
    """The committed trained weights: the learned path on the tiled Cholesky
    T=64 DAG equals the oracle's, acceptance decision included."""
    import os
    from paper_1502_07451_amd import learn
    if not os.path.exists(learn.WEIGHTS_PATH):
        pytest.skip("no trained weights")
    P = learn.load_weights()
    g = dagen.config_cholesky64_lu48()[0]
    say("case trained weights cholesky64")
    ref = oracle.partition(g, oracle.Options(ratio=(1, 4), eps_ppm=30000,
                                             flags=oracle.FLAG_LEARNED), model=P)
    model = gp.Model(P)
    h = gp.create(g)
    part, res = h.partition(gp.options(ratio=(1, 4), eps_ppm=30000, flags=gp.LEARNED,
                                       model=model.handle))
    h.close()
    model.close()
    assert ref.status == 0 and res.used_learned == ref.used_learned
    assert np.array_equal(part.cpu().numpy(), ref.part) and res.cut == ref.cut


def test_trained_weights_layered1m(gp):
    """The learned path with the committed trained weights on the 1,000,000-
    vertex layered DAG (1:3, eps 5 %), its other evaluation graph: the same
    assignment, cut, loads and acceptance decision as the oracle."""
    import os
    from paper_1502_07451_amd import learn
    if not os.path.exists(learn.WEIGHTS_PATH):
        pytest.skip("no trained weights")
    g = dagen.config_layered1m()
    say("case trained weights layered1m")
    model = gp.Model.load(learn.WEIGHTS_PATH)
    h = gp.create(g)
    part, res = h.partition(gp.options(ratio=(1, 3), eps_ppm=50000, flags=gp.LEARNED,
                                       model=model.handle))
    got = part.cpu().numpy()
    h.close()
    model.close()
    ref = oracle.partition(g, oracle.Options(ratio=(1, 3), eps_ppm=50000,
                                             flags=oracle.FLAG_LEARNED),
                           model=learn.load_weights())
    assert ref.status == 0 and res.used_learned == ref.used_learned
    assert np.array_equal(got, ref.part) and res.cut == ref.cut
    assert (res.load[0], res.load[1]) == ref.load and res.levels == ref.levels


def test_model_load_equals_create(gp):
    """gp_model_load reads the blob file the training driver writes; its scores
    equal those of gp_model_create on the same parameters."""
    import os
    from paper_1502_07451_amd import learn
    if not os.path.exists(learn.WEIGHTS_PATH):
        pytest.skip("no trained weights")
    g = dagen.cholesky(12, 512, jitter_pm=100, seed=3)
    say("case model load")
    a = gp.Model.load(learn.WEIGHTS_PATH)
    b = gp.Model(learn.load_weights())
    h = gp.create(g)
    sa = h.scores(a).cpu().numpy()
    sb = h.scores(b).cpu().numpy()
    h.close()
    a.close()
    b.close()
    assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))
