"""The allocation-free batched entry point against gp_partition_batch, through
the C ABI: the same assignments and results on two calls in a row, the
second with a smaller batch, and the rejection of bounds beyond its fixed
scratch."""
import sys

import numpy as np
import pytest

import dagen
from helpers import path_graph, random_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def graphs_of(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = i % 4
        if k == 0:
            out.append(dagen.layered(int(rng.integers(200, 9000)), int(rng.integers(3, 20)),
                                     rate=4, seed=i))
        elif k == 1:
            out.append(dagen.cholesky(int(rng.integers(3, 16)), 512, jitter_pm=100, seed=i))
        elif k == 2:
            out.append(random_graph(int(rng.integers(1, 300)), 0.05, rng, wmax=100, vmax=9))
        else:
            out.append(path_graph(int(rng.integers(1, 400))))
    return out


def both(gp, graphs, kw):
    import torch
    b = dagen.concat(graphs)
    dev = gp.batch_to_device(b)
    bt = gp.Batch()
    ref_part, ref_res = bt.partition(*dev, opts=gp.options(**kw))
    torch.cuda.synchronize()
    bt.close()
    part, res = gp.partition_batch_noalloc(*dev, opts=gp.options(**kw))
    torch.cuda.synchronize()
    got = gp.results_from_device(res, b.G)
    return ref_part.cpu().numpy(), ref_res, part.cpu().numpy(), got


@pytest.mark.parametrize("kw", [dict(ratio=(1, 4), eps_ppm=30000), dict(coarsen_to=64)],
                         ids=["default", "deep"])
def test_noalloc_equals_batch_twice(gp, kw):
    graphs = graphs_of(3, 40)
    for call, sub in enumerate((graphs, graphs[5:17])):
        say(f"case noalloc call {call} graphs={len(sub)} {kw}")
        rp, rr, gp_, gr = both(gp, sub, kw)
        assert [r.status for r in gr] == [r.status for r in rr], f"call {call}: statuses"
        assert np.array_equal(rp, gp_), f"call {call}: assignments differ"
        assert [r.as_dict() for r in rr] == [r.as_dict() for r in gr], f"call {call}"
        assert all(r.status == 0 for r in gr)


def test_noalloc_rejects_oversized(gp):
    import torch
    graphs = graphs_of(5, 4)
    b = dagen.concat(graphs)
    dev = gp.batch_to_device(b)
    say("case noalloc oversized")
    with pytest.raises(gp.GPError) as e:
        gp.partition_batch_noalloc(*dev, nmax=1 << 22, nnzmax=1 << 25, ntot=1 << 22,
                                   nnztot=1 << 25)
    assert e.value.status == gp.ENOMEM
    # a graph larger than the stated bound gets its own GP_EINVAL, the others run
    sizes = np.diff(b.voff)
    part, res = gp.partition_batch_noalloc(*dev, nmax=int(sizes.max()) - 1)
    torch.cuda.synchronize()
    got = gp.results_from_device(res, b.G)
    big = int(np.argmax(sizes))
    assert got[big].status == gp.EINVAL
    assert all(r.status == 0 for i, r in enumerate(got) if i != big and sizes[i] < sizes.max())
