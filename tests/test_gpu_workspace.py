"""Allocation failure forced from the host: a per-handle device-memory limit
(gp_set_workspace_limit) turns any growth past it into GP_ENOMEM, and the
handle stays usable - the next call with room gives the oracle's result."""
import sys

import numpy as np
import pytest

import dagen
import oracle
from oracle.kway import partition_kway

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def graph_bytes(g):
    # the handle's copy: xadj, adjncy, adjwgt, two cost columns, match, cmap, part
    return 4 * (g.n + 1) + 12 * g.nnz + 8 * 2 * g.n + 4 * 2 * g.n + g.n


def test_limit_refuses_then_recovers(gp):
    g = dagen.cholesky(24, 512, jitter_pm=100, seed=1)
    kw = dict(ratio=(1, 4), coarsen_to=256)
    say(f"case workspace {g.name} n={g.n} nnz={g.nnz}")
    ref = oracle.partition(g, oracle.Options(**kw))
    assert ref.status == 0 and ref.levels >= 2
    h = gp.create(g)
    used0 = h.workspace_bytes()
    assert used0 >= graph_bytes(g)
    for cap in (0, used0):
        h.set_workspace_limit(cap)
        with pytest.raises(gp.GPError) as e:
            h.partition(gp.options(**kw))
        assert e.value.status == gp.ENOMEM and h.workspace_bytes() == used0
    # a fresh handle run without a limit: the most a partition holds
    h2 = gp.create(g)
    part, res = h2.partition(gp.options(**kw))
    peak = h2.workspace_bytes()
    h2.close()
    assert np.array_equal(part.cpu().numpy(), ref.part) and peak > used0
    # every limit below it is refused part-way; the buffers grown so far stay
    # within the limit and serve the next call
    for k in range(1, 8):
        cap = used0 + (peak - used0) * k // 8
        h.set_workspace_limit(cap)
        with pytest.raises(gp.GPError) as e:
            h.partition(gp.options(**kw))
        assert e.value.status == gp.ENOMEM
        assert h.workspace_bytes() <= cap
        with pytest.raises(gp.GPError):
            h.level(0)
    h.set_workspace_limit(peak)
    part, res = h.partition(gp.options(**kw))
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert res.cut == ref.cut and (res.load[0], res.load[1]) == ref.load
    assert res.levels == ref.levels and h.workspace_bytes() == peak
    # nothing more to grow: the same call again under the same limit
    part, res = h.partition(gp.options(**kw))
    assert np.array_equal(part.cpu().numpy(), ref.part)
    with pytest.raises(gp.GPError) as e:
        h.set_workspace_limit(-2)
    assert e.value.status == gp.EINVAL
    h.close()


def test_limit_covers_kway_subgraphs(gp):
    g = dagen.layered(20000, 12, rate=3, seed=4)
    say(f"case workspace kway {g.name} n={g.n}")
    ref = partition_kway(g, 4, (1, 2, 3, 4), oracle.Options())
    h = gp.create(g)
    h.set_workspace_limit(h.workspace_bytes())
    with pytest.raises(gp.GPError) as e:
        h.partition_kway(4, (1, 2, 3, 4), gp.options())
    assert e.value.status == gp.ENOMEM
    h.set_workspace_limit(-1)
    before = h.workspace_bytes()
    part, res, load = h.partition_kway(4, (1, 2, 3, 4), gp.options())
    assert np.array_equal(part.cpu().numpy(), ref.part) and res.cut == ref.cut
    assert tuple(load) == ref.load
    # the subgraph handles were charged to this one and gave their bytes back
    after = h.workspace_bytes()
    assert before < after < before + 4 * graph_bytes(g) + (1 << 20)
    h.close()
