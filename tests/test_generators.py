"""Input generators: closed-form task and dependency counts, CSR form, seeds."""
import hashlib
from math import comb

import numpy as np
import pytest

import dagen
from helpers import assert_canonical


def chol_counts(T):
    n = T + T * (T - 1) + comb(T, 3)
    e = (T - 1) + 2 * (comb(T, 2) + comb(T - 1, 2)) + 2 * comb(T, 3) + comb(T - 1, 3)
    return n, e


def lu_counts(T):
    sq = sum(m * m for m in range(T))
    sqm = sum(m * m for m in range(T - 1))
    n = T + T * (T - 1) + sq
    e = (T - 1) + 2 * (comb(T, 2) + comb(T - 1, 2)) + 2 * sq + sqm
    return n, e


@pytest.mark.parametrize("T", [1, 2, 3, 4, 8, 13, 64])
def test_cholesky_counts(T):
    d = dagen.cholesky_dag(T, 64)
    n, e = chol_counts(T)
    assert d.n == n and len(d.src) == e
    g = dagen.dag_to_graph(d)
    assert g.m == e            # no two dependencies join the same pair of tasks
    assert_canonical(g.xadj, g.adjncy, g.adjwgt, g.n) if T <= 8 else None


def test_cholesky_named_sizes():
    assert chol_counts(8) == (120, 252)
    assert chol_counts(64) == (45760, 131040)
    assert lu_counts(48) == (38024, 109416)


@pytest.mark.parametrize("T", [1, 2, 3, 5, 48])
def test_lu_counts(T):
    d = dagen.lu_dag(T, 64)
    n, e = lu_counts(T)
    assert d.n == n and len(d.src) == e
    g = dagen.dag_to_graph(d)
    assert g.m == e


def test_dag_is_acyclic_in_program_order():
    # task ids follow program order, so every dependency points forward
    for d in (dagen.cholesky_dag(9, 8), dagen.lu_dag(7, 8), dagen.layered_dag(5000, 10)):
        assert np.all(d.src < d.dst)


def test_cholesky8_costs():
    g = dagen.config_cholesky8()
    b3 = 512 ** 3
    vals, counts = np.unique(g.vwgt[:, 0], return_counts=True)
    assert dict(zip(vals.tolist(), counts.tolist())) == {b3 // 3: 8, b3: 56, 2 * b3: 56}
    assert int(g.vwgt[:, 0].sum()) == 22_906_492_240
    assert np.array_equal(g.vwgt[:, 1], g.vwgt[:, 0] // 4)
    assert np.all(g.adjwgt == 2 * 1024 * 1024)
    assert g.n == 120 and g.m == 252


def test_cholesky8_golden_digest():
    # integer-only generator: the digest is the same on every host
    g = dagen.config_cholesky8()
    h = hashlib.sha256()
    for a in (g.xadj, g.adjncy, g.adjwgt, g.vwgt):
        h.update(np.ascontiguousarray(a).tobytes())
    with open(__file__.replace("test_generators.py", "golden/cholesky8.sha256")) as f:
        assert h.hexdigest() == f.read().split()[0]


def test_jitter_bounds():
    d = dagen.cholesky_dag(12, 128, jitter_pm=100)
    base = dagen.cholesky_dag(12, 128)
    ratio = d.vwgt[:, 0] / base.vwgt[:, 0]
    assert ratio.min() >= 0.9 - 1e-6 and ratio.max() <= 1.1 + 1e-6
    assert len(np.unique(ratio)) > 20
    assert np.array_equal(d.vwgt[:, 1], np.maximum(d.vwgt[:, 0] // 4, 1))


def test_layered_structure():
    n, L = 64000, 64
    d = dagen.layered_dag(n, L, rate=3, seed=5)
    layer = np.repeat(np.arange(L), n // L)
    off = layer[d.dst] - layer[d.src]
    assert off.min() >= 1 and off.max() <= 3
    assert not np.any(layer[d.src] == L - 1)
    deg = np.bincount(d.src, minlength=n)[: n - n // L]
    assert abs(deg.mean() - 4.0) < 0.05
    assert abs(np.log(d.vwgt[:, 0]).mean() - 8.0) < 0.05
    assert abs(np.log(d.bytes).mean() - 16.0) < 0.05
    assert np.all(d.vwgt[:, 1] == np.maximum(d.vwgt[:, 0] // 3, 1))
    g = dagen.dag_to_graph(d)
    # parallel arrows merged by summing bytes
    assert int(g.adjwgt.sum()) == 2 * int(d.bytes.sum())
    assert g.nnz <= 2 * len(d.src)


def test_to_csr_merges_and_sorts():
    src = np.array([3, 0, 3, 1, 0], np.int32)
    dst = np.array([0, 2, 0, 2, 1], np.int32)
    by = np.array([5, 7, 1, 2, 3], np.int64)
    g = dagen.to_csr(4, src, dst, by, np.ones((4, 2), np.int64))
    assert g.xadj.tolist() == [0, 3, 5, 7, 8]
    assert g.adjncy.tolist() == [1, 2, 3, 0, 2, 0, 1, 0]
    assert g.adjwgt.tolist() == [3, 7, 6, 3, 2, 7, 2, 6]


def test_seed_determinism():
    a = dagen.layered(3000, 8, seed=11)
    b = dagen.layered(3000, 8, seed=11)
    c = dagen.layered(3000, 8, seed=12)
    assert np.array_equal(a.adjncy, b.adjncy) and np.array_equal(a.vwgt, b.vwgt)
    assert not np.array_equal(a.vwgt, c.vwgt)


def test_batch_plan():
    size, kind, param, _ = dagen.batch_plan(4096, 100, 50000, 0)
    assert size[1::2].min() >= 100 and size.max() <= 50000
    assert np.all(kind[0::2] == 0) and np.all(kind[1::2] == 1)
    for s, T in zip(size[0::2][:50], param[0::2][:50]):
        assert chol_counts(int(T))[0] <= s
    lay = size[1::2]
    assert abs(lay.mean() - 49900 / np.log(500)) / (49900 / np.log(500)) < 0.08
    assert np.all(param[1::2] == np.clip(lay // 100, 4, 64))
