"""Training kernels of the learned proposal on the GPU.

* gradients (MFMA BF16 products, FP32 accumulation) against the oracle's
  FP64 backward of the same network at the same BF16-rounded weights;
* Adam steps lower the loss;
* the batched coarsest-level export equals the single-graph path's coarsest
  level (graph and refined plain bisection: the training labels).
"""
import sys

import numpy as np
import pytest
import torch

import dagen
import oracle
from helpers import random_graph

pytestmark = pytest.mark.gpu

NP = 25153


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_values(p32):
    """FP32 values of the BF16 (RNE) rounding of p32."""
    t = torch.from_numpy(np.ascontiguousarray(p32, np.float32)).to(torch.bfloat16)
    return t.to(torch.float32).numpy()


def small_graphs(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = i % 3
        if k == 0:
            g = random_graph(int(rng.integers(2, 300)), float(rng.uniform(0.01, 0.2)), rng,
                             wmax=10**7, vmax=10**6)
        elif k == 1:
            g = dagen.layered(int(rng.integers(50, 1500)), int(rng.integers(2, 12)), rate=3,
                              seed=seed * 100 + i)
        else:
            g = dagen.cholesky(int(rng.integers(3, 10)), 512, jitter_pm=100, seed=seed * 100 + i)
        out.append(g)
    return out


def to_trainer_data(graphs, labels, device="cuda"):
    bb = dagen.concat(graphs)
    import paper_1502_07451_amd as gp
    G, voff, eoff, xadj, adj, w, vw = gp.batch_to_device(bb, device)
    lab = torch.from_numpy(np.concatenate(labels).astype(np.int8)).to(device)
    return G, voff, eoff, xadj, adj, w, vw, lab


def layout():
    H = 64
    out = [("win", H * 4), ("b_in", H)]
    for l in range(3):
        out += [(f"ws{l}", H * H), (f"wn{l}", H * H), (f"b{l}", H)]
    return out + [("wo", H), ("bo", 1)]


@pytest.mark.parametrize("seed", range(3))
def test_gradients_vs_fp64(gp, seed):
    from paper_1502_07451_amd import learn
    graphs = small_graphs(seed, 6)
    rng = np.random.default_rng(seed)
    labels = [(rng.random(g.n) < 0.3).astype(np.int8) for g in graphs]
    p32 = learn.init_params(seed)
    p32[p32.size - 65:] *= 4.0  # a livelier output layer
    pb = bf16_values(p32)
    say(f"case grad seed={seed} sizes={[g.n for g in graphs]}")
    tr = gp.Trainer(pb)
    data = to_trainer_data(graphs, labels)
    tr.set_data(*data, balance_on=0)
    loss, grad = tr.grad(0, len(graphs))
    tr.close()
    ref = np.zeros(NP)
    ref_loss = 0.0
    for g, y in zip(graphs, labels):
        l, gr = oracle.mpnn_loss_grad_f64(g, g.vwgt[:, 0], y, pb.astype(np.float64))
        ref += gr / len(graphs)
        ref_loss += l / len(graphs)
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss) + 1e-6, (loss, ref_loss)
    tot = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    assert tot <= 2e-2, f"whole gradient: relative error {tot:.4g}"
    o = 0
    for name, k in layout():
        a, b = grad[o:o + k].astype(np.float64), ref[o:o + k]
        o += k
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / nb
        say(f"  {name}: relative error {rel:.4g}")
        assert rel <= 2e-2, f"{name}: relative error {rel:.4g}"


def test_adam_lowers_loss(gp):
    from paper_1502_07451_amd import learn
    graphs = small_graphs(7, 24)
    # labels from the plain pipeline: the oracle's partition of each graph
    labels = []
    for g in graphs:
        r = oracle.partition(g, oracle.Options(ratio=(1, 4), coarsen_to=1 << 30))
        labels.append((r.part == 0).astype(np.int8))
    tr = gp.Trainer(learn.init_params(3))
    tr.set_data(*to_trainer_data(graphs, labels), balance_on=0)
    first = tr.grad(0, len(graphs))[0]
    for _ in range(60):
        tr.step(0, len(graphs), 3e-3)
    last = tr.grad(0, len(graphs))[0]
    f32, b16 = tr.params()
    tr.close()
    say(f"loss {first:.5f} -> {last:.5f}")
    assert np.isfinite(last) and last < 0.9 * first
    assert np.array_equal(b16, torch.from_numpy(f32).to(torch.bfloat16).view(torch.int16)
                          .numpy().view(np.uint16))


def test_export_equals_single_graph_coarsest(gp):
    from paper_1502_07451_amd import learn
    graphs = [dagen.layered(20000, 16, rate=3, seed=1), dagen.cholesky(20, 512, 100, seed=2),
              dagen.lu(16, 512, 100, seed=3), dagen.layered(1500, 6, rate=4, seed=4)]
    bb = dagen.concat(graphs)
    opts = gp.options(ratio=(1, 4), eps_ppm=30000)
    say("case export")
    items = learn.export_coarsest(bb, opts, "cuda")
    for g, it in zip(graphs, items):
        h = gp.create(g)
        _, res = h.partition(opts)
        lv = h.level(res.levels)
        h.close()
        n, xadj, adj, w, vw, part = it
        assert n == lv["n"]
        assert np.array_equal(xadj, lv["xadj"]) and np.array_equal(adj, lv["adjncy"])
        assert np.array_equal(w, lv["adjwgt"]) and np.array_equal(vw, lv["vwgt"])
        assert np.array_equal(part, lv["part"])
