"""Pins of the oracle's learned-proposal network (inference emulation,
FP64 training gradient, proposal rule)."""
import numpy as np
import pytest
import torch

import dagen
import oracle
from helpers import edgeless_graph, random_graph

H = 64


def params_f32(rng, scale=0.3):
    n = oracle.mpnn_nparam()
    return (rng.standard_normal(n) * scale).astype(np.float32)


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000).astype(np.float32) * 10,
                        # exact ties: halfway between two bf16 values
                        from_bf16_bits(rng.integers(0, 1 << 15, 500).astype(np.uint16)) *
                        np.float32(1 + 2 ** -8),
                        np.array([0.0, -0.0, 1e-40, -3e-39, 65504.0], np.float32)])
    x = x[np.isfinite(x)]
    want = to_bf16_bits(x)
    got = np.array([oracle.bf16_round(float(v)) for v in x], np.uint16)
    assert np.array_equal(got, want)


def test_phi_closed_form():
    for k in range(62):
        assert oracle.phi(1 << k) == k
    rng = np.random.default_rng(1)
    for x in rng.integers(1, 1 << 62, 3000, dtype=np.int64).tolist() + list(range(1, 600)):
        p = oracle.phi(x)
        assert (p * 256) == int(p * 256)                  # multiple of 1/256
        # linear log2 of the mantissa (max gap 0.0861) truncated to 8 bits (< 1/256)
        assert -1e-9 <= np.log2(x) - p < 0.0861 + 1 / 256 + 1e-6


def layer_params(P, l):
    off = H * 4 + H + l * (2 * H * H + H)
    Ws = P[off:off + H * H].reshape(H, H)
    Wn = P[off + H * H:off + 2 * H * H].reshape(H, H)
    b = P[off + 2 * H * H:off + 2 * H * H + H]
    return Ws, Wn, b


def torch_reference(g, P, round_bf16=True):
    """Dense torch float32 network with bf16 rounding at the same points."""
    n = g.n
    x = np.zeros((n, 4), np.float32)
    deg = np.diff(g.xadj)
    tw = np.add.reduceat(g.adjwgt, g.xadj[:-1]) if g.nnz else np.zeros(n)
    tw = np.where(deg > 0, tw, 0)
    for v in range(n):
        x[v] = [oracle.phi(int(g.vwgt[v, 0])), oracle.phi(int(g.vwgt[v, 1])),
                oracle.phi(int(deg[v])), oracle.phi(int(tw[v]))]
    E = np.zeros((n, n), np.float32)
    for v in range(n):
        for q in range(g.xadj[v], g.xadj[v + 1]):
            E[v, g.adjncy[q]] = oracle.phi(int(g.adjwgt[q])) / 64
    inv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0).astype(np.float32)
    r = (lambda t: t.to(torch.bfloat16).to(torch.float32)) if round_bf16 else (lambda t: t)
    Win = torch.from_numpy(P[:H * 4].reshape(H, 4))
    bin_ = torch.from_numpy(P[H * 4:H * 5])
    h = r(torch.relu(torch.from_numpy(x) @ Win.T + bin_))
    Et = torch.from_numpy(E)
    for l in range(3):
        Ws, Wn, b = (torch.from_numpy(a) for a in layer_params(P, l))
        m = r((Et @ h) * torch.from_numpy(inv)[:, None])
        h = r(torch.relu(h @ Ws.T + m @ Wn.T + b))
    wo = torch.from_numpy(P[-H - 1:-1])
    return (h @ wo + float(P[-1])).numpy()


@pytest.mark.parametrize("seed", range(4))
def test_scores_structure_vs_dense_reference(seed):
    rng = np.random.default_rng(seed)
    g = random_graph(int(rng.integers(5, 60)), 0.15, rng, wmax=10**7, vmax=10**6)
    P = from_bf16_bits(to_bf16_bits(params_f32(rng, 0.15)))
    got = oracle.mpnn_scores(g, to_bf16_bits(P))
    ref = torch_reference(g, P)
    # only float32 summation order and the resulting bf16 ties differ
    assert np.allclose(got, ref, rtol=3e-2, atol=3e-2 * (1 + np.abs(ref).max()))
    # a wrong structure (transposed layer weights) is far off
    Pt = P.copy()
    for l in range(3):
        off = H * 5 + l * (2 * H * H + H)
        Pt[off:off + H * H] = Pt[off:off + H * H].reshape(H, H).T.reshape(-1)
    bad = oracle.mpnn_scores(g, to_bf16_bits(Pt))
    assert not np.allclose(bad, ref, rtol=3e-2, atol=3e-2 * (1 + np.abs(ref).max()))


def test_scores_exact_on_dyadic_inputs():
    # a cycle (every degree 2, so 1/deg is exact), edge phi = 4 (e = 1/16),
    # dyadic weights: every FP32 fma below is exact and the only rounding is
    # the BF16 conversion, which the float64 reference applies at the same
    # points through torch's round-to-nearest-even
    n = 16
    src = np.arange(n, dtype=np.int32)
    cpu = 1 << (3 * (np.arange(n) % 7))
    g = dagen.to_csr(n, src, (src + 1) % n, np.full(n, 16, np.int64),
                     np.stack([cpu, np.ones(n, np.int64)], 1))
    P = np.zeros(oracle.mpnn_nparam(), np.float32)
    P[0] = 1.0                       # Win[0][0]: h0[0] = phi(cpu) = 3 (v mod 7)
    P[4] = 0.25                      # Win[1][0]
    P[H * 4 + 1] = -0.5              # b_in[1]
    for l in range(3):
        off = H * 5 + l * (2 * H * H + H)
        P[off + 0] = 0.5             # Ws[0][0]
        P[off + 1] = 0.75            # Ws[0][1]
        P[off + H * H + 0] = 1.0     # Wn[0][0]
        P[off + H * H + H + 0] = -1.0  # Wn[1][0]
        P[off + 2 * H * H + 1] = 0.125  # b[1]
    P[-H - 1] = 1.0                  # wo[0]
    P[-H] = -2.0                     # wo[1]
    P[-1] = 0.5                      # bo
    got = oracle.mpnn_scores(g, to_bf16_bits(P))

    def rb(a):
        return torch.from_numpy(np.asarray(a, np.float64)).to(torch.bfloat16).double().numpy()

    phi = np.array([oracle.phi(int(c)) for c in cpu])
    h = np.zeros((n, 2))
    h[:, 0] = rb(np.maximum(phi, 0))
    h[:, 1] = rb(np.maximum(0.25 * phi - 0.5, 0))
    for l in range(3):
        m = rb((np.roll(h, 1, 0) + np.roll(h, -1, 0)) / 16 * 0.5)
        h0 = rb(np.maximum(0.5 * h[:, 0] + 0.75 * h[:, 1] + m[:, 0], 0))
        h1 = rb(np.maximum(0.125 - m[:, 0], 0))
        h = np.stack([h0, h1], 1)
    want = 0.5 + h[:, 0] - 2.0 * h[:, 1]
    assert np.array_equal(got.astype(np.float64), want)


def test_loss_gradient_central_differences():
    rng = np.random.default_rng(7)
    g = random_graph(10, 0.35, rng, wmax=5000, vmax=50)
    P = params_f32(rng, 0.2).astype(np.float64)
    y = rng.integers(0, 2, g.n).astype(np.int8)
    bw = g.vwgt[:, 0]
    loss, grad = oracle.mpnn_loss_grad_f64(g, bw, y, P)
    idx = np.concatenate([rng.choice(P.size, 400, replace=False),
                          np.arange(P.size - 65, P.size), np.arange(256, 320)])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.mpnn_loss_grad_f64(g, bw, y, Pp)[0] -
              oracle.mpnn_loss_grad_f64(g, bw, y, Pm)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])) + 1e-8, (i, fd, grad[i])


def test_loss_matches_closed_form_at_zero_weights():
    g = random_graph(9, 0.4, np.random.default_rng(3))
    P = np.zeros(oracle.mpnn_nparam(), np.float64)
    y = (np.arange(9) % 2).astype(np.int8)
    loss, grad = oracle.mpnn_loss_grad_f64(g, g.vwgt[:, 0], y, P)
    # every logit is 0: loss = log 2, d/dbo = sum_v w_v (1/2 - y_v)
    assert abs(loss - np.log(2)) < 1e-12
    wv = g.vwgt[:, 0] / g.vwgt[:, 0].sum()
    assert abs(grad[-1] - float((wv * (0.5 - y)).sum())) < 1e-12


def test_learned_partition_kept_only_when_strictly_better():
    rng = np.random.default_rng(5)
    for trial in range(6):
        g = dagen.layered(3000, 12, rate=3, seed=trial)
        model = to_bf16_bits(params_f32(rng, 0.2))
        plain = oracle.partition(g, oracle.Options(ratio=(1, 3)))
        learned = oracle.partition(g, oracle.Options(ratio=(1, 3), flags=oracle.FLAG_LEARNED),
                                   model=model)
        assert learned.status == 0
        if not learned.used_learned:
            assert np.array_equal(learned.part, plain.part) and learned.cut == plain.cut
        assert learned.levels == plain.levels


def test_proposal_fill_rule_zero_model():
    # all-zero weights: every score is 0, the order is by id, so the proposal
    # fills the grown side with the smallest ids that fit (then refinement)
    w = np.array([5, 1, 9, 2, 2, 7, 1, 1, 3, 4] * 5, np.int64)
    g = edgeless_graph(len(w), w)
    model = np.zeros(oracle.mpnn_nparam(), np.uint16)
    r = oracle.partition(g, oracle.Options(flags=oracle.FLAG_LEARNED), model=model)
    plain = oracle.partition(g, oracle.Options())
    # on an edgeless graph both routes give cut 0; the plain result is kept
    assert r.cut == 0 and r.used_learned == 0 and np.array_equal(r.part, plain.part)
