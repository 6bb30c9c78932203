"""GPU tests of the warm-start network's kernels against the FP64 oracle.

Shapes: 14 features -> 128 hidden (tanh) -> 5 outputs, FP32, with row
counts that span several 256-thread blocks and a ragged tail.  Forward
outputs, the packed parameter gradient of the mean squared error, Adam
steps and the warm-start scatter are compared with the numpy FP64 oracle
on the same seeded inputs.
"""
import numpy as np
import pytest

import paper_1811_11007_amd as pt
from oracle import mlp as om

pytestmark = pytest.mark.gpu

NI, NH, NO = pt.PT_NNI_FEATURES, 128, 5


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def inputs(seed, rows):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 1, om.n_params(NI, NH, NO)) * np.sqrt(1.0 / NI)
    x = rng.normal(0, 1, (rows, NI)).astype(np.float32)
    t = rng.normal(0, 0.5, (rows, NO)).astype(np.float32)
    return p.astype(np.float32), x, t


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


@pytest.mark.parametrize("rows", [1, 255, 1037, 40000])
def test_forward_and_gradient_against_oracle(ctx, rows):
    import torch
    say("mlp forward/gradient rows", rows)
    p, x, t = inputs(rows, rows)
    net = pt.MLP(ctx, NI, NH, NO, p)
    X, Tt = dev(x), dev(t)
    y = net.forward(X).cpu().numpy()
    _, yo = om.forward(x.astype(np.float64), p.astype(np.float64), NI, NH, NO)
    assert np.max(np.abs(y - yo)) <= 1e-4 * max(1.0, np.abs(yo).max())
    g = torch.empty(net.n_params, dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    net.gradient(X, Tt, g, loss)
    torch.cuda.synchronize()
    go = om.gradient(x.astype(np.float64), t.astype(np.float64), p.astype(np.float64), NI, NH, NO)
    gg = g.cpu().numpy()
    assert np.max(np.abs(gg - go)) <= 1e-4 * np.abs(go).max(), np.max(np.abs(gg - go))
    lo = om.loss(x.astype(np.float64), t.astype(np.float64), p.astype(np.float64), NI, NH, NO)
    assert abs(loss.item() / (rows * NO) - lo) <= 1e-5 * max(1.0, lo)
    net.close()


def test_adam_steps_against_oracle(ctx):
    import torch
    say("mlp adam")
    p, x, t = inputs(9, 3000)
    net = pt.MLP(ctx, NI, NH, NO, p)
    X, Tt = dev(x), dev(t)
    q = p.astype(np.float64)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    lr, eps = 1e-3, 1e-3
    for s in range(1, 4):
        net.train_step(X, Tt, lr=lr, eps=eps)
        g = om.gradient(x.astype(np.float64), t.astype(np.float64), q, NI, NH, NO)
        q, m, v = om.adam_step(q, g, m, v, s, lr, eps=eps)
    torch.cuda.synchronize()
    got = net.params()
    # each step moves a parameter by at most ~lr; FP32 gradients perturb the
    # step direction only where |g| is within rounding of eps
    assert np.max(np.abs(got - q)) <= 3 * lr * 1e-2, np.max(np.abs(got - q))
    net.close()


def test_training_reduces_loss_like_oracle(ctx):
    import torch
    say("mlp training")
    rng = np.random.default_rng(21)
    x = rng.normal(0, 1, (4096, NI)).astype(np.float32)
    A = rng.normal(0, 0.3, (NI, NO))
    t = np.tanh(x @ A).astype(np.float32)
    p = (rng.normal(0, 1, om.n_params(NI, NH, NO)) * np.sqrt(1.0 / NI)).astype(np.float32)
    net = pt.MLP(ctx, NI, NH, NO, p)
    X, Tt = dev(x), dev(t)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    net.gradient(X, Tt, torch.empty(net.n_params, device="cuda:0"), loss)
    first = loss.item()
    for _ in range(300):
        net.train_step(X, Tt, lr=3e-3)
    net.gradient(X, Tt, torch.empty(net.n_params, device="cuda:0"), loss)
    last = loss.item()
    # the oracle evaluates the trained parameters independently
    lo = om.loss(x.astype(np.float64), t.astype(np.float64), net.params().astype(np.float64), NI, NH, NO)
    assert abs(last / t.size - lo) <= 1e-5
    assert last < 0.1 * first, (first, last)
    net.close()


def test_warm_start_scatter_against_oracle(ctx):
    import torch
    say("mlp warm start")
    rows = 300
    p, x, _ = inputs(31, rows)
    p = p * 0.5
    net = pt.MLP(ctx, NI, NH, NO, p)
    rng = np.random.default_rng(32)
    n_len = rows * 7
    brlen = rng.exponential(0.05, n_len)
    pos = rng.permutation(n_len)[: rows * NO].reshape(rows, NO).astype(np.int32)
    pos[3, 2] = -1  # skipped
    base = rng.exponential(0.05, (rows, NO))
    base[5, 1] = 0.0
    base[6, 2] = -1.0  # negative lengths count as 0
    shift = 1e-4
    B = dev(brlen)
    net.warm_start(dev(x), dev(pos), dev(base), B, t_min=1e-8, t_max=100.0, shift=shift)
    got = B.cpu().numpy()
    _, y = om.forward(x.astype(np.float64), p.astype(np.float64), NI, NH, NO)
    want = brlen.copy()
    for r in range(rows):
        for o in range(NO):
            if pos[r, o] >= 0:
                v = (max(base[r, o], 0.0) + shift) * np.exp(y[r, o]) - shift
                want[pos[r, o]] = min(max(v, 1e-8), 100.0)
    assert np.max(np.abs(got - want) / want) <= 2e-4
    net.close()


def test_mlp_errors(ctx):
    with pytest.raises(pt.PTError):
        pt.MLP(ctx, 0, 4, 4, np.zeros(4))
    p, _, _ = inputs(1, 1)
    p[0] = np.nan
    with pytest.raises(pt.PTError):
        pt.MLP(ctx, NI, NH, NO, p)
    net = pt.MLP(ctx, NI, NH, NO, inputs(1, 1)[0])
    with pytest.raises(ValueError):
        net.set_params(np.zeros(3))
    net.close()


WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(pt.__file__), "warmstart_64x2500.json")


def test_warm_start_gain_on_held_out_alignment(ctx):
    """The trained network (fit on the seed-5 alignment) on a held-out
    64 x 2500 GTR+G4 alignment (seed 6): all 122 NNI neighbours of the
    optimised generating tree.

    Gains over the cold start (lengths inherited from the parent):
      - its starting lengths for the five touched edges are closer to the
        neighbours' optima (log(t + 1e-4) squared error, the centre edge by
        far the most);
      - radius-0 proposals (only the new edge optimised, the gate of the
        search) started from the better of the two starts reach partial
        likelihoods closer to the full optima.
    The full optima are the same from either start: the network moves only
    the starting point (the cold-start optimum is the reference)."""
    import torch
    from paper_1811_11007_amd.search import WarmStart
    from paper_1811_11007_amd.train_warmstart import optimise_start, workload
    say("warm start gain: held-out seed 6")
    e, b, aln = workload(6)
    n = 64
    A = pt.Alignment.from_synth(ctx, aln)
    b0, _ = optimise_start(ctx, A, e, b)
    ne, nb, tt = pt.pt_nni_neighbors(n, e, b0)
    F = pt.pt_nni_features(n, e, b0)
    warm = WarmStart.load(ctx, WEIGHTS)
    E = 2 * n - 3
    K = len(ne)
    T = pt.Trees(list(ne))
    pos = (np.arange(K)[:, None] * E + tt).astype(np.int32)
    base = b0[tt]

    def start(use_warm):
        B = dev(nb.ravel().copy())
        if use_warm:
            warm.apply(dev(F), dev(pos), dev(base), B)
        return B

    def run(B, mask=None):
        plan = pt.Plan(ctx, [A], T, pt.PT_PLAN_OPTIMIZE, pt.PT_FP32, mask=mask)
        lnl = torch.zeros(K, dtype=torch.float64, device="cuda:0")
        ps = torch.zeros(K, dtype=torch.int32, device="cuda:0")
        plan.optimize(B, lnl, ps)
        torch.cuda.synchronize()
        out = lnl.cpu().numpy(), ps.cpu().numpy(), B.cpu().numpy()
        plan.close()
        return out

    bw0 = start(True).cpu().numpy()
    lc, pc, bc = run(start(False))
    lw, pw, bw = run(start(True))
    s = 1e-4
    err_c = (np.log(nb.ravel()[pos] + s) - np.log(bc[pos] + s)) ** 2
    err_w = (np.log(bw0[pos] + s) - np.log(bc[pos] + s)) ** 2
    say("touched-length error cold", err_c.mean(axis=0).round(3), "warm", err_w.mean(axis=0).round(3))
    say("passes cold %d warm %d; max |dlnL| %.2e" % (pc.sum(), pw.sum(), np.max(np.abs(lw - lc))))
    assert err_w[:, 0].mean() < 0.5 * err_c[:, 0].mean()
    assert err_w[:, 1:].mean() < err_c[:, 1:].mean()
    close = np.abs(lw - lc) <= 1e-3
    assert close.mean() >= 0.97, np.sort(np.abs(lw - lc))[-5:]
    mask = np.zeros((K, E), np.uint8)
    mask[np.arange(K), tt[:, 0]] = 1
    l0c, _, _ = run(start(False), mask.ravel())
    l0w, _, _ = run(start(True), mask.ravel())
    l0 = np.maximum(l0c, l0w)
    full = np.maximum(lc, lw)
    gap_c, gap_d = np.mean(full - l0c), np.mean(full - l0)
    say("radius-0 gap to the full optimum: cold %.3f, better of both starts %.3f (warm better for %d of %d)" % (
        gap_c, gap_d, int((l0w > l0c).sum()), K))
    assert gap_d < 0.9 * gap_c


def key_int(k, n):
    W = (n + 63) // 64
    return [str(sum(int(row[w]) << (64 * w) for w in range(W))) for row in k]


def test_warm_started_optima_match_oracle(ctx):
    """The cold-start oracle judges the warm start's results.  The oracle
    optimised the held-out generating tree from its simulated lengths and
    four NNI neighbours from the lengths they inherit (stored by
    tests/golden/make_warm64.py); the GPU's optimum of the start tree and
    its warm-started optima of those neighbours must agree with them to the
    FP32 bar."""
    import json
    import os
    import torch
    from paper_1811_11007_amd.search import WarmStart
    from paper_1811_11007_amd.train_warmstart import optimise_start, workload
    say("warm start vs oracle: held-out seed 6")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "warm64_heldout.json")))
    e, b, aln = workload(g["seed"])
    n = g["n_taxa"]
    assert aln.n_patterns == g["n_patterns"]
    A = pt.Alignment.from_synth(ctx, aln)
    b0, l0 = optimise_start(ctx, A, e, b)
    assert key_int(pt.pt_topology_key(n, e), n) == g["start"]["key"]
    say("start: oracle %.6f gpu %.6f" % (g["start"]["lnl"], l0))
    assert abs(l0 - g["start"]["lnl"]) <= 1e-4
    ne, nb, tt = pt.pt_nni_neighbors(n, e, b0)
    F = pt.pt_nni_features(n, e, b0)
    warm = WarmStart.load(ctx, WEIGHTS)
    idx = [x["index"] for x in g["neighbours"]]
    for i, x in zip(idx, g["neighbours"]):
        assert key_int(pt.pt_topology_key(n, ne[i]), n) == x["key"]
    plan = pt.Plan(ctx, [A], pt.Trees([ne[i] for i in idx]), pt.PT_PLAN_OPTIMIZE, pt.PT_FP32)
    E = 2 * n - 3
    B = dev(np.concatenate([nb[i] for i in idx]))
    pos = (np.arange(len(idx))[:, None] * E + tt[idx]).astype(np.int32)
    warm.apply(dev(F[idx]), dev(pos), dev(b0[tt[idx]]), B)
    lnl = torch.zeros(len(idx), dtype=torch.float64, device="cuda:0")
    plan.optimize(B, lnl)
    got = lnl.cpu().numpy()
    want = np.array([x["lnl"] for x in g["neighbours"]])
    say("neighbours: max |gpu warm - oracle| %.2e" % np.max(np.abs(got - want)))
    assert np.max(np.abs(got - want)) <= 1e-4
    plan.close()
