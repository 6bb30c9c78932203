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
    base[5, 1] = 0.0  # floored at 1e-6
    B = dev(brlen)
    net.warm_start(dev(x), dev(pos), dev(base), B, t_min=1e-8, t_max=100.0)
    got = B.cpu().numpy()
    _, y = om.forward(x.astype(np.float64), p.astype(np.float64), NI, NH, NO)
    want = brlen.copy()
    for r in range(rows):
        for o in range(NO):
            if pos[r, o] >= 0:
                want[pos[r, o]] = min(max(max(base[r, o], 1e-6) * np.exp(y[r, o]), 1e-8), 100.0)
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
