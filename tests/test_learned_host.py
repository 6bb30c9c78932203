"""CPU tests of the warm-start network's oracle and of the host features.

The oracle network (numpy FP64) is pinned by central finite differences of
its own loss, by float64 torch autograd as an independent implementation,
and by Adam's bias-corrected closed form under a constant gradient.  The
library's host feature extractor is checked against the oracle's
split-based definition and against invariants of the clades.
"""
import math

import numpy as np
import pytest

import paper_1811_11007_amd as pt
import synth
from oracle import mlp as om
from oracle import topo

NI, NH, NO = 14, 16, 5


def rand_net(seed, ni=NI, nh=NH, no=NO, rows=37):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, om.n_params(ni, nh, no))
    x = rng.normal(0, 1, (rows, ni))
    t = rng.normal(0, 1, (rows, no))
    return p, x, t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_gradient_matches_central_differences(seed):
    p, x, t = rand_net(seed)
    g = om.gradient(x, t, p, NI, NH, NO)
    h = 1e-6
    for i in np.random.default_rng(seed).choice(p.size, 60, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (om.loss(x, t, p + e, NI, NH, NO) - om.loss(x, t, p - e, NI, NH, NO)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_oracle_matches_torch_autograd_float64():
    import torch
    p, x, t = rand_net(5, rows=23)
    W1, b1, W2, b2 = [torch.tensor(a.copy(), requires_grad=True) for a in om.unpack(p, NI, NH, NO)]
    X, Tt = torch.tensor(x), torch.tensor(t)
    y = torch.tanh(X @ W1 + b1) @ W2 + b2
    loss = ((y - Tt) ** 2).mean()
    loss.backward()
    _, yo = om.forward(x, p, NI, NH, NO)
    assert np.max(np.abs(yo - y.detach().numpy())) < 1e-12
    assert abs(om.loss(x, t, p, NI, NH, NO) - loss.item()) < 1e-12
    gt = np.concatenate([W1.grad.numpy().ravel(), b1.grad.numpy(), W2.grad.numpy().ravel(), b2.grad.numpy()])
    assert np.max(np.abs(om.gradient(x, t, p, NI, NH, NO) - gt)) < 1e-12


def test_adam_constant_gradient_closed_form():
    # With the same gradient every step the bias-corrected moments equal g and
    # g^2 exactly, so every step moves each parameter by lr * g / (|g| + eps).
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, 50)
    p = rng.normal(0, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    for step in range(1, 6):
        q, m, v = om.adam_step(p, g, m, v, step, lr, eps=eps)
        assert np.max(np.abs((p - q) - lr * g / (np.abs(g) + eps))) < 1e-15
        p = q


def test_adam_matches_torch_optimizer():
    import torch
    rng = np.random.default_rng(4)
    p0 = rng.normal(0, 1, 30)
    gs = rng.normal(0, 1, (7, 30))
    w = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(30), np.zeros(30)
    for s in range(7):
        opt.zero_grad()
        w.grad = torch.tensor(gs[s])
        opt.step()
        p, m, v = om.adam_step(p, gs[s], m, v, s + 1, 1e-2)
    assert np.max(np.abs(p - w.detach().numpy())) < 1e-12


def test_oracle_unpack_rejects_wrong_size():
    with pytest.raises(ValueError):
        om.unpack(np.zeros(10), NI, NH, NO)


def tree(n, seed):
    rng = np.random.default_rng(seed)
    return synth.yule_tree(n, rng, mean=0.05)


@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (9, 3), (27, 4), (64, 5)])
def test_oracle_features_invariants(n, seed):
    e, b = tree(n, seed)
    F = topo.nni_features(e, b, n)
    assert F.shape == (2 * (n - 3), pt.PT_NNI_FEATURES)
    touched = topo.nni_touched(e, n)
    for row, tt in zip(F, touched):
        # the four clades partition the taxa
        assert round(sum(math.exp(c) for c in row[5:9])) == n
        # clade lengths plus the five touched edges give the tree length
        inside = sum(math.exp(c) - 1e-3 for c in row[9:13])
        assert abs(inside + sum(b[list(tt)]) - b.sum()) < 1e-9
        assert abs(row[13] - math.log(b.sum())) < 1e-12
        assert np.allclose(row[:5], np.log(np.maximum(b[list(tt)], 1e-6)))


def test_oracle_touched_edges_are_the_move():
    # the neighbour differs from its parent exactly in the endpoints of the
    # moved edge and its swap partner
    n = 9
    e, b = tree(n, 7)
    for (ne, _), tt in zip(topo.nni_neighbors(e, b, n), topo.nni_touched(e, n)):
        diff = sorted(set(np.nonzero(np.any(ne != e, axis=1))[0].tolist()))
        assert diff == sorted([tt[1], tt[2]])
        assert set(e[tt[0]].tolist()) == set(ne[tt[0]].tolist())


@pytest.mark.parametrize("n,seed", [(4, 11), (6, 12), (27, 13), (50, 14), (64, 15)])
def test_host_features_match_oracle(n, seed):
    e, b = tree(n, seed)
    b = b.copy()
    b[seed % len(b)] = 0.0  # a zero length exercises the floor
    F = pt.pt_nni_features(n, e, b)
    G = topo.nni_features(e, b, n)
    assert F.dtype == np.float32
    assert np.max(np.abs(F - G)) <= 1e-5 * max(1.0, np.abs(G).max())
    _, _, tt = pt.pt_nni_neighbors(n, e, b)
    assert [tuple(r) for r in tt.tolist()] == [tuple(r) for r in topo.nni_touched(e, n)]


def test_host_features_errors():
    e, b = tree(5, 1)
    with pytest.raises(pt.PTError):
        pt.pt_nni_features(3, e[:3], b[:3])
    bad = e.copy()
    bad[0] = bad[1]
    with pytest.raises(pt.PTError):
        pt.pt_nni_features(5, bad, b)
