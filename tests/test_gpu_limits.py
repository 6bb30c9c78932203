"""GPU tests at the documented size limits, against the FP64 oracle.

- Branch optimisation accepts up to 32768 patterns per alignment and refuses
  more with PT_EUNSUPPORTED; the likelihood has no such limit.
- Transition matrices held in LDS must fit the device's LDS per block: the
  paper's largest inputs (67 taxa, Methods, "Data and Run-time
  Parameters") with four rate categories are evaluated, optimised and
  differentiated in both precisions; a tree far beyond any LDS (150 taxa,
  eight categories: about 300 KB of FP64 matrices) is refused for
  optimisation, while its lnL either matches the oracle or is refused.
"""
import numpy as np
import pytest

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc

pytestmark = pytest.mark.gpu

PT_EUNSUPPORTED = -4


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


E4 = np.array([[0, 4], [1, 4], [4, 5], [2, 5], [3, 5]], np.int32)
RATES, FREQS = np.array([1.0, 2.0, 1.0, 1.0, 2.0, 1.0]), np.array([0.3, 0.2, 0.2, 0.3])


def wide_alignment(P, seed):
    """4 taxa, P simulated sites kept uncompressed as patterns of weight 1
    (repeated columns are valid patterns)."""
    rng = np.random.default_rng(seed)
    states = synth.simulate(E4, np.full(5, 0.2), 4, RATES, FREQS, 0.5, P, rng)
    tips = synth.TIP_CODE[states.astype(np.int64)]
    return np.ascontiguousarray(tips, np.uint8), np.ones(P)


@pytest.mark.parametrize("P", [32768, 32769])
def test_pattern_limit_of_optimisation(ctx, P):
    say("pattern limit", P)
    tips, w = wide_alignment(P, 90 + P % 7)
    A = pt.Alignment(ctx, tips, w, RATES, FREQS, 0.5, 4)
    e = E4
    b = np.full(5, 0.1)
    D = oc.Data(tips, w, RATES, FREQS, 0.5, 4)
    l = pt.pt_batch_loglik(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)
    want = oc.loglik(D, e, b)
    assert abs(l[0] - want) <= 1e-6 * abs(want)
    if P > 32768:
        with pytest.raises(pt.PTError) as ei:
            pt.pt_batch_optimize_branches(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)
        assert ei.value.code == PT_EUNSUPPORTED
        return
    lo, _, _, st = pt.pt_batch_optimize_branches(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)
    wo = oc.optimize(D, e, b)[0]
    assert st[0] == 0
    assert abs(lo[0] - wo) <= 1e-6 * abs(wo)


def test_67_taxa_four_categories(ctx):
    """The paper's largest taxon count: lnL on both passes, full optimisation
    in both precisions and the gradient, against the oracle."""
    import torch
    rng = np.random.default_rng(92)
    n = 67
    e, b = synth.yule_tree(n, rng, mean=0.05)
    aln = synth.make_alignment(e, b, n, 600, rng, alpha=0.5, n_cats=4)
    A = pt.Alignment.from_synth(ctx, aln)
    D = oc.Data.from_alignment(aln)
    ne, nb, _ = pt.pt_nni_neighbors(n, e, b)
    pick = [0, 64, 127]
    T = pt.Trees([ne[i] for i in pick])
    lens = np.concatenate([nb[i] for i in pick])
    want = np.array([oc.loglik(D, ne[i], nb[i]) for i in pick])
    dev = torch.device("cuda:0")
    for prec in (pt.PT_FP64, pt.PT_FP32):
        for path in (pt.PT_LOGLIK_REGISTERS, pt.PT_LOGLIK_STORED):
            plan = pt.Plan(ctx, [A], T, pt.PT_PLAN_LOGLIK, prec)
            plan.set_loglik_path(path)
            d_b = torch.tensor(lens, dtype=torch.float64, device=dev)
            d_l = torch.zeros(len(pick), dtype=torch.float64, device=dev)
            plan.loglik(d_b, d_l)
            torch.cuda.synchronize()
            got = d_l.cpu().numpy()
            plan.close()
            say("67 taxa lnL prec", prec, "path", path, "max abs", np.max(np.abs(got - want)))
            if prec == pt.PT_FP64 or path == pt.PT_LOGLIK_REGISTERS:
                assert np.max(np.abs(got - want) / np.abs(want)) < 1e-11
            else:
                assert np.max(np.abs(got - want)) < 1e-4
    wo = np.array([oc.optimize(D, ne[i], nb[i])[0] for i in pick])
    for prec in (pt.PT_FP64, pt.PT_FP32):
        lo, _, _, st = pt.pt_batch_optimize_branches(ctx, [A], T, lens, precision=prec)
        say("67 taxa optimum prec", prec, "vs oracle", lo - wo)
        assert np.all(st == 0)
        if prec == pt.PT_FP64:
            assert np.max(np.abs(lo - wo) / np.abs(wo)) < 1e-6
        else:
            assert np.max(np.abs(lo - wo)) < 1e-4
    _, g, _ = pt.pt_batch_branch_grad(ctx, [A], T, lens, pt.PT_FP64)
    gw = np.concatenate([oc.gradient(D, ne[i], nb[i])[1] for i in pick])
    assert np.max(np.abs(g - gw) / np.maximum(1.0, np.abs(gw))) < 1e-7


def test_lds_limit(ctx):
    """150 taxa with eight categories: the FP64 matrices (297 edges x 8 x 128
    bytes, about 300 KB) exceed any LDS, so optimisation is refused; the lnL
    runs on the register-resident pass where the device's LDS holds its
    stack, and is otherwise refused, never wrong."""
    rng = np.random.default_rng(93)
    n = 150
    e, b = synth.yule_tree(n, rng, mean=0.05)
    aln = synth.make_alignment(e, b, n, 200, rng, alpha=0.5, n_cats=8)
    A = pt.Alignment.from_synth(ctx, aln)
    for prec in (pt.PT_FP64, pt.PT_FP32):
        with pytest.raises(pt.PTError) as ei:
            pt.pt_batch_optimize_branches(ctx, [A], pt.Trees([e]), b, precision=prec)
        assert ei.value.code == PT_EUNSUPPORTED
    want = oc.loglik(oc.Data.from_alignment(aln), e, b)
    try:
        got = pt.pt_batch_loglik(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)[0]
    except pt.PTError as err:
        assert err.code == PT_EUNSUPPORTED, err
        say("150 taxa x 8 categories lnL refused:", err)
        return
    say("150 taxa x 8 categories lnL", got, "oracle", want)
    assert abs(got - want) <= 1e-11 * abs(want)


def balanced_tree(n_leaves, rng, mean=0.1):
    """Perfectly balanced unrooted tree on a power of two leaves: pairs joined
    level by level, the two halves joined by edge 0.  The likelihood's
    register program is rooted on edge 0, so it needs log2(n) - 1 stack
    slots, the most any tree of n taxa needs."""
    nodes, nxt, edges = list(range(n_leaves)), n_leaves, []
    while len(nodes) > 2:
        up = []
        for i in range(0, len(nodes), 2):
            edges += [(nodes[i], nxt), (nodes[i + 1], nxt)]
            up.append(nxt)
            nxt += 1
        nodes = up
    e = np.array([(nodes[0], nodes[1])] + edges, np.int32)
    return e, rng.exponential(mean, size=len(e))


def test_register_stack_depths(ctx):
    """The register-resident lnL keeps a program's stack in registers up to
    four slots and in LDS beyond: balanced trees of 32 taxa (four slots) and
    64 taxa (five), and Yule trees, against the oracle in one batch."""
    rng = np.random.default_rng(95)
    for n in (32, 64):
        e, b = balanced_tree(n, rng)
        ey, by = synth.yule_tree(n, rng, mean=0.1)
        aln = synth.make_alignment(e, b, n, 400, rng, alpha=0.5, n_cats=4)
        D = oc.Data.from_alignment(aln)
        A = pt.Alignment.from_synth(ctx, aln)
        want = np.array([oc.loglik(D, e, b), oc.loglik(D, ey, by)])
        T = pt.Trees([e, ey])
        for batch in ([0, 1], [0], [1]):
            Tb = pt.Trees([[e, ey][i] for i in batch])
            lens = np.concatenate([[b, by][i] for i in batch])
            for prec in (pt.PT_FP64, pt.PT_FP32):
                got = pt.pt_batch_loglik(ctx, [A], Tb, lens, precision=prec)
                say("balanced/yule", n, "batch", batch, "prec", prec, "rel", np.abs(got - want[batch]) / np.abs(want[batch]))
                assert np.all(np.abs(got - want[batch]) <= 1e-11 * np.abs(want[batch]))
        del T
