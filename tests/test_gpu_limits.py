"""GPU tests at the documented size limits, against the FP64 oracle.

- Branch optimisation accepts up to 32768 patterns per alignment and refuses
  more with PT_EUNSUPPORTED; the likelihood has no such limit.
- A tree's transition matrices must fit the 64 KiB cache: with four rate
  categories 64 taxa (125 edges) fit and 65 taxa are refused.
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


def test_edge_category_limit(ctx):
    rng = np.random.default_rng(91)
    for n, ok in ((64, True), (65, False)):
        e, b = synth.yule_tree(n, rng, mean=0.05)
        aln = synth.make_alignment(e, b, n, 200, rng, alpha=0.5, n_cats=4)
        A = pt.Alignment.from_synth(ctx, aln)
        if ok:
            l = pt.pt_batch_loglik(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)
            want = oc.loglik(oc.Data.from_alignment(aln), e, b)
            assert abs(l[0] - want) <= 1e-6 * abs(want)
        else:
            with pytest.raises(pt.PTError) as ei:
                pt.pt_batch_loglik(ctx, [A], pt.Trees([e]), b, precision=pt.PT_FP64)
            assert ei.value.code == PT_EUNSUPPORTED
