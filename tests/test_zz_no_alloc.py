"""GPU test of pt_batch_loglik_noalloc, the likelihood entry point that
allocates no device memory (its per-device workspace is a fixed array of the
library): against pt_batch_loglik on the same inputs, on two calls in a row
(the second smaller, so stale workspace contents would show), and its
refusal of a batch beyond the workspace."""
import numpy as np
import pytest

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc

pytestmark = pytest.mark.gpu


def batch(seed, count, n, sites, K):
    rng = np.random.default_rng(seed)
    e, b = synth.yule_tree(n, rng, mean=0.05)
    aln = synth.make_alignment(e, b, n, sites, rng, alpha=0.5, n_cats=K)
    tops = [e] + [x for x, _ in synth.nni_bfs(e, b, n, count - 1)]
    lens = rng.exponential(0.05, size=(count, 2 * n - 3))
    return aln, tops, lens


def test_noalloc_matches_batch_loglik():
    ctx = pt.Context(0)
    # first call: two alignments of different sizes and category counts
    a1, t1, l1 = batch(301, 40, 40, 1200, 4)
    a2, t2, l2 = batch(302, 24, 17, 500, 2)
    A = [pt.Alignment.from_synth(ctx, a1), pt.Alignment.from_synth(ctx, a2)]
    T = pt.Trees(t1 + t2, [0] * 40 + [1] * 24)
    lens = np.concatenate([l1.ravel(), l2.ravel()])
    for prec in (pt.PT_FP64, pt.PT_FP32):
        want = pt.pt_batch_loglik(ctx, A, T, lens, prec)
        got = pt.pt_batch_loglik_noalloc(ctx, A, T, lens, prec)
        print("no-alloc, 64 trees, prec", prec, "max rel", np.max(np.abs(got - want) / np.abs(want)), flush=True)
        assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12
    D = oc.Data.from_alignment(a1)
    assert abs(got[0] - oc.loglik(D, t1[0], l1[0])) < 1e-10 * abs(got[0])
    # second call, smaller: one alignment, fewer and smaller trees
    a3, t3, l3 = batch(303, 5, 9, 300, 4)
    A3 = [pt.Alignment.from_synth(ctx, a3)]
    T3 = pt.Trees(t3)
    want = pt.pt_batch_loglik(ctx, A3, T3, l3.ravel(), pt.PT_FP64)
    got = pt.pt_batch_loglik_noalloc(ctx, A3, T3, l3.ravel(), pt.PT_FP64)
    print("no-alloc, 5 trees, max rel", np.max(np.abs(got - want) / np.abs(want)), flush=True)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12
    D3 = oc.Data.from_alignment(a3)
    for i in range(5):
        assert abs(got[i] - oc.loglik(D3, t3[i], l3[i])) < 1e-10 * abs(got[i])
    # a batch beyond the 64 MiB workspace: 1200 trees of 64 taxa with four
    # categories need about 1200 x 125 x 4 x 128 bytes of matrices
    a4, t4, l4 = batch(304, 4, 64, 100, 4)
    A4 = [pt.Alignment.from_synth(ctx, a4)]
    T4 = pt.Trees(t4 * 300)
    with pytest.raises(pt.PTError) as ei:
        pt.pt_batch_loglik_noalloc(ctx, A4, T4, np.tile(l4.ravel(), 300), pt.PT_FP64)
    assert ei.value.code == -2 and "no-allocation workspace" in str(ei.value)
    # invalid input is refused before any device work
    with pytest.raises(pt.PTError) as ei:
        pt.pt_batch_loglik_noalloc(ctx, A3, T3, -l3.ravel(), pt.PT_FP64)
    assert ei.value.code == -1
    # the workspace still serves after the refusals
    got = pt.pt_batch_loglik_noalloc(ctx, A3, T3, l3.ravel(), pt.PT_FP64)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12
    ctx.close()
