"""GPU tests of the stored pass's and the gradient's tile sizes
(pt_plan_set_tile_patterns, pt_plan_autotune_tiles).

Every tile size must give the oracle's likelihood (stored oracle values of
the C3 starting lengths) and the oracle's gradient (stored C4 gradients), in
both precisions, over graph replays; the sizes agree with each other up to
the order of the per-tile sums; the autotuner keeps one of them, and a later
plan of the same shape class starts with it.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_1811_11007_amd as pt
from synth import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FP64_REL = 1e-6
FP32_ABS = 1e-4


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def test_stored_pass_at_every_tile_size(ctx):
    """lnL of 128 C3 topologies (32 from each alignment) by the stored pass
    at 64, 128 and 256 patterns per tile, against the oracle."""
    alns, trees, lens, idx = workloads.c3_inputs()
    g = json.load(open(os.path.join(GOLDEN, "c3_batch512.json")))
    pick = [i for i in range(512) if i % 128 < 32]
    off = np.concatenate([[0], np.cumsum([len(t) for t in trees])])
    want = np.asarray(g["start_lnl"])[pick]
    A = [pt.Alignment.from_synth(ctx, a) for a in alns]
    T = pt.Trees([trees[i] for i in pick], idx[pick])
    dev = torch.device("cuda:0")
    b = torch.tensor(np.concatenate([lens[off[i]:off[i + 1]] for i in pick]), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    for prec in (pt.PT_FP64, pt.PT_FP32):
        plan = pt.Plan(ctx, A, T, pt.PT_PLAN_LOGLIK, prec)
        plan.set_loglik_path(pt.PT_LOGLIK_STORED)
        got = {}
        for pats in (64, 128, 256, 64):
            plan.set_tile_patterns(pats)
            assert plan.tile_patterns() == pats
            l = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
            with torch.cuda.stream(stream):
                plan.set_graphs(True)
                for _ in range(2):  # the second call replays the captured graph
                    l.zero_()
                    plan.loglik(b, l, stream=stream)
                stream.synchronize()
            got[pats] = l.cpu().numpy()
            err = np.abs(got[pats] - want)
            say("stored pass prec %d, %d patterns per tile: max |dlnL| %.3g" % (prec, pats, err.max()))
            if prec == pt.PT_FP64:
                assert np.max(err / np.abs(want)) < 1e-11
            else:
                assert err.max() < FP32_ABS
        for pats in (64, 128):
            assert np.max(np.abs(got[pats] - got[256]) / np.abs(got[256])) < 1e-12
        plan.close()
    with pytest.raises(pt.PTError) as ei:
        plan = pt.Plan(ctx, A, T, pt.PT_PLAN_LOGLIK, pt.PT_FP64)
        try:
            plan.set_tile_patterns(96)
        finally:
            plan.close()
    assert ei.value.code == -1


def test_gradient_at_every_tile_size_and_autotuned(ctx):
    """Gradients of 64 C4 trees at every tile size against the oracle
    gradient; the autotuner's choice gives the same, and a new plan of the
    same shape class starts with it."""
    aln, tops, lens = workloads.c4_inputs()
    g = json.load(open(os.path.join(GOLDEN, "c4_grad256.json")))
    pick = list(range(0, 256, 4))
    wl = np.asarray(g["lnl"])[pick]
    wg = np.asarray(g["grad"])[pick]
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees([tops[i] for i in pick])
    dev = torch.device("cuda:0")
    b = torch.tensor(lens[pick].ravel(), dtype=torch.float64, device=dev)
    for prec in (pt.PT_FP64, pt.PT_FP32):
        plan = pt.Plan(ctx, [A], T, pt.PT_PLAN_GRAD, prec)
        res = {}
        for pats in (64, 128, 256):
            plan.set_tile_patterns(pats)
            l = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
            gr = torch.zeros(T.n_edges, dtype=torch.float64, device=dev)
            plan.grad(b, l, gr)
            torch.cuda.synchronize()
            res[pats] = (l.cpu().numpy(), gr.cpu().numpy().reshape(len(pick), 97))
            e = np.max(np.abs(res[pats][1] - wg) / np.maximum(1.0, np.abs(wg)))
            say("gradient prec %d, %d patterns per tile: max err %.3g" % (prec, pats, e))
            assert e < (1e-7 if prec == pt.PT_FP64 else 1e-3)
            if prec == pt.PT_FP64:
                assert np.max(np.abs(res[pats][0] - wl) / np.abs(wl)) < 1e-11
            else:
                assert np.max(np.abs(res[pats][0] - wl)) < FP32_ABS
        best = plan.autotune_tiles(b)
        assert best in (64, 128, 256) and plan.tile_patterns() == best
        say("autotuned patterns per tile (prec %d): %d" % (prec, best))
        l = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
        gr = torch.zeros(T.n_edges, dtype=torch.float64, device=dev)
        plan.grad(b, l, gr)
        torch.cuda.synchronize()
        assert np.array_equal(gr.cpu().numpy().reshape(len(pick), 97), res[best][1])
        plan.close()
        again = pt.Plan(ctx, [A], T, pt.PT_PLAN_GRAD, prec)
        assert again.tile_patterns() == best
        again.close()


def test_few_categories_at_every_tile_size(ctx):
    """The stored pass and the gradient with one and two rate categories
    (their own tile kernel instantiations, each requesting its update's
    matrices ahead: 8 and 16 lanes of 16 bytes per edge), at 64, 128 and 256
    patterns per tile with ragged last tiles, in both precisions, against
    the oracle."""
    import synth
    from oracle import core as oc
    rng = np.random.default_rng(97)
    dev = torch.device("cuda:0")
    for K in (1, 2):
        for n, sites in ((12, 700), (30, 450)):
            e0, b0 = synth.yule_tree(n, rng, mean=0.08)
            aln = synth.make_alignment(e0, b0, n, sites, rng, alpha=0.7, n_cats=K)
            D = oc.Data.from_alignment(aln)
            A = pt.Alignment.from_synth(ctx, aln)
            tops = [e0] + [synth.yule_tree(n, rng, mean=0.08)[0] for _ in range(3)]
            lens = [b0 * rng.uniform(0.6, 1.4, size=len(b0)) for _ in tops]
            want = [oc.gradient(D, t, l) for t, l in zip(tops, lens)]
            wl = np.array([w[0] for w in want])
            wg = np.concatenate([w[1] for w in want])
            T = pt.Trees(tops)
            b = torch.tensor(np.concatenate(lens), dtype=torch.float64, device=dev)
            for prec in (pt.PT_FP64, pt.PT_FP32):
                pl = pt.Plan(ctx, [A], T, pt.PT_PLAN_LOGLIK, prec)
                pl.set_loglik_path(pt.PT_LOGLIK_STORED)
                pg = pt.Plan(ctx, [A], T, pt.PT_PLAN_GRAD, prec)
                for pats in (64, 128, 256):
                    pl.set_tile_patterns(pats)
                    pg.set_tile_patterns(pats)
                    l = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
                    pl.loglik(b, l)
                    lg = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
                    gg = torch.zeros_like(b)
                    pg.grad(b, lg, gg)
                    torch.cuda.synchronize()
                    got, gl, gr = l.cpu().numpy(), lg.cpu().numpy(), gg.cpu().numpy()
                    eg = np.max(np.abs(gr - wg) / np.maximum(1.0, np.abs(wg)))
                    say("K", K, "n", n, "prec", prec, "tile", pats, "lnL", np.max(np.abs(got - wl)),
                        "grad lnL", np.max(np.abs(gl - wl)), "grad", eg)
                    if prec == pt.PT_FP64:
                        assert np.max(np.abs(got - wl) / np.abs(wl)) < FP64_REL
                        assert np.max(np.abs(gl - wl) / np.abs(wl)) < FP64_REL
                        assert eg < 1e-7
                    else:
                        assert np.max(np.abs(got - wl)) < FP32_ABS
                        assert np.max(np.abs(gl - wl)) < FP32_ABS
                        assert eg < 1e-3
                pl.close()
                pg.close()
