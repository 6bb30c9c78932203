"""GPU tests of the optimisation kernel with several blocks per tree.

For batches too small to fill the device, pt_plan_set_launch splits each
tree's patterns over G blocks whose Newton and lnL sums are combined across
blocks.  Every shape must give the oracle's optima (FP64 within 1e-6
relative, FP32 partials within 1e-4 absolute), converge (status 0, never the
timed-out status 2), and be refused when its blocks could not all be
resident at once.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc
from oracle import topo

pytestmark = pytest.mark.gpu

FP64_REL = 1e-6
FP32_ABS = 1e-4


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def c2_batch():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_hillclimb.json")))
    rng = np.random.default_rng(g["seed"])
    e, b = synth.yule_tree(g["n_taxa"], rng, mean=0.05)
    aln = synth.make_alignment(e, b, g["n_taxa"], g["n_sites"], rng, alpha=0.5, n_cats=4)
    n = g["n_taxa"]
    want = {tuple(int(x) for x in nb["key"]): nb["lnl"] for nb in g["neighbours"]}
    ne, nbl, _ = pt.pt_nni_neighbors(n, np.asarray(g["base_edges"], np.int32), np.asarray(g["base_brlen"]))
    W = (n + 63) // 64
    keys = [tuple(sum(int(r[w]) << (64 * w) for w in range(W)) for r in pt.pt_topology_key(n, x)) for x in ne]
    return aln, ne, nbl, np.array([want[k] for k in keys])


def run_plan(plan, lens, n_trees, replays=2):
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    b0 = torch.tensor(np.ravel(lens), dtype=torch.float64, device=dev)
    bb = torch.empty_like(b0)
    lnl = torch.zeros(n_trees, dtype=torch.float64, device=dev)
    st = torch.zeros(n_trees, dtype=torch.int32, device=dev)
    out = []
    with torch.cuda.stream(stream):
        plan.set_graphs(True)
        for _ in range(replays):
            bb.copy_(b0, non_blocking=True)
            plan.optimize(bb, lnl, None, st, stream=stream)
            stream.synchronize()
            out.append((lnl.cpu().numpy().copy(), st.cpu().numpy().copy(), bb.cpu().numpy().copy()))
    return out


@pytest.mark.parametrize("precision", [pt.PT_FP32, pt.PT_FP64])
def test_c2_batch_split_over_blocks(ctx, precision):
    aln, ne, nbl, ref = c2_batch()
    A = pt.Alignment.from_synth(ctx, aln)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne)), pt.PT_PLAN_OPTIMIZE, precision)
    accepted = []
    for block, groups in ((512, 2), (256, 3), (512, 4), (512, 5), (256, 5), (256, 8), (512, 8)):
        try:
            plan.set_launch(block, groups)
        except pt.PTError as err:
            assert err.code == -4, err
            say("shape", block, groups, "refused:", err)
            continue
        assert plan.launch_shape()[::2] == (block, groups)
        accepted.append((block, groups))
        say("C2 precision", precision, "block", block, "groups", groups)
        for lnl, st, _ in run_plan(plan, nbl, len(ne)):
            assert np.all(st == 0), st
            if precision == pt.PT_FP64:
                assert np.max(np.abs(lnl - ref) / np.abs(ref)) < FP64_REL
            else:
                assert np.max(np.abs(lnl - ref)) < FP32_ABS
    # 48 trees fit with up to 5 blocks each at one block per compute unit
    assert (512, 2) in accepted and (512, 5) in accepted or (256, 5) in accepted
    plan.close()


def test_split_edge_cases(ctx):
    """Shares with no patterns (3 and 4 taxa, 60 sites, 8 blocks), radius-0
    masks, the MAP prior and per-tree Gamma shapes, against the oracle."""
    rng = np.random.default_rng(81)
    for n in (3, 4, 9):
        e, b = synth.random_tree(n, rng, mean=0.1)
        aln = synth.make_alignment(e, b, n, 60, rng, alpha=0.5, n_cats=4)
        A = pt.Alignment.from_synth(ctx, aln)
        D = oc.Data.from_alignment(aln)
        plan = pt.Plan(ctx, [A], pt.Trees([e, e]), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
        plan.set_launch(256, 8)
        say("split edge case n", n, "patterns", aln.n_patterns)
        lnl, st, _ = run_plan(plan, np.concatenate([b, b]), 2, replays=1)[0]
        assert np.all(st == 0)
        want = oc.optimize(D, e, b)[0]
        assert np.max(np.abs(lnl - want)) < FP64_REL * abs(want)
        plan.close()
    # 12 taxa x 500 sites: radius-0 masks, MAP prior, per-tree shapes
    e, b = synth.yule_tree(12, rng, mean=0.08)
    aln = synth.make_alignment(e, b, 12, 500, rng, alpha=0.5, n_cats=4)
    A = pt.Alignment.from_synth(ctx, aln)
    D = oc.Data.from_alignment(aln)
    ne, nb, touched = pt.pt_nni_neighbors(12, e, b)
    k = 6
    mask = pt.pt_radius_masks(12, ne[:k], touched[:k, 0], 0)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne[:k])), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64, mask=mask.ravel())
    plan.set_launch(512, 4)
    lnl, st, _ = run_plan(plan, nb[:k], k, replays=1)[0]
    for i in range(k):
        assert abs(lnl[i] - oc.optimize(D, ne[i], nb[i], mask=mask[i])[0]) < 1e-8 * abs(lnl[i])
    plan.close()
    alphas = np.array([0.1, 0.3, 0.5, 1.0, 2.0, 8.0])
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne[:k])), pt.PT_PLAN_OPTIMIZE | pt.PT_PLAN_LOGLIK, pt.PT_FP32)
    plan.set_launch(512, 5)
    plan.set_alpha(alphas)
    dev = torch.device("cuda:0")
    d_b = torch.tensor(nb[:k].ravel(), dtype=torch.float64, device=dev)
    d_l = torch.zeros(k, dtype=torch.float64, device=dev)
    o = pt.opt_default(pt.PT_FP32)
    o.prior_rate = 10.0
    plan.optimize(d_b, d_l, opt=o)
    got = d_l.cpu().numpy()
    for i in range(k):
        want = oc.optimize(oc.with_alpha(D, alphas[i]), ne[i], nb[i], prior_rate=10.0)[0]
        assert abs(got[i] - want) < FP32_ABS
    plan.close()


def test_split_refused_when_not_resident(ctx):
    rng = np.random.default_rng(82)
    e, b = synth.yule_tree(6, rng, mean=0.1)
    aln = synth.make_alignment(e, b, 6, 100, rng, alpha=0.5, n_cats=4)
    A = pt.Alignment.from_synth(ctx, aln)
    plan = pt.Plan(ctx, [A], pt.Trees([e] * 600), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
    before = plan.launch_shape()
    for block, groups in ((512, 8), (256, 9), (256, 0)):
        with pytest.raises(pt.PTError) as ei:
            plan.set_launch(block, groups)
        assert ei.value.code == -4
        assert plan.launch_shape() == before
    plan.close()


def test_relaxed_steps_reach_the_oracle_optimum(ctx):
    """From a tree's second pass on the kernel over-relaxes edge steps above
    tol_t; the fixed point must still be the maximum the oracle's plain
    coordinate steps reach.  At tight tolerances every C2 neighbour's FP64
    lnL matches the stored oracle optimum far inside the default bar."""
    aln, ne, nbl, ref = c2_batch()
    A = pt.Alignment.from_synth(ctx, aln)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne)), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
    plan.set_launch(256, 4)
    o = pt.opt_default(pt.PT_FP64)
    o.tol_lnl, o.tol_t, o.tol_newton, o.max_passes = 1e-10, 1e-7, 1e-11, 500
    dev = torch.device("cuda:0")
    b = torch.tensor(np.ravel(nbl), dtype=torch.float64, device=dev)
    lnl = torch.zeros(len(ne), dtype=torch.float64, device=dev)
    ps = torch.zeros(len(ne), dtype=torch.int32, device=dev)
    st = torch.zeros(len(ne), dtype=torch.int32, device=dev)
    plan.optimize(b, lnl, ps, st, opt=o)
    torch.cuda.synchronize()
    l, p, s = lnl.cpu().numpy(), ps.cpu().numpy(), st.cpu().numpy()
    say("tight FP64: max |dlnL| %.2e, passes mean %.1f max %d" % (np.max(np.abs(l - ref)), p.mean(), p.max()))
    assert np.all(s == 0), s
    assert np.max(np.abs(l - ref)) < 1e-7
    plan.close()


def test_timed_out_waits_fall_back_to_one_block_per_tree(ctx):
    """With the cross-block wait limit forced down to a few clocks from the
    host (every wait stays bounded, so every kernel still ends), a plan call
    on trees split over several blocks reports status 2 and NaN for the trees
    whose waits ran out, and the synchronous call re-runs its chunk with one
    block per tree and returns the oracle's optima with status 0."""
    aln, ne, nbl, ref = c2_batch()
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees(list(ne))
    ctx.set_group_wait(8)
    try:
        plan = pt.Plan(ctx, [A], T, pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
        plan.set_launch(256, 4)
        lnl, st, _ = run_plan(plan, nbl, len(ne), replays=1)[0]
        broken = st == 2
        say("forced time-outs: %d of %d trees status 2" % (broken.sum(), len(ne)))
        assert np.all((st == 0) | broken)
        assert np.all(np.isnan(lnl[broken]))
        plan.close()
        for prec, ok in ((pt.PT_FP64, lambda l: np.max(np.abs(l - ref) / np.abs(ref)) < FP64_REL),
                         (pt.PT_FP32, lambda l: np.max(np.abs(l - ref)) < FP32_ABS)):
            l, b, ps, s = pt.pt_batch_optimize_branches(ctx, [A], T, np.ravel(nbl), precision=prec)
            assert np.all(s == 0), s
            assert ok(l)
    finally:
        ctx.set_group_wait(0)
    l, b, ps, s = pt.pt_batch_optimize_branches(ctx, [A], T, np.ravel(nbl), precision=pt.PT_FP64)
    assert np.all(s == 0) and np.max(np.abs(l - ref) / np.abs(ref)) < FP64_REL
