"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: FP64 path within 1e-6 relative of the oracle (checked much
tighter where the arithmetic allows); FP32-storage path within 1e-4 absolute
in lnL.  Inputs are seeded synthetic alignments shaped like the workloads:
5 taxa x 200 sites JC69, 27 taxa x 1949 sites GTR+G4, and small uneven
batches spanning several pattern tiles with ragged tails.
"""
import math
import os

import numpy as np
import pytest

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


def case(n, sites, seed, K=4, jc=False, mean=0.05, yule=True):
    rng = np.random.default_rng(seed)
    edges, brlen = (synth.yule_tree if yule else synth.random_tree)(n, rng, mean=mean)
    aln = synth.make_alignment(edges, brlen, n, sites, rng, alpha=0.5, n_cats=K, jc=jc)
    return edges, brlen, aln


def say(*a):
    print(*a, flush=True)


def test_loglik_c1_all_topologies(ctx):
    """5 taxa x 200 sites JC69: every topology, FP64 and FP32."""
    rng = np.random.default_rng(1)
    edges, brlen = synth.random_tree(5, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 5, 200, rng, n_cats=1, jc=True)
    tops = synth.all_topologies(5)
    lens = rng.exponential(0.1, size=(15, 7))
    D = oc.Data.from_alignment(aln)
    want = np.array([oc.loglik(D, t, b) for t, b in zip(tops, lens)])
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees(tops)
    got = pt.pt_batch_loglik(ctx, [A], T, lens.ravel(), pt.PT_FP64)
    say("C1 fp64 max rel", np.max(np.abs(got - want) / np.abs(want)))
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12
    got32 = pt.pt_batch_loglik(ctx, [A], T, lens.ravel(), pt.PT_FP32)
    assert np.max(np.abs(got32 - want)) < FP32_ABS


def test_loglik_c2_shape(ctx):
    edges, brlen, aln = case(27, 1949, 2)
    D = oc.Data.from_alignment(aln)
    want = oc.loglik(D, edges, brlen)
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees([edges])
    g64 = pt.pt_batch_loglik(ctx, [A], T, brlen, pt.PT_FP64)[0]
    g32 = pt.pt_batch_loglik(ctx, [A], T, brlen, pt.PT_FP32)[0]
    say("C2 loglik", want, g64 - want, g32 - want)
    assert abs(g64 - want) <= 1e-11 * abs(want)
    assert abs(g32 - want) <= FP32_ABS


def test_loglik_uneven_batch(ctx):
    """Several alignments, n from 2 to 40, patterns from 1 to ~900, K 1..8."""
    specs = [(2, 50, 1), (3, 300, 4), (4, 1, 2), (9, 700, 3), (17, 257, 8), (40, 1200, 4), (12, 513, 5)]
    alns, cases = [], []
    for i, (n, S, K) in enumerate(specs):
        e, b, a = case(n, S, 100 + i, K=K, mean=0.1)
        alns.append(a)
        cases.append((e, b))
    A = [pt.Alignment.from_synth(ctx, a) for a in alns]
    idx = []
    edges, lens, want = [], [], []
    rng = np.random.default_rng(7)
    for rep in range(3):
        for i, (e, b) in enumerate(cases):
            bb = b * rng.uniform(0.5, 1.5, size=len(b))
            idx.append(i)
            edges.append(e)
            lens.append(bb)
            want.append(oc.loglik(oc.Data.from_alignment(alns[i]), e, bb))
    T = pt.Trees(edges, idx)
    want = np.array(want)
    g64 = pt.pt_batch_loglik(ctx, A, T, np.concatenate(lens), pt.PT_FP64)
    g32 = pt.pt_batch_loglik(ctx, A, T, np.concatenate(lens), pt.PT_FP32)
    say("uneven fp64 max rel", np.max(np.abs(g64 - want) / np.abs(want)), "fp32 max abs", np.max(np.abs(g32 - want)))
    assert np.max(np.abs(g64 - want) / np.abs(want)) < 1e-11
    assert np.max(np.abs(g32 - want)) < FP32_ABS


def test_scaling_fp32_underflow(ctx):
    """64 taxa on very long branches: every L_p ~ 4^-64 = 2^-128, below the
    FP32 range, so FP32 partials only survive through scaling.  Leaves are
    then independent, lnL = sum_p sum_leaves ln pi_x exactly."""
    n = 64
    rng = np.random.default_rng(9)
    edges, _ = synth.random_tree(n, rng)
    tips = synth.TIP_CODE[rng.integers(0, 4, size=(n, 37))]
    freqs = np.array([0.1, 0.2, 0.3, 0.4])
    A = pt.Alignment(ctx, tips, np.ones(37), np.ones(6), freqs, 1.0, 1)
    lens = np.full(len(edges), 200.0)
    want = float(np.sum(np.log(freqs[np.log2(tips).astype(int)])))
    got = pt.pt_batch_loglik(ctx, [A], pt.Trees([edges]), lens, pt.PT_FP32)[0]
    assert abs(got - want) < FP32_ABS, (got, want)
    got = pt.pt_batch_loglik(ctx, [A], pt.Trees([edges]), lens, pt.PT_FP64)[0]
    assert abs(got - want) < 1e-12 * abs(want), (got, want)


def test_optimize_c1(ctx):
    """All 15 five-taxon topologies, full optimisation, FP64 and FP32."""
    rng = np.random.default_rng(1)
    edges, brlen = synth.random_tree(5, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 5, 200, rng, n_cats=1, jc=True)
    D = oc.Data.from_alignment(aln)
    tops = synth.all_topologies(5)
    want = np.array([oc.optimize(D, t, np.full(7, 0.1))[0] for t in tops])
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees(tops)
    l64, b64, ps, st = pt.pt_batch_optimize_branches(ctx, [A], T, np.full(15 * 7, 0.1), precision=pt.PT_FP64)
    say("C1 opt fp64 max rel", np.max(np.abs(l64 - want) / np.abs(want)), "passes", ps)
    assert np.all(st == 0)
    assert np.max(np.abs(l64 - want) / np.abs(want)) < 1e-9
    # reported lnL is the lnL at the reported lengths
    at = pt.pt_batch_loglik(ctx, [A], T, b64, pt.PT_FP64)
    assert np.max(np.abs(at - l64)) < 1e-9
    l32, _, _, st32 = pt.pt_batch_optimize_branches(ctx, [A], T, np.full(15 * 7, 0.1), precision=pt.PT_FP32)
    assert np.max(np.abs(l32 - want)) < FP32_ABS


def test_optimize_c2_neighbours(ctx):
    """27 taxa x 1949 sites GTR+G4: NNI neighbours of the generating tree,
    lengths inherited, full optimisation; a sample against the oracle."""
    edges, brlen, aln = case(27, 1949, 2)
    nb = topo.nni_neighbors(edges, brlen, 27)
    sample = [0, 17, 47]
    D = oc.Data.from_alignment(aln)
    want = np.array([oc.optimize(D, nb[i][0], nb[i][1])[0] for i in sample])
    A = pt.Alignment.from_synth(ctx, aln)
    T = pt.Trees([nb[i][0] for i in sample])
    lens = np.concatenate([nb[i][1] for i in sample])
    l64, _, ps, st = pt.pt_batch_optimize_branches(ctx, [A], T, lens, precision=pt.PT_FP64)
    l32, _, ps32, st32 = pt.pt_batch_optimize_branches(ctx, [A], T, lens, precision=pt.PT_FP32)
    say("C2 opt", want, l64 - want, l32 - want, ps, ps32)
    assert np.max(np.abs(l64 - want) / np.abs(want)) < FP64_REL
    assert np.max(np.abs(l32 - want)) < FP32_ABS


def test_gradient_vs_oracle(ctx):
    edges, brlen, aln = case(20, 800, 4, mean=0.08)
    D = oc.Data.from_alignment(aln)
    lw, gw, hw = oc.gradient(D, edges, brlen)
    A = pt.Alignment.from_synth(ctx, aln)
    l, g, h = pt.pt_batch_branch_grad(ctx, [A], pt.Trees([edges]), brlen, pt.PT_FP64, hess=True)
    say("grad fp64", np.max(np.abs(g - gw)), np.max(np.abs(h - hw)))
    assert abs(l[0] - lw) < 1e-10 * abs(lw)
    assert np.max(np.abs(g - gw) / np.maximum(1, np.abs(gw))) < 1e-8
    assert np.max(np.abs(h - hw) / np.maximum(1, np.abs(hw))) < 1e-7
    l32, g32, _ = pt.pt_batch_branch_grad(ctx, [A], pt.Trees([edges]), brlen, pt.PT_FP32)
    assert np.max(np.abs(g32 - gw) / np.maximum(1, np.abs(gw))) < 1e-3


def test_optimize_c2_full_batch_as_benchmarked(ctx):
    """All 48 neighbours of the stored hill-climbed tree in one plan, in the
    launch configuration the benchmark times (autotuned shape, HIP graph),
    against the oracle optima stored by tests/golden/make_c2.py."""
    import json
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_hillclimb.json")))
    rng = np.random.default_rng(g["seed"])
    e, b = synth.yule_tree(g["n_taxa"], rng, mean=0.05)
    aln = synth.make_alignment(e, b, g["n_taxa"], g["n_sites"], rng, alpha=0.5, n_cats=4)
    n = g["n_taxa"]
    A = pt.Alignment.from_synth(ctx, aln)
    want = {tuple(int(x) for x in nb["key"]): nb["lnl"] for nb in g["neighbours"]}
    ne, nbl, _ = pt.pt_nni_neighbors(n, np.asarray(g["base_edges"], np.int32), np.asarray(g["base_brlen"]))
    W = (n + 63) // 64
    keys = [tuple(sum(int(r[w]) << (64 * w) for w in range(W)) for r in pt.pt_topology_key(n, x)) for x in ne]
    ref = np.array([want[k] for k in keys])
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    for prec, tol in ((pt.PT_FP32, FP32_ABS), (pt.PT_FP64, None)):
        plan = pt.Plan(ctx, [A], pt.Trees(list(ne)), pt.PT_PLAN_OPTIMIZE, prec)
        b0 = torch.tensor(nbl.ravel(), dtype=torch.float64, device=dev)
        bb = torch.empty_like(b0)
        lnl = torch.zeros(len(ne), dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            plan.autotune(b0)
            plan.set_graphs(True)
            for rep in range(3):   # replays of one captured graph
                bb.copy_(b0, non_blocking=True)
                plan.optimize(bb, lnl, stream=stream)
                stream.synchronize()
                got = lnl.cpu().numpy()
                say("C2 batch prec", prec, "rep", rep, "max abs", np.max(np.abs(got - ref)))
                if tol is None:
                    assert np.max(np.abs(got - ref) / np.abs(ref)) < FP64_REL
                else:
                    assert np.max(np.abs(got - ref)) < tol
        plan.close()


@pytest.mark.parametrize("path", ["registers", "stored"])
def test_loglik_paths_uneven_batch(ctx, path):
    """Both lnL passes on one plan over uneven alignments (n 2..40, patterns
    1 to 1200, K 1..8 in one layout, several tiles with ragged tails): the
    register-resident pass (no partial stored, FP64 in either precision) and
    the stored post-order pass."""
    import torch
    specs = [(2, 50, 1), (3, 300, 4), (4, 1, 2), (9, 700, 3), (17, 257, 8), (40, 1200, 4), (12, 513, 5)]
    code = pt.PT_LOGLIK_REGISTERS if path == "registers" else pt.PT_LOGLIK_STORED
    dev = torch.device("cuda:0")
    alns, edges, lens, want, idx = [], [], [], [], []
    rng = np.random.default_rng(70)
    for i, (n, S, k) in enumerate(specs):
        e, b, a = case(n, S, 200 + i, K=k, mean=0.1)
        alns.append(a)
        for rep in range(2):
            bb = b * rng.uniform(0.5, 1.5, size=len(b))
            idx.append(i)
            edges.append(e)
            lens.append(bb)
            want.append(oc.loglik(oc.Data.from_alignment(a), e, bb))
    A = [pt.Alignment.from_synth(ctx, a) for a in alns]
    T = pt.Trees(edges, idx)
    want = np.array(want)
    for prec in (pt.PT_FP64, pt.PT_FP32):
        plan = pt.Plan(ctx, A, T, pt.PT_PLAN_LOGLIK, prec)
        plan.set_loglik_path(code)
        d_b = torch.tensor(np.concatenate(lens), dtype=torch.float64, device=dev)
        d_l = torch.zeros(T.n_trees, dtype=torch.float64, device=dev)
        plan.loglik(d_b, d_l)
        torch.cuda.synchronize()
        got = d_l.cpu().numpy()
        plan.close()
        say(path, "prec", prec, "max abs", np.max(np.abs(got - want)))
        if prec == pt.PT_FP64 or path == "registers":
            assert np.max(np.abs(got - want) / np.abs(want)) < 1e-11
        else:
            assert np.max(np.abs(got - want)) < FP32_ABS


def test_loglik_path_errors(ctx):
    rng = np.random.default_rng(71)
    e, b = synth.yule_tree(6, rng)
    aln = synth.make_alignment(e, b, 6, 50, rng)
    A = pt.Alignment.from_synth(ctx, aln)
    plan = pt.Plan(ctx, [A], pt.Trees([e]), pt.PT_PLAN_LOGLIK, pt.PT_FP64)
    with pytest.raises(pt.PTError) as ei:
        plan.set_loglik_path(7)
    assert ei.value.code == -1
    plan.close()
    plan = pt.Plan(ctx, [A], pt.Trees([e]), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
    with pytest.raises(pt.PTError) as ei:
        plan.set_loglik_path(pt.PT_LOGLIK_STORED)
    assert ei.value.code == -1
    plan.close()
