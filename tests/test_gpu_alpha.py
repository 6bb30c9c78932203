"""GPU tests of per-topology Gamma-shape optimisation.

The paper can optimise the shape alpha of the Gamma rate distribution for
each visited topology (Methods, "Phylogenetic Topographer").  Each plan tree
has its own model descriptor: pt_plan_set_alpha changes the tree's category
rates, and pt_plan_optimize_alpha alternates batched length optimisation
with a lockstep Brent search over log alpha.  Compared with the FP64 oracle
at each tree's shape and with the oracle's joint optimum: FP64 within 1e-6
relative, FP32 partials within 1e-4 absolute.
"""
import numpy as np
import pytest
import torch

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc

pytestmark = pytest.mark.gpu

FP32_ABS = 1e-4


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def case(seed, n=8, sites=400):
    rng = np.random.default_rng(seed)
    e, b = synth.yule_tree(n, rng, mean=0.08)
    aln = synth.make_alignment(e, b, n, sites, rng, alpha=0.5, n_cats=4)
    ne, nb, _ = pt.pt_nni_neighbors(n, e, b)
    return aln, ne, nb


@pytest.mark.parametrize("precision", [pt.PT_FP64, pt.PT_FP32])
def test_set_alpha_loglik_and_optimum(ctx, precision):
    aln, ne, nb = case(48)
    A = pt.Alignment.from_synth(ctx, aln)
    D = oc.Data.from_alignment(aln)
    k = 6
    alphas = np.array([0.05, 0.2, 0.5, 1.0, 5.0, 50.0])
    dev = torch.device("cuda", 0)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne[:k])), pt.PT_PLAN_LOGLIK | pt.PT_PLAN_OPTIMIZE, precision)
    d_b = torch.tensor(nb[:k].ravel(), dtype=torch.float64, device=dev)
    d_l = torch.zeros(k, dtype=torch.float64, device=dev)
    print("set_alpha precision", precision, flush=True)

    def close(got, want):
        return abs(got - want) < (1e-6 * abs(want) if precision == pt.PT_FP64 else FP32_ABS)

    plan.set_alpha(alphas)
    plan.loglik(d_b, d_l)
    got = d_l.cpu().numpy()
    for i in range(k):
        assert close(got[i], oc.loglik(oc.with_alpha(D, alphas[i]), ne[i], nb[i]))
    # optimisation uses the same per-tree shapes
    plan.optimize(d_b, d_l)
    got = d_l.cpu().numpy()
    for i in range(k):
        assert close(got[i], oc.optimize(oc.with_alpha(D, alphas[i]), ne[i], nb[i])[0])
    # None returns every tree to the alignment's own shape
    d_b.copy_(torch.tensor(nb[:k].ravel(), dtype=torch.float64))
    plan.set_alpha(None)
    plan.loglik(d_b, d_l)
    got = d_l.cpu().numpy()
    for i in range(k):
        assert close(got[i], oc.loglik(D, ne[i], nb[i]))
    plan.close()


@pytest.mark.parametrize("precision", [pt.PT_FP64, pt.PT_FP32])
def test_optimize_alpha_against_oracle(ctx, precision):
    aln, ne, nb = case(49)
    A = pt.Alignment.from_synth(ctx, aln)
    D = oc.Data.from_alignment(aln)
    k = 8
    dev = torch.device("cuda", 0)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne[:k])), pt.PT_PLAN_LOGLIK | pt.PT_PLAN_OPTIMIZE, precision)
    d_b = torch.tensor(nb[:k].ravel(), dtype=torch.float64, device=dev)
    print("optimize_alpha precision", precision, flush=True)
    lnl, alpha, rounds = plan.optimize_alpha(d_b, np.ones(k))
    print("rounds", rounds, "alpha", alpha, flush=True)
    E = ne.shape[1]
    bo = d_b.cpu().numpy().reshape(k, E)
    for i in range(k):
        want, _, wa, _ = oc.optimize_alpha(D, ne[i], nb[i], 1.0)
        if precision == pt.PT_FP64:
            assert abs(lnl[i] - want) < 1e-6 * abs(want)
            assert abs(np.log(alpha[i] / wa)) < 1e-2
        else:
            assert abs(lnl[i] - want) < FP32_ABS
            assert abs(np.log(alpha[i] / wa)) < 5e-2
        # the reported lnL belongs to the returned shape and lengths
        at = oc.loglik(oc.with_alpha(D, alpha[i]), ne[i], bo[i])
        assert abs(lnl[i] - at) < (1e-6 * abs(at) if precision == pt.PT_FP64 else FP32_ABS)
    plan.close()


def test_alpha_errors(ctx):
    aln, ne, nb = case(50, n=6, sites=100)
    A = pt.Alignment.from_synth(ctx, aln)
    dev = torch.device("cuda", 0)
    plan = pt.Plan(ctx, [A], pt.Trees(list(ne[:2])), pt.PT_PLAN_LOGLIK | pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
    d_b = torch.tensor(nb[:2].ravel(), dtype=torch.float64, device=dev)
    for bad in ([1.0, 0.0], [1.0, -2.0], [np.nan, 1.0], [np.inf, 1.0]):
        with pytest.raises(pt.PTError) as ei:
            plan.set_alpha(bad)
        assert ei.value.code == -1
    for kw in (dict(alpha_min=0.0), dict(alpha_max=0.01), dict(tol_alpha=0.0), dict(max_rounds=0)):
        with pytest.raises(pt.PTError):
            plan.optimize_alpha(d_b, np.ones(2), **kw)
    with pytest.raises(pt.PTError):
        plan.optimize_alpha(d_b, [1.0, 500.0])  # start outside the bounds
    only_opt = pt.Plan(ctx, [A], pt.Trees(list(ne[:2])), pt.PT_PLAN_OPTIMIZE, pt.PT_FP64)
    with pytest.raises(pt.PTError):
        only_opt.optimize_alpha(d_b, np.ones(2))
    only_opt.close()
    plan.close()
