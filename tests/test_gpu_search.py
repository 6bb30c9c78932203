"""GPU tests of the threshold search against brute force on small trees.

For n = 6 taxa the oracle optimises every one of the 105 unrooted topologies
(FP64).  With full optimisation of proposals (radius -1) and the global
maximum as the start, the search's good set must equal the NNI-connected
component, containing the start, of the superlevel set {T : lnL(T) >= lmax + T}
(Methods, "Phylogenetic Topographer": every unvisited neighbour of a good
topology is proposed, and full optimisation judges it exactly).  With radius
0, 1 or 2 (only the lengths near the new edge optimised when proposing) the
good set is a subset of it.

Branch-length likelihoods can have several local optima, and which one an
optimiser reaches depends on its starting lengths.  The oracle therefore
optimises every topology from six starts; a threshold is used only if no
topology's optima straddle it (or lie within 1e-3 of it), so that the
superlevel set does not depend on the starts.
"""
import math

import numpy as np
import pytest

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc
from oracle import topo
from paper_1811_11007_amd.search import ThresholdSearch, hls_summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pt.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def component(start_key, members, n, by_key):
    """NNI-connected component of `members` (oracle keys) containing start_key."""
    seen = {start_key}
    todo = [start_key]
    while todo:
        k = todo.pop()
        e = by_key[k]
        for ne, _ in topo.nni_neighbors(e, np.full(len(e), 0.1), n):
            kk = topo.key(ne, n)
            if kk in members and kk not in seen:
                seen.add(kk)
                todo.append(kk)
    return seen


@pytest.mark.parametrize("seed", [71, 72])
def test_search_equals_superlevel_component(ctx, seed):
    n, sites = 6, 150
    rng = np.random.default_rng(seed)
    e, b = synth.yule_tree(n, rng, mean=0.15)
    aln = synth.make_alignment(e, b, n, sites, rng, alpha=0.5, n_cats=4)
    D = oc.Data.from_alignment(aln)
    tops = topo.all_topologies(n)
    assert len(tops) == 105
    E = 2 * n - 3
    say("search brute force: seed", seed, "oracle over", len(tops), "topologies")
    srng = np.random.default_rng(1000 + seed)
    starts = [np.full(E, 0.1)] + [np.exp(srng.normal(-2.5, 1.5, E)) for _ in range(5)]
    opt = np.array([[oc.optimize(D, t, s0)[0] for s0 in starts] for t in tops])
    lnl = opt.max(axis=1)
    low = opt.min(axis=1)
    keys = [topo.key(t, n) for t in tops]
    by_key = dict(zip(keys, tops))
    best = int(np.argmax(lnl))
    lmax = lnl[best]
    # a threshold with no topology within 1e-3 of its boundary and a
    # non-trivial superlevel set
    T, best_size = None, 0
    for cand in (-4.0, -6.0, -9.0, -13.0, -20.0, -30.0):
        cut = lmax + cand
        gap = min(np.min(np.abs(lnl - cut)), np.min(np.abs(low - cut)))
        straddle = np.any((low < cut) & (lnl >= cut))
        size = int(np.sum(lnl >= cut))
        if gap > 1e-3 and not straddle and best_size < size <= 80:
            T, best_size = cand, size
    assert T is not None
    members = {k for k, l in zip(keys, lnl) if l >= lmax + T}
    comp = component(keys[best], members, n, by_key)
    say("threshold", T, "superlevel", len(members), "component", len(comp))
    A = pt.Alignment.from_synth(ctx, aln)
    start = [(tops[best], np.full(E, 0.1))]
    res = ThresholdSearch(ctx, A, threshold=T, radius=-1, precision=pt.PT_FP64, batch=64).run(start)
    got = {topo.key(v[1], n): v[0] for v in res.good.values()}
    assert set(got) == comp
    assert abs(res.lmax - lmax) <= 1e-6 * abs(lmax)
    delta = 0.0
    for k, l in got.items():
        i = keys.index(k)
        # one of the topology's optima (the search starts from inherited lengths)
        assert low[i] - 1e-6 * abs(l) <= l <= lnl[i] + 1e-6 * abs(l)
        delta = max(delta, abs(l - lnl[i]))
    # HLS summary: split frequencies of the good set against the oracle's
    # from its own optima over the component.  Each weight ratio moves by at
    # most exp(2 delta), which bounds every frequency's error.
    splits, freq, newick = hls_summary(n, res)
    want = topo.split_frequencies(sorted(comp), [lnl[keys.index(k)] for k in sorted(comp)])
    assert {int(s[0]) for s in splits} == set(want)
    bound = math.expm1(2 * delta) + 1e-12
    for s, f in zip(splits, freq):
        assert abs(f - want[int(s[0])]) <= bound
    say("HLS consensus", newick, "max |dlnL|", delta)
    for radius in (0, 1, 2):
        res_r = ThresholdSearch(ctx, A, threshold=T, radius=radius, precision=pt.PT_FP64, batch=64).run(start)
        got_r = {topo.key(v[1], n) for v in res_r.good.values()}
        say("radius", radius, "found", len(got_r), "of", len(comp))
        assert got_r <= comp
        assert keys[best] in got_r
