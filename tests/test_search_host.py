"""CPU tests of the threshold search's host logic.

The search (FIFO todo queue, visited and good tables keyed by the library's
host topology keys, NNI proposals, final filter by the last lmax + T) runs
with its batch optimiser replaced by the FP64 oracle, so no GPU is needed.
On 6 taxa, with full proposal optimisation from the global maximum, the good
set must be the NNI-connected component of the superlevel set that contains
the start (Methods, "Phylogenetic Topographer"); radius 0 must give a subset.
"""
import numpy as np
import pytest

import synth
from oracle import core as oc
from oracle import topo
from paper_1811_11007_amd import search as S


class OracleSearch(S.ThresholdSearch):
    """The search with each batch optimised tree by tree by the oracle."""

    def __init__(self, data, n, **kw):
        class _Aln:
            n_taxa = n
        super().__init__(None, _Aln(), opt=object(), **kw)
        self.data = data
        self.batches_seen = []

    def _optimize(self, edge_lists, brlen, masks=None, warm_rows=None):
        assert warm_rows is None
        E = 2 * self.n - 3
        lnl, out, ps = [], np.array(brlen, dtype=np.float64), []
        for i, e in enumerate(edge_lists):
            m = None if masks is None else masks[i]
            l, b, p, _ = oc.optimize(self.data, e, out[i * E:(i + 1) * E], mask=m)
            out[i * E:(i + 1) * E] = b
            lnl.append(l)
            ps.append(p)
        self.batches_seen.append(len(edge_lists))
        return np.array(lnl), out, np.array(ps, np.int32)


def brute_force(seed, n=6, sites=150):
    rng = np.random.default_rng(seed)
    e, b = synth.yule_tree(n, rng, mean=0.15)
    aln = synth.make_alignment(e, b, n, sites, rng, alpha=0.5, n_cats=4)
    D = oc.Data.from_alignment(aln)
    tops = topo.all_topologies(n)
    E = 2 * n - 3
    srng = np.random.default_rng(1000 + seed)
    starts = [np.full(E, 0.1)] + [np.exp(srng.normal(-2.5, 1.5, E)) for _ in range(5)]
    opt = np.array([[oc.optimize(D, t, s0)[0] for s0 in starts] for t in tops])
    return D, tops, opt.max(axis=1), opt.min(axis=1)


@pytest.mark.parametrize("seed", [72])
def test_search_logic_against_brute_force(seed):
    n = 6
    D, tops, lnl, low = brute_force(seed, n)
    keys = [topo.key(t, n) for t in tops]
    by_key = dict(zip(keys, tops))
    best = int(np.argmax(lnl))
    lmax = lnl[best]
    T = -20.0
    cut = lmax + T
    assert min(np.min(np.abs(lnl - cut)), np.min(np.abs(low - cut))) > 1e-3
    assert not np.any((low < cut) & (lnl >= cut))
    members = {k for k, l in zip(keys, lnl) if l >= cut}
    comp = {keys[best]}
    todo = [keys[best]]
    while todo:
        k = todo.pop()
        for ne, _ in topo.nni_neighbors(by_key[k], np.full(2 * n - 3, 0.1), n):
            kk = topo.key(ne, n)
            if kk in members and kk not in comp:
                comp.add(kk)
                todo.append(kk)
    start = [(tops[best], np.full(2 * n - 3, 0.1))]
    s = OracleSearch(D, n, threshold=T, radius=-1, batch=16)
    res = s.run(start)
    got = {topo.key(v[1], n) for v in res.good.values()}
    assert got == comp
    assert abs(res.lmax - lmax) < 1e-9 * abs(lmax)
    # the good set's split frequencies and consensus (host library calls)
    splits, freq, newick = S.hls_summary(n, res)
    want = topo.split_frequencies([topo.key(v[1], n) for v in res.good.values()],
                                  [v[0] for v in res.good.values()])
    assert {int(x[0]): f for x, f in zip(splits, freq)} == pytest.approx(want, rel=1e-12)
    assert newick.startswith("(0,") and newick.endswith(");")
    # batches of at most 16 trees; every good topology was visited
    assert max(s.batches_seen) <= 16
    assert res.visited >= len(res.good)
    s0 = OracleSearch(D, n, threshold=T, radius=0, batch=16)
    res0 = s0.run(start)
    got0 = {topo.key(v[1], n) for v in res0.good.values()}
    assert got0 <= comp and keys[best] in got0
    # radius 1 optimises three lengths per proposal: never more than the full component
    s1 = OracleSearch(D, n, threshold=T, radius=1, batch=16)
    got1 = {topo.key(v[1], n) for v in s1.run(start).good.values()}
    assert got1 <= comp and keys[best] in got1


def test_search_rejects_bad_settings():
    with pytest.raises(ValueError):
        OracleSearch(None, 6, threshold=1.0)
    with pytest.raises(ValueError):
        OracleSearch(None, 6, threshold=-1.0, radius=-2)
    with pytest.raises(ValueError):
        OracleSearch(None, 6, threshold=-1.0, radius=0.5)


def paper_loop(D, n, start, T, radius):
    """The topographer's loop written out one topology at a time (Methods,
    "Phylogenetic Topographer"): pop the next todo entry; skip it if
    visited; otherwise visit it (optimise every length), update lmax, and if
    its lnL is at least lmax + T, record it as good and, for each of its
    NNI neighbours not yet visited, optimise the lengths within the radius
    of the new edge and push it onto todo when that lnL is at least
    lmax + T.  The good set is filtered by the final lmax + T."""
    from paper_1811_11007_amd import _lib as Lh
    E = 2 * n - 3
    todo = [(topo.key(start[0], n), start[0], start[1])]
    visited, good = set(), {}
    lmax = -np.inf
    head = 0
    while head < len(todo):
        k, e, b = todo[head]
        head += 1
        if k in visited:
            continue
        visited.add(k)
        l, bo, _, _ = oc.optimize(D, e, b)
        lmax = max(lmax, l)
        if l < lmax + T:
            continue
        good[k] = l
        ne, nb, tt = Lh.pt_nni_neighbors(n, np.asarray(e, np.int32), bo)
        for j in range(len(ne)):
            kk = topo.key(ne[j], n)
            if kk in visited:
                continue
            mask = None
            if radius >= 0:
                mask = np.zeros(E, np.uint8)
                mask[sorted(topo.radius_edges(ne[j], n, int(tt[j][0]), radius))] = 1
            lp, bp, _, _ = oc.optimize(D, ne[j], nb[j], mask=mask)
            if lp >= lmax + T:
                todo.append((kk, ne[j], bp))
    return {k for k, l in good.items() if l >= lmax + T}


@pytest.mark.parametrize("radius", [0, 1])
def test_search_matches_the_papers_loop(radius):
    """One topology per batch, the batched search gives the good set of the
    loop written out step by step; in particular a neighbour rejected from
    one parent's lengths can still be queued from a later parent's."""
    n = 6
    rng = np.random.default_rng(73)
    e, b = synth.yule_tree(n, rng, mean=0.15)
    aln = synth.make_alignment(e, b, n, 150, rng, alpha=0.5, n_cats=4)
    D = oc.Data.from_alignment(aln)
    start = (e, np.full(2 * n - 3, 0.1))
    T = -6.0
    want = paper_loop(D, n, start, T, radius)
    s = OracleSearch(D, n, threshold=T, radius=radius, batch=1)
    got = {topo.key(v[1], n) for v in s.run([start]).good.values()}
    assert got == want


class WarmOracleSearch(OracleSearch):
    """The oracle search with a stand-in warm start: the five touched lengths
    of a retried proposal start at their values in the proposal's fully
    optimised tree (what a perfect network would predict)."""

    def __init__(self, data, n, **kw):
        super().__init__(data, n, **kw)
        self.warm = object()  # only its presence matters to the host loop
        self.warm_calls = 0

    def _optimize(self, edge_lists, brlen, masks=None, warm_rows=None):
        b = np.array(brlen, dtype=np.float64)
        if warm_rows is not None:
            self.warm_calls += 1
            E = 2 * self.n - 3
            _, pos, _ = warm_rows
            for i, e in enumerate(edge_lists):
                full = oc.optimize(self.data, e, b[i * E:(i + 1) * E])[1]
                b[pos[i]] = full[pos[i] - i * E]
        return super()._optimize(edge_lists, b, masks, None)


def test_warm_retry_of_near_misses_only_adds():
    """The warm start retries proposals the cold start's partial optimum
    leaves within warm_margin below the gate.  From the global maximum
    (lmax fixed from the first visit) the gate never changes, so every
    proposal the cold search queues, the warm search queues too: its good
    set contains the cold search's, and nothing outside the NNI component
    of the superlevel set; here the stand-in network's retries add good
    topologies that the cold radius-0 gate missed."""
    n = 6
    D, tops, lnl, _ = brute_force(72, n)
    keys = [topo.key(t, n) for t in tops]
    best = int(np.argmax(lnl))
    T = -20.0
    start = [(tops[best], np.full(2 * n - 3, 0.1))]
    cold = OracleSearch(D, n, threshold=T, radius=0, batch=16).run(start)
    got_c = {topo.key(v[1], n) for v in cold.good.values()}
    members = {k for k, l in zip(keys, lnl) if l >= lnl[best] + T}
    s = WarmOracleSearch(D, n, threshold=T, radius=0, batch=16, warm_margin=40.0)
    res = s.run(start)
    got_w = {topo.key(v[1], n) for v in res.good.values()}
    print("cold good", len(got_c), "warm good", len(got_w), "component", len(members),
          "retried", res.warm_tried, "passed", res.warm_passed)
    assert got_c <= got_w <= members
    assert res.warm_tried > 0 and s.warm_calls > 0
    assert 0 < res.warm_passed <= res.warm_tried
    assert len(got_w) > len(got_c)
    assert abs(res.lmax - cold.lmax) < 1e-9 * abs(cold.lmax)
