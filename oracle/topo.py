"""Oracle topology operations in plain Python.  TEST INFRASTRUCTURE ONLY.

* Splits: every edge of an unrooted tree cuts the taxa in two; a split is
  written as the bitmask of the side that does not hold taxon 0.
* Topology key: the sorted tuple of the non-trivial splits (the paper keys
  its hash tables by a canonical string of the topology, Methods,
  "Phylogenetic Topographer"; any canonical form with the same uniqueness
  property serves).
* NNI neighbours: across every internal edge (u, v) with the other
  subtrees {a, b} at u and {c, d} at v, the two rearrangements exchange b
  with c and b with d (Methods, "Phylogenetic Topographer"; 2(n-3) per tree).
* Enumeration: all (2n-5)!! unrooted binary topologies by stepwise
  addition of taxa onto every edge.
* Radius masks: the edges within radius r of a new edge, measured from one
  of its endpoints (Methods, "Phylogenetic Topographer", the radius option;
  r = 0 is the new edge alone, r = 1 adds two neighbouring edges, r = -1 is
  every edge).
* Split frequencies of a high-likelihood set: each topology weighted by its
  maximised likelihood normalised over the set; a split's frequency is the
  summed weight of the topologies holding it (Results, "Split Frequency
  Comparison").  The majority-rule consensus keeps the splits above 1/2.
"""
from __future__ import annotations

import math

import numpy as np


def _adj(edges, n):
    n_nodes = 2 if n == 2 else 2 * n - 2
    adj = [[] for _ in range(n_nodes)]
    for e, (a, b) in enumerate(np.asarray(edges).tolist()):
        adj[a].append((b, e))
        adj[b].append((a, e))
    return adj


def edge_splits(edges, n):
    """Per edge, the leaf bitmask of its side without taxon 0."""
    adj = _adj(edges, n)
    E = len(adj) - 1
    out = [0] * E

    def below(v, parent_edge):
        mask = (1 << v) if (v < n and v != 0) else 0
        for c, e in adj[v]:
            if e == parent_edge:
                continue
            m = below(c, e)
            out[e] = m
            mask |= m
        return mask

    below(0, -1)
    return out


def key(edges, n):
    """Canonical key: sorted non-trivial splits (both sides >= 2 taxa)."""
    ks = [s for s in edge_splits(edges, n)
          if 2 <= bin(s).count("1") <= n - 2]
    return tuple(sorted(ks))


def lengths_by_split(edges, brlen, n):
    """{split: length} for every edge (pendant edges included)."""
    return dict(zip(edge_splits(edges, n), np.asarray(brlen, float).tolist()))


def nni_neighbors(edges, brlen, n):
    """All NNI neighbours as (edges, brlen) pairs; lengths stay with their
    subtrees and the central edge keeps its length."""
    edges = np.asarray(edges, dtype=np.int32)
    adj = _adj(edges, n)
    res = []
    for e, (u, v) in enumerate(edges.tolist()):
        if u < n or v < n:
            continue
        eu = [x for (_, x) in adj[u] if x != e]
        ev = [x for (_, x) in adj[v] if x != e]
        eb = eu[1]
        for ec in ev:
            new = edges.copy()
            new[eb] = [v if x == u else x for x in new[eb].tolist()]
            new[ec] = [u if x == v else x for x in new[ec].tolist()]
            res.append((new, np.asarray(brlen, float).copy()))
    return res


def nni_touched(edges, n):
    """Per NNI neighbour (nni_neighbors order), the five edges it touches:
    the central edge, the edge moved from u, the edge of v it swaps with,
    the edge that stays at u and the edge that stays at v."""
    edges = np.asarray(edges, dtype=np.int32)
    adj = _adj(edges, n)
    out = []
    for e, (u, v) in enumerate(edges.tolist()):
        if u < n or v < n:
            continue
        eu = [x for (_, x) in adj[u] if x != e]
        ev = [x for (_, x) in adj[v] if x != e]
        for k, ec in enumerate(ev):
            out.append((e, eu[1], ec, eu[0], ev[1 - k]))
    return out


def radius_edges(edges, n, centre, r):
    """The set of edges a radius-r proposal optimises.  The selected node u
    is the first endpoint of the centre edge that is an internal node (the
    paper leaves the choice open).  With the centre edge cut out, an edge
    (x, y) on u's side lies at depth 1 + min(dist(u, x), dist(u, y)) and the
    centre edge at depth 0; the edges of depth <= r are optimised."""
    edges = np.asarray(edges).tolist()
    E = len(edges)
    if r == -1:
        return set(range(E))
    u = edges[centre][0] if edges[centre][0] >= n else edges[centre][1]
    if u < n:
        return {centre}
    adj = _adj(edges, n)
    dist = {u: 0}
    frontier = [u]
    while frontier:  # breadth-first distances without the centre edge
        nxt = []
        for x in frontier:
            for y, e in adj[x]:
                if e != centre and y not in dist:
                    dist[y] = dist[x] + 1
                    nxt.append(y)
        frontier = nxt
    out = {centre}
    for e, (x, y) in enumerate(edges):
        if e != centre and x in dist and y in dist and 1 + min(dist[x], dist[y]) <= r:
            out.add(e)
    return out


def nni_features(edges, brlen, n):
    """Warm-start features of every NNI neighbour, from splits alone.

    Per move: log t of the five touched edges (t floored at 1e-6); for the
    four non-central ones, the log leaf count and log(clade length + 1e-3)
    of the clade on their side away from the central edge; and the log of
    the tree length.  The clade of edge x away from the central edge c is
    the side of x that lies wholly on one side of c; its length sums the
    edges one of whose sides lies inside it."""
    edges = np.asarray(edges, dtype=np.int32)
    brlen = np.asarray(brlen, dtype=np.float64)
    full = (1 << n) - 1
    sp = edge_splits(edges, n)
    sides = [(s, full ^ s) for s in sp]
    total = float(brlen.sum())
    rows = []
    for tt in nni_touched(edges, n):
        c, cc = sides[tt[0]]
        f = [np.log(max(brlen[x], 1e-6)) for x in tt]
        cnt, ln = [], []
        for x in tt[1:]:
            clade = [s for s in sides[x] if (s & c) == s or (s & cc) == s]
            assert len(clade) == 1
            F = clade[0]
            inside = sum(brlen[y] for y in range(len(sp))
                         if y != x and any((s & F) == s for s in sides[y]))
            cnt.append(np.log(bin(F).count("1")))
            ln.append(np.log(inside + 1e-3))
        rows.append(f + cnt + ln + [np.log(total)])
    return np.array(rows)


def all_topologies(n):
    """Every unrooted binary topology on n >= 3 taxa (edge lists)."""
    out = []

    def add(edges, leaf, nxt):
        if leaf == n:
            out.append(np.array(edges, dtype=np.int32))
            return
        for i in range(len(edges)):
            a, b = edges[i]
            grown = edges[:i] + [(a, nxt)] + edges[i + 1:] + [(nxt, b), (nxt, leaf)]
            add(grown, leaf + 1, nxt + 1)

    add([(0, n), (1, n), (2, n)], 3, n + 1)
    return out


def double_factorial_count(n):
    """(2n-5)!! for n >= 3."""
    c = 1
    for k in range(3, 2 * n - 4, 2):
        c *= k
    return c


def split_frequencies(keys, lnl):
    """{split: frequency} for topologies given by their keys (tuples of
    splits) and maximised lnL values."""
    lmax = max(lnl)
    weights = [math.exp(l - lmax) for l in lnl]
    total = sum(weights)
    freq = {}
    for k, w in zip(keys, weights):
        for s in k:
            freq[s] = freq.get(s, 0.0) + w / total
    return freq


def majority_splits(freq):
    """The splits of frequency above 1/2."""
    return {s for s, f in freq.items() if f > 0.5}
