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
"""
from __future__ import annotations

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
