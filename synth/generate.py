"""Seeded generators for trees, GTR+Gamma parameters and alignments.

Conventions shared by every consumer of these inputs:

* An unrooted binary tree on ``n`` taxa has ``2n-3`` edges given as an
  ``int32[E][2]`` array of node ids.  Leaves are ``0..n-1`` (alignment rows),
  internal nodes ``n..2n-3``.  Edge orientation and order carry no meaning.
  ``n = 2`` is a single edge ``(0, 1)``.
* Branch lengths are ``float64[E]`` in expected substitutions per site and
  are indexed like the edges.
* Nucleotide states are A, C, G, T = 0..3; a tip code is a 4-bit mask with
  bit ``j`` set when state ``j`` is possible (one-hot for simulated data).
* Exchangeabilities are ordered AC, AG, AT, CG, CT, GT.

Sequences are simulated by the jump process of the continuous-time Markov
chain (exponential waiting times, jumps in proportion to the off-diagonal
rates).  Rate variation across sites draws every site's rate from the
continuous Gamma(alpha, rate alpha) law.  Nothing here evaluates a
transition probability or a likelihood.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TIP_CODE = np.array([1, 2, 4, 8], dtype=np.uint8)
_PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@dataclass
class Alignment:
    """Site patterns of one alignment plus the model it was simulated under."""

    tips: np.ndarray      # uint8 [n_taxa][n_patterns] tip codes
    weights: np.ndarray   # float64 [n_patterns] pattern multiplicities
    rates: np.ndarray     # float64 [6] exchangeabilities
    freqs: np.ndarray     # float64 [4] base frequencies
    alpha: float          # Gamma shape used for inference
    n_cats: int           # number of discrete Gamma categories for inference
    n_sites: int          # columns before compression

    @property
    def n_taxa(self) -> int:
        return int(self.tips.shape[0])

    @property
    def n_patterns(self) -> int:
        return int(self.tips.shape[1])


def _finish(edges, n, rng, mean):
    """Shuffle edge order and orientation, draw iid Exp(mean) lengths."""
    edges = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    perm = rng.permutation(len(edges))
    edges = edges[perm]
    flip = rng.random(len(edges)) < 0.5
    edges[flip] = edges[flip][:, ::-1]
    brlen = rng.exponential(mean, size=len(edges))
    return np.ascontiguousarray(edges), brlen


def yule_tree(n: int, rng: np.random.Generator, mean: float = 0.05):
    """Pure-birth (Yule) topology with the root suppressed; iid Exp lengths."""
    if n < 2:
        raise ValueError("need at least two taxa")
    children: dict[int, list[int]] = {0: []}
    lineages = [0]
    nxt = 1
    while len(lineages) < n:
        i = int(rng.integers(len(lineages)))
        v = lineages[i]
        a, b = nxt, nxt + 1
        nxt += 2
        children[v] = [a, b]
        children[a] = []
        children[b] = []
        lineages[i] = a
        lineages.append(b)
    leaf_ids = rng.permutation(n)
    label: dict[int, int] = {}
    for j, v in enumerate(lineages):
        label[v] = int(leaf_ids[j])
    nxt_internal = n
    for v in sorted(children):
        if v != 0 and children[v]:
            label[v] = nxt_internal
            nxt_internal += 1
    edges = []
    for v in sorted(children):
        if v == 0:
            continue
        for c in children[v]:
            edges.append((label[v], label[c]))
    c1, c2 = children[0]
    edges.append((label[c1], label[c2]))
    return _finish(edges, n, rng, mean)


def random_tree(n: int, rng: np.random.Generator, mean: float = 0.1):
    """Uniformly random unrooted labelled topology by random stepwise addition."""
    if n < 2:
        raise ValueError("need at least two taxa")
    if n == 2:
        return _finish([(0, 1)], n, rng, mean)
    edges = [(0, n), (1, n), (2, n)]
    nxt = n + 1
    for leaf in range(3, n):
        i = int(rng.integers(len(edges)))
        a, b = edges[i]
        m = nxt
        nxt += 1
        edges[i] = (a, m)
        edges.append((m, b))
        edges.append((m, leaf))
    return _finish(edges, n, rng, mean)


def all_topologies(n: int) -> list[np.ndarray]:
    """Every unrooted binary topology on n >= 3 taxa, by stepwise addition."""
    if n < 3:
        return [np.array([[0, 1]], dtype=np.int32)]
    out: list[np.ndarray] = []

    def grow(edges, leaf, nxt):
        if leaf == n:
            out.append(np.array(edges, dtype=np.int32))
            return
        for i in range(len(edges)):
            a, b = edges[i]
            e2 = list(edges)
            e2[i] = (a, nxt)
            e2.append((nxt, b))
            e2.append((nxt, leaf))
            grow(e2, leaf + 1, nxt + 1)

    grow([(0, n), (1, n), (2, n)], 3, n + 1)
    return out


def gtr_params(rng: np.random.Generator):
    """Exchangeabilities ~ Dirichlet(1 x 6), frequencies ~ Dirichlet(10 x 4)."""
    rates = rng.dirichlet(np.ones(6))
    freqs = rng.dirichlet(10.0 * np.ones(4))
    return rates, freqs


def _jump_rates(rates, freqs):
    """Off-diagonal jump rates in units of expected substitutions per site."""
    R = np.zeros((4, 4))
    for r, (i, j) in zip(rates, _PAIRS):
        R[i, j] = r * freqs[j]
        R[j, i] = r * freqs[i]
    mu = float(np.dot(freqs, R.sum(axis=1)))
    return R / mu


def _evolve(states, tau, R, rng):
    out = states.copy()
    remaining = tau.copy()
    exit_rate = R.sum(axis=1)
    cum = np.cumsum(R / exit_rate[:, None], axis=1)
    cum[:, -1] = 1.0
    active = remaining > 0
    while active.any():
        idx = np.nonzero(active)[0]
        wait = rng.exponential(1.0 / exit_rate[out[idx]])
        jump = wait < remaining[idx]
        remaining[idx] -= wait
        j_idx = idx[jump]
        if len(j_idx):
            u = rng.random(len(j_idx))
            out[j_idx] = (u[:, None] >= cum[out[j_idx]]).sum(axis=1)
        active[idx[~jump]] = False
    return out


def simulate(edges, brlen, n, rates, freqs, alpha, n_sites, rng):
    """Simulate an n x n_sites state matrix (int8, states 0..3) on the tree.

    ``alpha=None`` gives every site rate 1; otherwise site rates are drawn
    from Gamma(shape alpha, rate alpha).
    """
    edges = np.asarray(edges)
    R = _jump_rates(np.asarray(rates, float), np.asarray(freqs, float))
    if alpha is None:
        site_rate = np.ones(n_sites)
    else:
        site_rate = rng.gamma(alpha, 1.0 / alpha, size=n_sites)
    n_nodes = 2 if n == 2 else 2 * n - 2
    adj: list[list[tuple[int, int]]] = [[] for _ in range(n_nodes)]
    for e, (a, b) in enumerate(edges):
        adj[a].append((b, e))
        adj[b].append((a, e))
    root = 0 if n == 2 else n
    seq = np.zeros((n_nodes, n_sites), dtype=np.int8)
    seq[root] = rng.choice(4, size=n_sites, p=freqs)
    stack = [(root, -1)]
    while stack:
        v, parent = stack.pop()
        for c, e in adj[v]:
            if c == parent:
                continue
            seq[c] = _evolve(seq[v], brlen[e] * site_rate, R, rng)
            stack.append((c, v))
    return seq[:n]


def compress(states: np.ndarray):
    """Unique columns in first-occurrence order: (tips uint8[n][P], weights)."""
    cols: dict[bytes, int] = {}
    order: list[int] = []
    counts: list[int] = []
    st = np.ascontiguousarray(states.T)
    for s in range(st.shape[0]):
        key = st[s].tobytes()
        j = cols.get(key)
        if j is None:
            cols[key] = len(order)
            order.append(s)
            counts.append(1)
        else:
            counts[j] += 1
    tips = TIP_CODE[states[:, order]]
    return np.ascontiguousarray(tips), np.asarray(counts, dtype=np.float64)


def make_alignment(edges, brlen, n, n_sites, rng, alpha=0.5, n_cats=4,
                   jc=False) -> Alignment:
    """Draw a model (GTR from Dirichlet, or JC69), simulate, compress."""
    if jc:
        rates, freqs = np.ones(6), np.full(4, 0.25)
    else:
        rates, freqs = gtr_params(rng)
    states = simulate(edges, brlen, n, rates, freqs,
                      None if n_cats == 1 else alpha, n_sites, rng)
    tips, w = compress(states)
    return Alignment(tips, w, rates, freqs, alpha, n_cats, n_sites)


# ---------------------------------------------------------------- topologies

def _splits(edges, n):
    """Leaf bitmask of the side of every edge that does not hold leaf 0."""
    n_nodes = 2 if n == 2 else 2 * n - 2
    adj: list[list[tuple[int, int]]] = [[] for _ in range(n_nodes)]
    for e, (a, b) in enumerate(edges):
        adj[int(a)].append((int(b), e))
        adj[int(b)].append((int(a), e))
    below = [0] * n_nodes
    out = [0] * len(edges)
    order, parent_edge = [], {0: -1}
    stack, seen = [0], {0}
    while stack:
        v = stack.pop()
        order.append(v)
        for c, e in adj[v]:
            if c not in seen:
                seen.add(c)
                parent_edge[c] = e
                stack.append(c)
    for v in reversed(order):
        if v < n and v != 0:
            below[v] |= 1 << v
        e = parent_edge[v]
        if e >= 0:
            out[e] = below[v]
            a, b = edges[e]
            p = int(a) if int(b) == v else int(b)
            below[p] |= below[v]
    return out


def topology_id(edges, n) -> frozenset:
    """Set of non-trivial splits; equal for equal unrooted topologies."""
    return frozenset(s for s in _splits(edges, n)
                     if bin(s).count("1") not in (0, 1, n - 1))


def _nni(edges, n):
    """The 2(n-3) NNI rearrangements, each as a new edge array."""
    n_nodes = 2 * n - 2
    inc: list[list[int]] = [[] for _ in range(n_nodes)]
    for e, (a, b) in enumerate(edges):
        inc[int(a)].append(e)
        inc[int(b)].append(e)
    res = []
    for e, (u, v) in enumerate(edges):
        u, v = int(u), int(v)
        if u < n or v < n:
            continue
        eu = sorted(x for x in inc[u] if x != e)
        ev = sorted(x for x in inc[v] if x != e)
        for swap_with in (ev[0], ev[1]):
            new = edges.copy()
            eb = eu[1]
            new[eb] = [v if int(x) == u else int(x) for x in new[eb]]
            new[swap_with] = [u if int(x) == v else int(x) for x in new[swap_with]]
            res.append(new)
    return res


def nni_bfs(edges, brlen, n, count):
    """Breadth-first NNI walk: up to ``count`` distinct topologies other than
    the start, each carrying the lengths inherited edge by edge."""
    start = topology_id(edges, n)
    seen = {start}
    frontier = [(np.asarray(edges, np.int32), np.asarray(brlen, float))]
    out = []
    while frontier and len(out) < count:
        nxt = []
        for ed, bl in frontier:
            for new in _nni(ed, n):
                key = topology_id(new, n)
                if key in seen:
                    continue
                seen.add(key)
                out.append((new, bl.copy()))
                nxt.append((new, bl))
                if len(out) == count:
                    return out
        frontier = nxt
    return out
