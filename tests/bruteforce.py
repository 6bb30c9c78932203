"""Brute-force tree likelihood by explicit summation over ancestral states.

This is the definition of the likelihood written out (no pruning): for every
assignment of states to the internal nodes, the probability of the root
state times the transition probability along every edge, summed, averaged
over the rate categories.  Transition matrices come from scipy's matrix
exponential, so nothing here is shared with the oracle's arithmetic.
Exponential in the number of internal nodes: use for n <= 6.
"""
import itertools

import numpy as np
from scipy.linalg import expm


def loglik(edges, brlen, tips, weights, Q, freqs, cat_rates):
    edges = np.asarray(edges)
    n = tips.shape[0]
    if n == 2:
        root, internal = 0, []
    else:
        root, internal = n, list(range(n, 2 * n - 2))
    n_nodes = 2 if n == 2 else 2 * n - 2
    adj = [[] for _ in range(n_nodes)]
    for e, (a, b) in enumerate(edges.tolist()):
        adj[a].append((b, e))
        adj[b].append((a, e))
    oriented = []  # (parent, child, edge) away from the root
    stack, seen = [root], {root}
    while stack:
        v = stack.pop()
        for c, e in adj[v]:
            if c not in seen:
                seen.add(c)
                oriented.append((v, c, e))
                stack.append(c)
    K = len(cat_rates)
    mats = [[expm(np.asarray(Q) * brlen[e] * r) for e in range(len(edges))]
            for r in cat_rates]
    total = 0.0
    for p in range(tips.shape[1]):
        L = 0.0
        for Pm in mats:
            for assign in itertools.product(range(4), repeat=len(internal)):
                state = dict(zip(internal, assign))
                if n == 2:
                    # root is leaf 0: sum over its allowed states
                    acc = 0.0
                    for x0 in range(4):
                        if not (tips[0, p] >> x0) & 1:
                            continue
                        acc += freqs[x0] * sum(Pm[0][x0, j] for j in range(4)
                                               if (tips[1, p] >> j) & 1)
                    L += acc / K
                    continue
                prob = freqs[state[root]]
                for (par, ch, e) in oriented:
                    xs = state[par]
                    if ch < n:
                        prob *= sum(Pm[e][xs, j] for j in range(4) if (tips[ch, p] >> j) & 1)
                    else:
                        prob *= Pm[e][xs, state[ch]]
                L += prob / K
        total += weights[p] * np.log(L)
    return total
