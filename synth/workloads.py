"""The seeded benchmark and parity workloads, by name.

Each function only draws inputs (alignments, topologies, starting lengths)
with the generators of this package; the library and the oracle both
consume them.  Sizes follow the paper's data range (27 to 67 taxa, about
1000 to 2500 sites; Methods, "Data and Run-time Parameters").
"""
from __future__ import annotations

import numpy as np

from .generate import make_alignment, nni_bfs, yule_tree

# (taxa, sites, seed) of the four uneven alignments of the batching workload
C3_SHAPES = [(27, 1949, 31), (36, 1812, 32), (50, 1133, 33), (64, 1008, 34)]
C3_PER_ALIGNMENT = 128


def c3_inputs():
    """Batching workload: four uneven GTR+G4 alignments (27x1949, 36x1812,
    50x1133, 64x1008 taxa x sites), 128 topologies each from a breadth-first
    NNI walk around the generating tree, lengths inherited from it: 512
    topologies.  Returns (alignments, edge arrays, flat lengths, alignment
    index per topology)."""
    alns, trees, lens, idx = [], [], [], []
    for i, (n, S, seed) in enumerate(C3_SHAPES):
        rng = np.random.default_rng(seed)
        e, b = yule_tree(n, rng, mean=0.05)
        alns.append(make_alignment(e, b, n, S, rng, alpha=0.5, n_cats=4))
        for te, tb in nni_bfs(e, b, n, C3_PER_ALIGNMENT):
            trees.append(te)
            lens.append(tb)
            idx.append(i)
    return alns, trees, np.concatenate(lens), np.array(idx, np.int32)


def c4_inputs(n_trees: int = 256):
    """Gradient workload: 50 taxa x 1500 sites GTR+G4, seed 4; topologies
    from a breadth-first NNI walk around the generating tree, each with its
    own lengths ~ Exp(mean 0.05).  Returns (alignment, edge arrays,
    lengths[n_trees][97])."""
    rng = np.random.default_rng(4)
    e, b = yule_tree(50, rng, mean=0.05)
    aln = make_alignment(e, b, 50, 1500, rng, alpha=0.5, n_cats=4)
    tops = [x for x, _ in nni_bfs(e, b, 50, n_trees)]
    lens = rng.exponential(0.05, size=(n_trees, 97))
    return aln, tops, lens


def c5_alignment(seed: int):
    """Search workload: 64 taxa x 2500 sites GTR+G4 on a Yule tree with
    Exp(mean 0.05) lengths (seed 5 trains the warm-start network, seed 6 is
    held out).  Returns (edges, lengths, alignment)."""
    rng = np.random.default_rng(seed)
    edges, brlen = yule_tree(64, rng, mean=0.05)
    aln = make_alignment(edges, brlen, 64, 2500, rng, alpha=0.5, n_cats=4)
    return edges, brlen, aln


def c5_loglik_trees(seed: int = 6, count: int = 32):
    """Likelihood parity set at the search shape: ``count`` topologies of a
    breadth-first NNI walk around the seed's generating tree, with lengths
    ~ Exp(mean 0.05) drawn from a generator seeded with seed + 1000.
    Returns (alignment, edge arrays, lengths[count][125])."""
    edges, brlen, aln = c5_alignment(seed)
    tops = [x for x, _ in nni_bfs(edges, brlen, 64, count)]
    rng = np.random.default_rng(seed + 1000)
    lens = rng.exponential(0.05, size=(count, 125))
    return aln, tops, lens
