"""The stored 27-taxon workload: reproducible inputs and a true local maximum.

tests/golden/c2_hillclimb.json is written by tests/golden/make_c2.py, which
calls only the oracle.  These checks re-derive what they can on the CPU.
"""
import json
import os

import numpy as np

import synth
from oracle import core as oc
from oracle import topo

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_hillclimb.json")


def load():
    g = json.load(open(GOLDEN))
    rng = np.random.default_rng(g["seed"])
    e, b = synth.yule_tree(g["n_taxa"], rng, mean=0.05)
    aln = synth.make_alignment(e, b, g["n_taxa"], g["n_sites"], rng, alpha=0.5, n_cats=4)
    return g, aln


def test_generator_reproduces_stored_alignment():
    g, aln = load()
    assert aln.n_patterns == g["n_patterns"]
    assert int(aln.tips.astype(np.int64).sum()) == g["tips_sum"]


def test_neighbours_are_the_nni_set_of_the_base_tree():
    g, _ = load()
    n = g["n_taxa"]
    keys = {tuple(int(x) for x in nb["key"]) for nb in g["neighbours"]}
    ref = {topo.key(e, n) for e, _ in topo.nni_neighbors(np.asarray(g["base_edges"]), np.asarray(g["base_brlen"]), n)}
    assert keys == ref and len(keys) == 2 * (n - 3)


def test_base_tree_is_a_local_maximum():
    g, _ = load()
    assert all(nb["converged"] for nb in g["neighbours"])
    assert max(nb["lnl"] for nb in g["neighbours"]) < g["base_lnl"]


def test_one_stored_optimum_recomputes():
    g, aln = load()
    D = oc.Data.from_alignment(aln)
    nb = g["neighbours"][5]
    l, _, _, _ = oc.optimize(D, np.asarray(nb["edges"]), np.asarray(nb["start_brlen"]))
    assert abs(l - nb["lnl"]) < 1e-9
    assert abs(oc.loglik(D, np.asarray(g["base_edges"]), np.asarray(g["base_brlen"])) - g["base_lnl"]) < 1e-8
