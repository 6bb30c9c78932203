"""Host-side tests of the C-ABI library: no device work.

The library must load and export every entry point include/pt.h declares;
model set-up, tree validation and the topology operations run on the host
and are checked against scipy and the oracle's independent topology code.
"""
import math
import os
import re

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import gammainc, gammaincinv

import paper_1811_11007_amd as pt
import synth
from oracle import core as oc
from oracle import topo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 20
    L = pt.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pt.EXPORTS)


def test_no_device_means_a_loud_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pt.PTError):
        pt.Context(0)


def scipy_rates(alpha, K):
    cuts = [gammaincinv(alpha, i / K) for i in range(1, K)]
    cum = [0.0] + [gammainc(alpha + 1.0, y) for y in cuts] + [1.0]
    return np.array([K * (cum[i + 1] - cum[i]) for i in range(K)])


@pytest.mark.parametrize("alpha", [0.05, 0.3, 0.5, 1.0, 4.0, 200.0])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 8])
def test_model_gamma_rates(alpha, K):
    r, _, _, _ = pt.pt_model_info(np.ones(6), np.full(4, 0.25), alpha, K)
    want = [1.0] if K == 1 else scipy_rates(alpha, K)
    assert np.max(np.abs(r - want)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_model_eigensystem_reproduces_expm(seed):
    rng = np.random.default_rng(seed)
    rates, freqs = synth.gtr_params(rng)
    _, U, Ui, lam = pt.pt_model_info(rates, freqs, 0.5, 4)
    Q = oc.rate_matrix(rates, freqs)   # pinned to the GTR definition by the oracle tests
    assert np.max(np.abs(U @ Ui - np.eye(4))) < 1e-13
    for t in (1e-6, 0.01, 0.3, 2.0, 50.0):
        P = U @ np.diag(np.exp(lam * t)) @ Ui
        assert np.max(np.abs(P - expm(Q * t))) < 1e-13


@pytest.mark.parametrize("bad", [
    dict(freqs=[0.3, 0.3, 0.3, 0.3]), dict(freqs=[0.5, 0.5, 0.0, 0.0]),
    dict(rates=[1, 1, 1, 1, 1, -1]), dict(rates=[1, 1, 1, 1, 1, math.nan]),
    dict(alpha=0.0, n_cats=4), dict(alpha=-1.0, n_cats=4), dict(n_cats=0), dict(n_cats=9),
])
def test_model_validation(bad):
    args = dict(rates=np.ones(6), freqs=np.full(4, 0.25), alpha=0.5, n_cats=4)
    args.update(bad)
    with pytest.raises(pt.PTError) as ei:
        pt.pt_model_info(args["rates"], args["freqs"], args["alpha"], args["n_cats"])
    assert ei.value.code == -1


def test_tree_validation():
    rng = np.random.default_rng(5)
    edges, _ = synth.random_tree(7, rng)
    pt.pt_tree_check(7, edges)
    pt.pt_tree_check(2, [[0, 1]])
    pt.pt_tree_check(3, [[0, 3], [1, 3], [3, 2]])
    bad = []
    e = edges.copy(); e[0, 0] = 99; bad.append(e)           # id out of range
    e = edges.copy(); e[0, 1] = e[0, 0]; bad.append(e)      # self loop
    e = edges.copy(); e[1] = e[0]; bad.append(e)            # parallel edge -> degrees off
    e = edges.copy(); e[:, :] = np.where(e == 0, 1, e); bad.append(e)  # leaf of degree 2
    for b in bad:
        with pytest.raises(pt.PTError) as ei:
            pt.pt_tree_check(7, b)
        assert ei.value.code == -1
    # a cycle with every degree right: two disjoint pieces are impossible with
    # 2n-3 edges and correct degrees, so check the connectivity message path
    cyc = np.array([[0, 4], [4, 5], [5, 4], [1, 5], [2, 3]], dtype=np.int32)
    with pytest.raises(pt.PTError):
        pt.pt_tree_check(4, cyc)
    with pytest.raises(pt.PTError):
        pt.pt_tree_check(1, [[0, 0]])


def key_as_ints(k, n):
    W = (n + 63) // 64
    return tuple(sum(int(row[w]) << (64 * w) for w in range(W)) for row in k)


@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (9, 3), (27, 4), (64, 5), (65, 6), (130, 7)])
def test_topology_key_matches_oracle(n, seed):
    rng = np.random.default_rng(seed)
    edges, _ = synth.random_tree(n, rng)
    k = pt.pt_topology_key(n, edges)
    assert key_as_ints(k, n) == topo.key(edges, n)


@pytest.mark.parametrize("n,seed", [(4, 11), (6, 12), (27, 13), (50, 14), (64, 15)])
def test_nni_neighbours_match_oracle(n, seed):
    rng = np.random.default_rng(seed)
    edges, brlen = synth.yule_tree(n, rng)
    oe, ob, ot = pt.pt_nni_neighbors(n, edges, brlen)
    ref = topo.nni_neighbors(edges, brlen, n)
    assert len(ref) == len(oe) == 2 * (n - 3)
    for i, (re_, rb) in enumerate(ref):
        assert np.array_equal(oe[i], re_)
        assert np.array_equal(ob[i], rb)
        # touched: the central edge and the four edges around it
        centre = ot[i][0]
        u, v = edges[centre]
        around = {x for x in range(len(edges)) if x != centre and (u in edges[x] or v in edges[x])}
        assert set(ot[i][1:].tolist()) == around


@pytest.mark.parametrize("n,seed", [(4, 21), (9, 22), (27, 23), (64, 24)])
def test_radius_masks_match_oracle(n, seed):
    rng = np.random.default_rng(seed)
    edges, brlen = synth.yule_tree(n, rng)
    oe, _, ot = pt.pt_nni_neighbors(n, edges, brlen)
    E = 2 * n - 3
    for r in (-1, 0, 1, 2, 3, 2 * n):
        got = pt.pt_radius_masks(n, oe, ot[:, 0], r)
        assert got.shape == (len(oe), E)
        for i in range(len(oe)):
            want = topo.radius_edges(oe[i], n, int(ot[i, 0]), r)
            assert set(np.flatnonzero(got[i]).tolist()) == want
    # every centre of one tree, including pendant edges
    stack = np.repeat(np.asarray(edges, np.int32)[None], E, axis=0)
    got = pt.pt_radius_masks(n, stack, np.arange(E), 2)
    for c in range(E):
        assert set(np.flatnonzero(got[c]).tolist()) == topo.radius_edges(edges, n, c, 2)


def test_radius_masks_reject_bad_input():
    edges, _ = synth.yule_tree(6, np.random.default_rng(0))
    stack = np.asarray(edges, np.int32)[None]
    for centre, r in ((9, 0), (-1, 0), (0, -2)):
        with pytest.raises(pt.PTError) as ei:
            pt.pt_radius_masks(6, stack, [centre], r)
        assert ei.value.code == -1
    bad = stack.copy()
    bad[0, 0] = [0, 0]
    with pytest.raises(pt.PTError):
        pt.pt_radius_masks(6, bad, [0], 1)
    assert pt.pt_radius_masks(6, stack[:0], np.zeros(0, np.int32), 1).shape == (0, 9)


def test_opt_defaults_and_layout():
    """pt_opt as the binding lays it out matches the header (its size and the
    prior_rate default of 0, maximum likelihood); no device is needed."""
    import ctypes
    assert ctypes.sizeof(pt._lib.pt_opt) == 56
    for prec in (pt.PT_FP32, pt.PT_FP64):
        o = pt.opt_default(prec)
        assert o.prior_rate == 0.0 and o.max_passes == 200 and o.t_min == 1e-8


def parse_consensus(newick, n):
    """{clade bitmask without taxon 0: label} of a Newick string rooted at
    taxon 0 with numeric leaves and clade labels, and the leaf set."""
    pos = 0
    clades = {}
    leaves = set()

    def node():
        nonlocal pos
        if newick[pos] == "(":
            pos += 1
            mask = 0
            while True:
                mask |= node()
                if newick[pos] == ",":
                    pos += 1
                    continue
                assert newick[pos] == ")"
                pos += 1
                break
            j = pos
            while pos < len(newick) and newick[pos] not in ",);":
                pos += 1
            if newick[j:pos]:
                clades[mask] = float(newick[j:pos])
            return mask
        j = pos
        while newick[pos] not in ",);":
            pos += 1
        leaf = int(newick[j:pos])
        leaves.add(leaf)
        return 0 if leaf == 0 else 1 << leaf

    node()
    assert newick[pos:] == ";"
    return clades, leaves


@pytest.mark.parametrize("n,seed,count", [(6, 31, 30), (9, 32, 200), (70, 33, 40)])
def test_split_frequencies_and_consensus_match_oracle(n, seed, count):
    rng = np.random.default_rng(seed)
    trees = []
    e, _ = synth.yule_tree(n, rng)
    for _ in range(count):  # a random NNI walk: sets with shared splits
        ne, _, _ = pt.pt_nni_neighbors(n, e)
        e = ne[rng.integers(len(ne))]
        trees.append(e)
    keys = pt.pt_topology_keys(n, np.stack(trees))
    lnl = rng.normal(-5000.0, 2.0, size=count)
    splits, freq = pt.pt_split_frequencies(n, keys, lnl)
    W = (n + 63) // 64
    as_int = [sum(int(r[w]) << (64 * w) for w in range(W)) for r in splits]
    want = topo.split_frequencies([key_as_ints(k, n) for k in keys], lnl)
    assert set(as_int) == set(want)
    for s, f in zip(as_int, freq):
        assert f == pytest.approx(want[s], rel=1e-12, abs=1e-300)
    assert np.all(np.diff(freq) <= 0)
    newick = pt.pt_majority_consensus(n, splits, freq)
    clades, leaves = parse_consensus(newick, n)
    assert leaves == set(range(n))
    assert set(clades) == topo.majority_splits(want)
    for c, lab in clades.items():
        assert abs(lab - want[c]) <= 5e-7


def test_consensus_of_one_topology_and_star():
    n = 8
    e, _ = synth.yule_tree(n, np.random.default_rng(34))
    k = pt.pt_topology_keys(n, np.asarray(e, np.int32)[None])
    splits, freq = pt.pt_split_frequencies(n, k, [-10.0])
    assert np.all(freq == 1.0)
    clades, _ = parse_consensus(pt.pt_majority_consensus(n, splits, freq), n)
    assert set(clades) == set(key_as_ints(k[0], n))
    assert pt.pt_majority_consensus(n, splits, freq * 0.5) == "(0,1,2,3,4,5,6,7);"


def test_hls_summary_rejects_bad_input():
    import ctypes
    n = 6
    tops = synth.all_topologies(n)[:4]
    keys = pt.pt_topology_keys(n, np.stack(tops))
    for bad_lnl in ([0.0, np.nan, 0.0, 0.0], [0.0, np.inf, 0.0, 0.0]):
        with pytest.raises(pt.PTError):
            pt.pt_split_frequencies(n, keys, bad_lnl)
    k0 = keys.copy()
    k0[1, 0, 0] |= 1  # taxon 0 in a split
    with pytest.raises(pt.PTError):
        pt.pt_split_frequencies(n, k0, np.zeros(4))
    # a capacity below the number of distinct splits reports the number needed
    out = np.zeros((2, 1), np.uint64)
    fr = np.zeros(2)
    m = ctypes.c_int32(0)
    rc = pt.lib().pt_split_frequencies(n, 4, keys.ctypes.data_as(ctypes.c_void_p),
                                       np.zeros(4).ctypes.data_as(ctypes.c_void_p), 2, ctypes.byref(m),
                                       out.ctypes.data_as(ctypes.c_void_p), fr.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1 and m.value == len(pt.pt_split_frequencies(n, keys, np.zeros(4))[0])
    # consensus: incompatible splits above 1/2, a trivial split, frequency > 1
    for s, f in (([[6], [10]], [0.6, 0.6]), ([[2]], [0.9]), ([[6]], [1.5])):
        with pytest.raises(pt.PTError):
            pt.pt_majority_consensus(n, np.array(s, np.uint64), f)


def test_enumerated_topologies_have_distinct_keys():
    keys = {key_as_ints(pt.pt_topology_key(7, t), 7) for t in synth.all_topologies(7)}
    assert len(keys) == 945
