"""Pins of the CPU oracle to mathematics it does not compute itself.

Each test checks the oracle against something independent of its own
arithmetic: closed forms, library routines (scipy), brute-force summation
over ancestral states, invariants of the model, or exact combinatorics.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import brentq
from scipy.sparse.csgraph import shortest_path
from scipy.special import gammainc, gammaincinv

import synth
from oracle import core as oc
from oracle import topo
from tests import bruteforce

PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def scipy_gamma_rates(alpha, K):
    """Category means of Gamma(alpha, rate alpha) over K equal quantiles."""
    cuts = [gammaincinv(alpha, i / K) for i in range(1, K)]
    cum = [0.0] + [gammainc(alpha + 1.0, y) for y in cuts] + [1.0]
    return np.array([K * (cum[i + 1] - cum[i]) for i in range(K)])


def rand_model(seed):
    rng = np.random.default_rng(seed)
    return synth.gtr_params(rng)


# ----------------------------------------------------------------- model

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rate_matrix_invariants(seed):
    rates, freqs = rand_model(seed)
    Q = oc.rate_matrix(rates, freqs)
    assert np.allclose(Q.sum(axis=1), 0.0, atol=1e-15)
    # time reversibility
    D = np.diag(freqs)
    assert np.allclose(D @ Q, (D @ Q).T, atol=1e-15)
    # one expected substitution per unit time
    assert abs(-np.dot(freqs, np.diag(Q)) - 1.0) < 1e-14
    # off-diagonals proportional to exchangeability times target frequency
    ratios = [Q[i, j] / (r * freqs[j]) for r, (i, j) in zip(rates, PAIRS)]
    ratios += [Q[j, i] / (r * freqs[i]) for r, (i, j) in zip(rates, PAIRS)]
    assert np.ptp(ratios) < 1e-13 * np.mean(ratios)


@pytest.mark.parametrize("t", [0.0, 1e-8, 0.01, 0.3, 2.0, 40.0])
def test_pmatrix_jc_closed_form(t):
    Q = oc.rate_matrix(np.ones(6), np.full(4, 0.25))
    P, _, _ = oc.pmatrix(Q, t)
    e = math.exp(-4.0 * t / 3.0)
    want = np.full((4, 4), 0.25 - 0.25 * e)
    np.fill_diagonal(want, 0.25 + 0.75 * e)
    assert np.max(np.abs(P - want)) < 1e-14


@pytest.mark.parametrize("seed", [3, 4])
@pytest.mark.parametrize("t", [1e-6, 0.05, 0.7, 5.0, 100.0])
def test_pmatrix_vs_scipy(seed, t):
    rates, freqs = rand_model(seed)
    Q = oc.rate_matrix(rates, freqs)
    P, dP, d2P = oc.pmatrix(Q, t)
    ref = expm(Q * t)
    assert np.max(np.abs(P - ref)) < 1e-13
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
    # derivatives against central differences of scipy's exponential
    h = 1e-5
    fd1 = (expm(Q * (t + h)) - expm(Q * (t - h))) / (2 * h)
    assert np.max(np.abs(dP - fd1)) < 1e-8
    h = 1e-3   # second differences: roundoff ~ eps/h^2, truncation ~ h^2
    fd2 = (expm(Q * (t + h)) - 2 * ref + expm(Q * (t - h))) / (h * h)
    assert np.max(np.abs(d2P - fd2)) < 1e-5


def test_chapman_kolmogorov():
    rates, freqs = rand_model(5)
    Q = oc.rate_matrix(rates, freqs)
    a, _, _ = oc.pmatrix(Q, 0.13)
    b, _, _ = oc.pmatrix(Q, 0.29)
    c, _, _ = oc.pmatrix(Q, 0.42)
    assert np.max(np.abs(a @ b - c)) < 1e-14


@pytest.mark.parametrize("a", [0.1, 0.5, 1.0, 3.0, 20.0])
@pytest.mark.parametrize("x", [1e-3, 0.3, 1.0, 4.0, 30.0])
def test_incomplete_gamma_vs_scipy(a, x):
    assert abs(oc.gammp(a, x) - gammainc(a, x)) < 1e-13


@pytest.mark.parametrize("alpha", [0.05, 0.5, 1.0, 2.7, 50.0])
@pytest.mark.parametrize("K", [2, 4, 8])
def test_gamma_rates_vs_scipy(alpha, K):
    r = oc.gamma_rates(alpha, K)
    assert np.max(np.abs(r - scipy_gamma_rates(alpha, K))) < 1e-10
    assert abs(r.mean() - 1.0) < 1e-12
    assert np.all(np.diff(r) > 0)


def test_gamma_rates_limits():
    assert oc.gamma_rates(0.5, 1)[0] == 1.0
    assert np.max(np.abs(oc.gamma_rates(1e6, 4) - 1.0)) < 2e-3


# ------------------------------------------------------------ likelihood

def small_case(n, seed, K=4, sites=60, jc=False, mean=0.15):
    rng = np.random.default_rng(seed)
    edges, brlen = synth.random_tree(n, rng, mean=mean)
    aln = synth.make_alignment(edges, brlen, n, sites, rng, alpha=0.7, n_cats=K, jc=jc)
    return edges, brlen, aln


def brute(edges, brlen, aln):
    Q = oc.rate_matrix(aln.rates, aln.freqs)
    cats = scipy_gamma_rates(aln.alpha, aln.n_cats) if aln.n_cats > 1 else [1.0]
    return bruteforce.loglik(edges, brlen, aln.tips, aln.weights, Q, aln.freqs, cats)


@pytest.mark.parametrize("n,seed,K,jc", [(2, 1, 1, True), (2, 2, 4, False), (3, 3, 4, False),
                                          (4, 4, 1, False), (4, 5, 4, False), (5, 6, 4, False),
                                          (5, 7, 1, True)])
def test_pruning_vs_bruteforce(n, seed, K, jc):
    edges, brlen, aln = small_case(n, seed, K=K, jc=jc)
    want = brute(edges, brlen, aln)
    got = oc.loglik(oc.Data.from_alignment(aln), edges, brlen)
    assert abs(got - want) <= 1e-12 * abs(want)


def test_bruteforce_ambiguous_codes():
    edges, brlen, aln = small_case(5, 8, K=2)
    tips = aln.tips.copy()
    tips[1, ::3] = 15          # gap / N
    tips[3, 1::4] = 1 | 4      # purine
    aln.tips = tips
    want = brute(edges, brlen, aln)
    got = oc.loglik(oc.Data.from_alignment(aln), edges, brlen)
    assert abs(got - want) <= 1e-12 * abs(want)


def test_config_c1_bruteforce_all_topologies():
    """5 taxa x 200 sites, JC69, every one of the 15 topologies."""
    rng = np.random.default_rng(1)
    edges, brlen = synth.random_tree(5, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 5, 200, rng, n_cats=1, jc=True)
    D = oc.Data.from_alignment(aln)
    for top in synth.all_topologies(5):
        bl = rng.exponential(0.1, size=7)
        want = brute(top, bl, aln)
        assert abs(oc.loglik(D, top, bl) - want) <= 1e-12 * abs(want)


def test_pulley_principle():
    rng = np.random.default_rng(11)
    edges, brlen = synth.yule_tree(12, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 12, 300, rng)
    D = oc.Data.from_alignment(aln)
    vals = [oc.loglik(D, edges, brlen, at_edge=e) for e in range(len(edges))]
    vals += [oc.loglik_node(D, edges, brlen, root=v) for v in range(12, 22)]
    assert np.ptp(vals) <= 1e-12 * abs(vals[0])


def test_long_branch_limit():
    """All lengths huge: leaves independent, L_p = prod_leaves pi_x."""
    rng = np.random.default_rng(12)
    edges, _ = synth.random_tree(9, rng)
    aln = synth.make_alignment(edges, np.full(15, 0.2), 9, 100, rng, n_cats=1)
    D = oc.Data.from_alignment(aln)
    got = oc.loglik(D, edges, np.full(15, 800.0))
    state = np.log2(aln.tips).astype(int)
    want = float(np.sum(aln.weights * np.log(aln.freqs[state]).sum(axis=0)))
    assert abs(got - want) <= 1e-12 * abs(want)


def test_zero_lengths():
    rng = np.random.default_rng(13)
    edges, _ = synth.random_tree(6, rng)
    tips = np.array([[1, 2, 8, 1]] * 6, dtype=np.uint8)
    rates, freqs = rand_model(13)
    D = oc.Data(tips, [1.0, 2.0, 3.0, 1.0], rates, freqs, 0.5, 4)
    got = oc.loglik(D, edges, np.zeros(9))
    want = 1.0 * math.log(freqs[0]) + 2 * math.log(freqs[1]) + 3 * math.log(freqs[3]) + math.log(freqs[0])
    assert abs(got - want) < 1e-12
    tips2 = tips.copy()
    tips2[2, 0] = 4
    D2 = oc.Data(tips2, [1.0, 2.0, 3.0, 1.0], rates, freqs, 0.5, 4)
    assert oc.loglik(D2, edges, np.zeros(9)) == -math.inf


def test_compression_invariance():
    rng = np.random.default_rng(14)
    n, S = 10, 400
    edges, brlen = synth.yule_tree(n, rng, mean=0.1)
    rates, freqs = synth.gtr_params(rng)
    states = synth.simulate(edges, brlen, n, rates, freqs, 0.5, S, rng)
    tips, w = synth.compress(states)
    assert tips.shape[1] < S and w.sum() == S
    full = synth.TIP_CODE[states]
    a = oc.loglik(oc.Data(tips, w, rates, freqs, 0.5, 4), edges, brlen)
    b = oc.loglik(oc.Data(full, np.ones(S), rates, freqs, 0.5, 4), edges, brlen)
    assert abs(a - b) <= 1e-12 * abs(b)


def test_scaling_exact_when_not_needed():
    rng = np.random.default_rng(15)
    edges, brlen = synth.yule_tree(27, rng)
    aln = synth.make_alignment(edges, brlen, 27, 500, rng)
    D = oc.Data.from_alignment(aln)
    assert oc.loglik(D, edges, brlen, scaling=True) == pytest.approx(
        oc.loglik(D, edges, brlen, scaling=False), rel=1e-13)


def test_scaling_rescues_underflow():
    """600 taxa on huge branches: every L_p is near 0.25^600 ~ 1e-361, below
    the double range.  With scaling the exact long-branch value comes out."""
    n = 600
    rng = np.random.default_rng(16)
    edges, _ = synth.random_tree(n, rng)
    E = len(edges)
    tips = synth.TIP_CODE[rng.integers(0, 4, size=(n, 3))]
    freqs = np.full(4, 0.25)
    D = oc.Data(tips, np.ones(3), np.ones(6), freqs, 1.0, 1)
    want = 3 * n * math.log(0.25)
    got = oc.loglik(D, edges, np.full(E, 200.0), scaling=True)
    assert abs(got - want) <= 1e-11 * abs(want)
    assert oc.loglik(D, edges, np.full(E, 200.0), scaling=False) == -math.inf


# ------------------------------------------------------------ derivatives

def test_edge_derivatives_vs_central_differences():
    rng = np.random.default_rng(17)
    edges, brlen = synth.yule_tree(9, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 9, 300, rng)
    D = oc.Data.from_alignment(aln)
    h = 1e-5
    for e in range(len(edges)):
        l0, d1, d2 = oc.edge_derivs(D, edges, brlen, e)
        bp, bm = brlen.copy(), brlen.copy()
        bp[e] += h
        bm[e] -= h
        lp, lm = oc.loglik(D, edges, bp), oc.loglik(D, edges, bm)
        fd1 = (lp - lm) / (2 * h)
        fd2 = (lp - 2 * l0 + lm) / (h * h)
        assert abs(d1 - fd1) <= 1e-6 * max(1.0, abs(d1))
        _, d1p, _ = oc.edge_derivs(D, edges, bp, e)
        _, d1m, _ = oc.edge_derivs(D, edges, bm, e)
        assert abs(d2 - (d1p - d1m) / (2 * h)) <= 1e-5 * max(1.0, abs(d2))
        assert abs(d2 - fd2) <= 2e-2 * max(1.0, abs(d2))


def test_gradient_all_edges():
    rng = np.random.default_rng(18)
    edges, brlen = synth.yule_tree(8, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 8, 200, rng)
    D = oc.Data.from_alignment(aln)
    l, g, hd = oc.gradient(D, edges, brlen)
    assert l == pytest.approx(oc.loglik(D, edges, brlen), rel=1e-14)
    for e in range(len(edges)):
        _, d1, d2 = oc.edge_derivs(D, edges, brlen, e)
        assert g[e] == d1 and hd[e] == d2


# ------------------------------------------------------------ optimiser

def jc_two_taxon(N, k):
    """Closed-form ML length and lnL for two JC69 sequences, k mismatches."""
    p = k / N
    x = 1.0 - 4.0 * p / 3.0
    t = -0.75 * math.log(x)
    lnl = N * math.log(0.25) + (N - k) * math.log(0.25 + 0.75 * x) + k * math.log(0.25 - 0.25 * x)
    return t, lnl


def two_taxon_data(N, k):
    tips = np.array([[1] * N, [1] * (N - k) + [2] * k], dtype=np.uint8)
    return oc.Data(tips, np.ones(N), np.ones(6), np.full(4, 0.25), 1.0, 1)


@pytest.mark.parametrize("N,k", [(200, 37), (200, 1), (1000, 300), (50, 20)])
def test_two_taxon_closed_form(N, k):
    t_hat, l_hat = jc_two_taxon(N, k)
    for start in (1e-4, 0.1, 5.0):
        l, b, _, conv = oc.optimize(two_taxon_data(N, k), [[0, 1]], [start])
        assert conv
        assert abs(b[0] - t_hat) < 1e-9
        assert abs(l - l_hat) < 1e-9


def test_two_taxon_example_value():
    """N = 200 sites with 37 differences."""
    t_hat, l_hat = jc_two_taxon(200, 37)
    assert t_hat == pytest.approx(0.21243560653793642, abs=1e-15)
    assert l_hat == pytest.approx(-413.68575471496695, abs=1e-10)


def test_two_taxon_boundaries():
    # no differences: the optimum is the lower bound, where each site has
    # probability (1/4) P_ii(t_min)
    l, b, _, _ = oc.optimize(two_taxon_data(100, 0), [[0, 1]], [0.3])
    assert abs(b[0] - oc.T_MIN) < 1e-15
    pii = 0.25 + 0.75 * math.exp(-4.0 * oc.T_MIN / 3.0)
    assert abs(l - 100 * math.log(0.25 * pii)) < 1e-9
    # p >= 3/4: the likelihood increases towards t = infinity, where every
    # site has probability 1/16; lnL is flat to machine precision far below t_max
    l, b, _, _ = oc.optimize(two_taxon_data(100, 80), [[0, 1]], [0.3])
    assert b[0] > 20.0
    assert abs(l - 100 * math.log(1.0 / 16.0)) < 1e-9


def _kkt(D, edges, b):
    for e in range(len(edges)):
        _, d1, d2 = oc.edge_derivs(D, edges, b, e)
        if b[e] <= oc.T_MIN:
            assert d1 <= 1e-6
        else:
            assert abs(d1) <= 1e-5
            assert d2 < 0


@pytest.mark.parametrize("n,seed", [(4, 20), (5, 21), (8, 22)])
def test_optimum_kkt_and_local_max(n, seed):
    edges, brlen, aln = small_case(n, seed, sites=300, mean=0.1)
    D = oc.Data.from_alignment(aln)
    l, b, _, conv = oc.optimize(D, edges, brlen)
    assert conv
    _kkt(D, edges, b)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        pert = np.maximum(b * np.exp(rng.normal(0, 0.01, size=len(b))), oc.T_MIN)
        assert oc.loglik(D, edges, pert) <= l + 1e-9


def _golden_section_ascent(D, edges, b, sweeps=60):
    """Independent optimiser: 1-D golden-section search per edge on log t."""
    b = b.copy()
    g = (math.sqrt(5) - 1) / 2
    for _ in range(sweeps):
        for e in range(len(b)):
            def f(x):
                bb = b.copy()
                bb[e] = math.exp(x)
                return oc.loglik(D, edges, bb)
            lo, hi = math.log(oc.T_MIN), math.log(5.0)
            c, d = hi - g * (hi - lo), lo + g * (hi - lo)
            fc, fd = f(c), f(d)
            for _ in range(80):
                if fc > fd:
                    hi, d, fd = d, c, fc
                    c = hi - g * (hi - lo)
                    fc = f(c)
                else:
                    lo, c, fc = c, d, fd
                    d = lo + g * (hi - lo)
                    fd = f(d)
            b[e] = math.exp(0.5 * (lo + hi))
    return oc.loglik(D, edges, b), b


def test_optimum_vs_golden_section():
    edges, brlen, aln = small_case(5, 23, K=4, sites=200, mean=0.1)
    D = oc.Data.from_alignment(aln)
    l, b, _, _ = oc.optimize(D, edges, brlen)
    lg, bg = _golden_section_ascent(D, edges, brlen, sweeps=25)
    assert abs(l - lg) < 1e-6
    assert np.max(np.abs(b - bg) / np.maximum(b, 1e-3)) < 1e-3


# --------------------------------------------- MAP lengths (exponential prior)
#
# With an Exponential(rate) prior on every length the optimiser maximises
# lnL + sum_e (log rate - rate * t_e) (Methods, "Phylogenetic Topographer":
# the optional branch-length prior; the paper's runs use rate 10).

def jc_two_taxon_dlnl(N, k, t):
    """d lnL / dt of two JC69 sequences with k mismatches, written out."""
    x = math.exp(-4.0 * t / 3.0)
    return -(N - k) * x / (0.25 + 0.75 * x) + k * (x / 3.0) / (0.25 - 0.25 * x)


def jc_two_taxon_lnl(N, k, t):
    x = math.exp(-4.0 * t / 3.0)
    return N * math.log(0.25) + (N - k) * math.log(0.25 + 0.75 * x) + k * math.log(0.25 - 0.25 * x)


@pytest.mark.parametrize("N,k,rate", [(200, 37, 10.0), (1000, 300, 1.0), (100, 80, 10.0), (200, 1, 50.0)])
def test_two_taxon_map_closed_form(N, k, rate):
    """The MAP length solves d lnL / dt = rate; brentq on the written-out
    derivative finds it independently.  With k/N >= 3/4 the ML length is
    unbounded but the MAP length is finite."""
    t_star = brentq(lambda t: jc_two_taxon_dlnl(N, k, t) - rate, 1e-9, 50.0, xtol=1e-15, rtol=1e-15)
    obj_star = jc_two_taxon_lnl(N, k, t_star) + math.log(rate) - rate * t_star
    for start in (1e-4, 0.1, 5.0):
        l, b, _, conv = oc.optimize(two_taxon_data(N, k), [[0, 1]], [start], prior_rate=rate)
        assert conv
        assert abs(b[0] - t_star) < 1e-9 * max(1.0, t_star)
        assert abs(l - obj_star) < 1e-9 * abs(obj_star)


def test_two_taxon_map_lower_bound():
    # no mismatches: lnL falls with t, so the prior keeps t at the lower bound
    l, b, _, _ = oc.optimize(two_taxon_data(100, 0), [[0, 1]], [0.3], prior_rate=10.0)
    assert abs(b[0] - oc.T_MIN) < 1e-15
    assert abs(l - (jc_two_taxon_lnl(100, 0, oc.T_MIN) + math.log(10.0) - 10.0 * oc.T_MIN)) < 1e-9


@pytest.mark.parametrize("n,seed,rate", [(5, 25, 10.0), (8, 26, 3.0)])
def test_map_optimum_kkt(n, seed, rate):
    edges, brlen, aln = small_case(n, seed, sites=300, mean=0.1)
    D = oc.Data.from_alignment(aln)
    obj, b, _, conv = oc.optimize(D, edges, brlen, prior_rate=rate)
    assert conv
    assert obj == pytest.approx(oc.loglik(D, edges, b) + len(b) * math.log(rate) - rate * b.sum(), abs=1e-9)
    for e in range(len(b)):
        _, d1, d2 = oc.edge_derivs(D, edges, b, e)
        if b[e] <= oc.T_MIN:
            assert d1 - rate <= 1e-6
        else:
            assert abs(d1 - rate) <= 1e-5
            assert d2 < 0
    # the prior shortens the tree, and a vanishing rate gives the ML lengths
    _, bm, _, _ = oc.optimize(D, edges, brlen)
    assert b.sum() < bm.sum()
    _, b0, _, _ = oc.optimize(D, edges, brlen, prior_rate=1e-12)
    assert np.max(np.abs(b0 - bm)) < 1e-7


def test_mask_only_moves_masked_edges():
    edges, brlen, aln = small_case(7, 24, sites=200)
    D = oc.Data.from_alignment(aln)
    mask = np.zeros(11, np.uint8)
    mask[[2, 5]] = 1
    _, b, _, _ = oc.optimize(D, edges, brlen, mask=mask)
    keep = mask == 0
    assert np.array_equal(b[keep], np.maximum(brlen[keep], oc.T_MIN))
    for e in (2, 5):
        _, d1, _ = oc.edge_derivs(D, edges, b, e)
        assert abs(d1) < 1e-5 or b[e] == oc.T_MIN


# ------------------------------------------------------------ topology

@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_topology_counts(n):
    tops = topo.all_topologies(n)
    assert len(tops) == topo.double_factorial_count(n) == [3, 15, 105, 945, 10395][n - 4]
    assert len({topo.key(t, n) for t in tops}) == len(tops)
    assert {topo.key(t, n) for t in synth.all_topologies(n)} == {topo.key(t, n) for t in tops}


@pytest.mark.parametrize("n,seed", [(4, 1), (6, 2), (9, 3), (27, 4), (64, 5)])
def test_nni_neighbours(n, seed):
    rng = np.random.default_rng(seed)
    edges, brlen = synth.random_tree(n, rng)
    k0 = topo.key(edges, n)
    nb = topo.nni_neighbors(edges, brlen, n)
    keys = [topo.key(e, n) for e, _ in nb]
    assert len(nb) == 2 * (n - 3) == len(set(keys))
    assert k0 not in keys
    # each neighbour differs from the parent by exactly one split
    for k in keys:
        assert len(set(k) ^ set(k0)) == 2
    # symmetry: the parent is a neighbour of each neighbour
    for e, _ in nb[:6]:
        assert k0 in {topo.key(x, n) for x, _ in topo.nni_neighbors(e, brlen, n)}
    # lengths stay with their splits; the new central split takes the old central length
    old = topo.lengths_by_split(edges, brlen, n)
    for e, b in nb:
        new = topo.lengths_by_split(e, b, n)
        assert len(set(new) - set(old)) == 1
        assert sorted(new.values()) == sorted(old.values())
    # the generator's own NNI walk reaches the same neighbour set
    gen = {topo.key(e, n) for e, _ in synth.nni_bfs(edges, brlen, n, 2 * (n - 3))}
    assert gen == set(keys)


def test_key_invariance():
    rng = np.random.default_rng(30)
    n = 12
    edges, _ = synth.random_tree(n, rng)
    k = topo.key(edges, n)
    perm = np.arange(2 * n - 2)
    perm[n:] = n + rng.permutation(n - 2)
    relabelled = perm[edges]
    shuffled = relabelled[rng.permutation(len(edges))]
    flipped = shuffled.copy()
    flipped[::2] = flipped[::2, ::-1]
    assert topo.key(flipped, n) == k


def test_nni_graph_n5():
    tops = topo.all_topologies(5)
    keys = {topo.key(t, 5): t for t in tops}
    degree = {}
    for k, t in keys.items():
        nb = {topo.key(e, 5) for e, _ in topo.nni_neighbors(t, np.ones(7), 5)}
        assert nb <= set(keys)
        degree[k] = len(nb)
    assert set(degree.values()) == {4}
    # connected
    seen, stack = set(), [next(iter(keys))]
    while stack:
        k = stack.pop()
        if k in seen:
            continue
        seen.add(k)
        stack += [topo.key(e, 5) for e, _ in topo.nni_neighbors(keys[k], np.ones(7), 5)]
    assert len(seen) == 15


# ---------------------------------------------------------- radius masks
#
# A 6-taxon caterpillar written out by hand: leaves 0..5, internal 6..9.
CATERPILLAR = [(0, 6), (1, 6), (6, 7), (2, 7), (7, 8), (3, 8), (8, 9), (4, 9), (5, 9)]


@pytest.mark.parametrize("centre,r,want", [
    (4, 0, {4}),                     # radius 0: the new edge alone
    (4, 1, {4, 2, 3}),               # radius 1: the new edge and two neighbours
    (4, 2, {4, 2, 3, 0, 1}),
    (4, 3, {4, 2, 3, 0, 1}),         # u's side holds 3 leaves: 2*3-1 edges
    (6, 1, {6, 4, 5}),
    (6, 2, {6, 4, 5, 2, 3}),
    (6, 3, {6, 4, 5, 2, 3, 0, 1}),
    (2, 1, {2, 0, 1}),
    (0, 1, {0, 1, 2}),               # a pendant edge walks from its internal end
    (4, -1, set(range(9))),
])
def test_radius_edges_by_hand(centre, r, want):
    assert topo.radius_edges(CATERPILLAR, 6, centre, r) == want


@pytest.mark.parametrize("n,seed", [(8, 1), (27, 2)])
def test_radius_edges_invariants(n, seed):
    rng = np.random.default_rng(seed)
    edges, _ = synth.random_tree(n, rng)
    E = 2 * n - 3
    A = np.zeros((2 * n - 2, 2 * n - 2))
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    dist = shortest_path(A, unweighted=True)
    for c in range(E):
        u = edges[c][0] if edges[c][0] >= n else edges[c][1]
        sets = [topo.radius_edges(edges, n, c, r) for r in range(2 * n)]
        assert sets[0] == {c}
        for a, b in zip(sets, sets[1:]):
            assert a <= b
        # radius 1: the centre and the other two edges at u
        at_u = {e for e in range(E) if u in edges[e]}
        assert sets[1] == at_u
        # large radius: the centre plus every edge of the rooted subtree at u,
        # which has 2L - 2 edges for its L leaves (the leaves nearer u than v)
        v = edges[c][1] if u == edges[c][0] else edges[c][0]
        L = int(np.sum(dist[:n, u] < dist[:n, v]))
        assert len(sets[-1]) == 2 * L - 1


# ------------------------------------------------------- split frequencies

def _dfact(m):
    return 1 if m <= 0 else m * _dfact(m - 2)


@pytest.mark.parametrize("n", [5, 6, 7])
def test_split_frequencies_uniform_closed_form(n):
    """With equal likelihoods over all (2n-5)!! topologies, a split with sides
    of a and n-a taxa lies in (2a-3)!! (2(n-a)-3)!! of them (a rooted tree
    on each side)."""
    tops = topo.all_topologies(n)
    keys = [topo.key(t, n) for t in tops]
    freq = topo.split_frequencies(keys, [0.0] * len(keys))
    for s, f in freq.items():
        a = bin(s).count("1")
        assert f == pytest.approx(_dfact(2 * a - 3) * _dfact(2 * (n - a) - 3) / _dfact(2 * n - 5), rel=1e-12)
    # every non-trivial split occurs
    assert len(freq) == 2 ** (n - 1) - 1 - n


def test_split_frequencies_by_hand():
    # two 5-taxon topologies sharing the split {1,2} (bitmask 6), the first
    # with {1,2,3} (14), the second with {1,2,4} (22); weights 3 : 1
    keys = [(6, 14), (6, 22)]
    freq = topo.split_frequencies(keys, [0.0, -math.log(3.0)])
    assert freq == pytest.approx({6: 1.0, 14: 0.75, 22: 0.25}, rel=1e-15)
    assert topo.majority_splits(freq) == {6, 14}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_split_frequency_invariants(seed):
    n = 7
    rng = np.random.default_rng(seed)
    tops = topo.all_topologies(n)
    pick = rng.choice(len(tops), size=40, replace=False)
    keys = [topo.key(tops[i], n) for i in pick]
    lnl = rng.normal(-100.0, 3.0, size=len(keys))
    freq = topo.split_frequencies(keys, lnl)
    assert sum(freq.values()) == pytest.approx(n - 3, rel=1e-12)
    assert all(0.0 < f <= 1.0 + 1e-12 for f in freq.values())
    maj = sorted(topo.majority_splits(freq))
    for x in maj:      # majority splits never conflict: as clades without
        for y in maj:  # taxon 0 they are nested or disjoint
            assert (x & y) == 0 or (x & y) == x or (x & y) == y
    # one dominant topology: its splits, and only they, are in the majority
    lnl2 = np.full(len(keys), -1000.0)
    lnl2[5] = 0.0
    assert topo.majority_splits(topo.split_frequencies(keys, lnl2)) == set(keys[5])


# ------------------------------------------- per-topology Gamma-shape optimum

@pytest.mark.parametrize("seed", [5, 6])
def test_alpha_optimum_against_profile_grid(seed):
    """The joint optimum over lengths and alpha must beat every point of a
    profile-likelihood grid (lengths fully optimised at each fixed alpha,
    with the pinned length optimiser), sit between the grid neighbours of
    the best grid point, and be stationary in alpha and in every length."""
    rng = np.random.default_rng(seed)
    edges, brlen = synth.yule_tree(6, rng, mean=0.1)
    aln = synth.make_alignment(edges, brlen, 6, 400, rng, alpha=0.5, n_cats=4)
    D = oc.Data.from_alignment(aln)
    l, b, a, _ = oc.optimize_alpha(D, edges, brlen, 1.0)
    grid = np.geomspace(0.05, 20.0, 31)
    prof = np.array([oc.optimize(oc.with_alpha(D, g), edges, brlen)[0] for g in grid])
    i = int(np.argmax(prof))
    assert l >= prof[i] - 1e-9
    assert grid[max(i - 1, 0)] <= a <= grid[min(i + 1, len(grid) - 1)]
    h = 1e-4
    dl = (oc.loglik(oc.with_alpha(D, a * math.exp(h)), edges, b) -
          oc.loglik(oc.with_alpha(D, a * math.exp(-h)), edges, b)) / (2 * h)
    assert abs(dl) < 1e-4
    _kkt(oc.with_alpha(D, a), edges, b)
    assert l == pytest.approx(oc.loglik(oc.with_alpha(D, a), edges, b), abs=1e-9)


def test_alpha_irrelevant_without_categories():
    edges, brlen, aln = small_case(5, 27, sites=200, mean=0.1)
    D = oc.Data(aln.tips, aln.weights, aln.rates, aln.freqs, 0.7, 1)
    l, _, a, rounds = oc.optimize_alpha(D, edges, brlen, 0.7)
    assert a == 0.7 and rounds <= 2
    assert l == pytest.approx(oc.optimize(D, edges, brlen)[0], abs=1e-12)
