"""ctypes binding of the C oracle (pt_oracle.c).  TEST INFRASTRUCTURE ONLY.

Each function follows the definition stated in pt_oracle.c: tree
log-likelihood by Felsenstein pruning with exact per-pattern scaling, edge
derivatives by re-rooting, and coordinate-wise safeguarded Newton
optimisation of branch lengths (the paper, Methods, "Phylogenetic
Topographer": visiting a topology optimises its branch lengths to maximise
the likelihood).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Defaults of the oracle optimiser (the paper leaves them to its likelihood
# library; these are far tighter than any parity tolerance).
T_MIN, T_MAX = 1e-8, 100.0
TOL_LNL, TOL_T, TOL_NEWTON = 1e-10, 1e-9, 1e-12
MAX_PASSES, MAX_NEWTON = 500, 100


def build(force: bool = True) -> str:
    """Compile pt_oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        up = ctypes.POINTER(ctypes.c_uint8)
        c_int, c_d = ctypes.c_int, ctypes.c_double
        L.or_rate_matrix.argtypes = [dp, dp, dp]
        L.or_expm.argtypes = [dp, dp]
        L.or_pmatrix.argtypes = [dp, c_d, dp, dp, dp]
        L.or_gammp.argtypes = [c_d, c_d]
        L.or_gammp.restype = c_d
        L.or_gamma_rates.argtypes = [c_d, c_int, dp]
        common = [c_int, ip, dp, c_int, up, dp, dp, dp, c_d, c_int]
        L.or_loglik_at.argtypes = common + [c_int, c_int, dp]
        L.or_loglik_node.argtypes = common + [c_int, c_int, dp]
        L.or_edge_derivs.argtypes = common + [c_int, dp, dp, dp]
        L.or_gradient.argtypes = common + [dp, dp, dp]
        L.or_optimize.argtypes = [c_int, ip, dp, up, c_int, up, dp, dp, dp, c_d, c_int,
                                  c_d, c_d, c_d, c_d, c_d, c_int, c_int, c_d,
                                  dp, ip, ip]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _u(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check(rc):
    if rc == -1:
        raise ValueError("oracle: invalid argument")
    if rc == -2:
        raise MemoryError("oracle: out of memory")
    if rc:
        raise RuntimeError("oracle: error %d" % rc)


class Data:
    """Alignment patterns plus model: the fixed inputs of every call."""

    def __init__(self, tips, weights, rates, freqs, alpha=1.0, n_cats=1):
        self.tips = np.ascontiguousarray(tips, dtype=np.uint8)
        self.w = np.ascontiguousarray(weights, dtype=np.float64)
        self.rates = np.ascontiguousarray(rates, dtype=np.float64)
        self.freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        self.alpha = float(alpha)
        self.K = int(n_cats)
        self.n = int(self.tips.shape[0])
        self.P = int(self.tips.shape[1])

    @classmethod
    def from_alignment(cls, aln):
        return cls(aln.tips, aln.weights, aln.rates, aln.freqs, aln.alpha, aln.n_cats)

    def args(self):
        return (self.P, _u(self.tips), _d(self.w), _d(self.rates), _d(self.freqs),
                ctypes.c_double(self.alpha), self.K)


def rate_matrix(rates, freqs):
    Q = np.zeros(16)
    r = np.ascontiguousarray(rates, float)
    f = np.ascontiguousarray(freqs, float)
    lib().or_rate_matrix(_d(r), _d(f), _d(Q))
    return Q.reshape(4, 4)


def expm(A):
    A = np.ascontiguousarray(A, float).reshape(16)
    E = np.zeros(16)
    lib().or_expm(_d(A), _d(E))
    return E.reshape(4, 4)


def pmatrix(Q, t):
    Q = np.ascontiguousarray(Q, float).reshape(16)
    P, d1, d2 = np.zeros(16), np.zeros(16), np.zeros(16)
    lib().or_pmatrix(_d(Q), float(t), _d(P), _d(d1), _d(d2))
    return P.reshape(4, 4), d1.reshape(4, 4), d2.reshape(4, 4)


def gammp(a, x):
    return lib().or_gammp(float(a), float(x))


def gamma_rates(alpha, K):
    r = np.zeros(K)
    _check(lib().or_gamma_rates(float(alpha), int(K), _d(r)))
    return r


def _tree(edges, brlen):
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    b = np.ascontiguousarray(brlen, dtype=np.float64)
    return e, b


def loglik(data: Data, edges, brlen, at_edge=0, scaling=True):
    e, b = _tree(edges, brlen)
    out = np.zeros(1)
    _check(lib().or_loglik_at(data.n, _i(e), _d(b), *data.args(), int(scaling), int(at_edge), _d(out)))
    return float(out[0])


def loglik_node(data: Data, edges, brlen, root, scaling=True):
    e, b = _tree(edges, brlen)
    out = np.zeros(1)
    _check(lib().or_loglik_node(data.n, _i(e), _d(b), *data.args(), int(scaling), int(root), _d(out)))
    return float(out[0])


def edge_derivs(data: Data, edges, brlen, edge):
    e, b = _tree(edges, brlen)
    o = np.zeros(3)
    _check(lib().or_edge_derivs(data.n, _i(e), _d(b), *data.args(), int(edge),
                                _d(o[0:]), _d(o[1:]), _d(o[2:])))
    return float(o[0]), float(o[1]), float(o[2])


def gradient(data: Data, edges, brlen):
    """(lnL, grad[E], hessian diagonal[E])."""
    e, b = _tree(edges, brlen)
    g, h, l = np.zeros(len(b)), np.zeros(len(b)), np.zeros(1)
    _check(lib().or_gradient(data.n, _i(e), _d(b), *data.args(), _d(l), _d(g), _d(h)))
    return float(l[0]), g, h


def optimize(data: Data, edges, brlen, mask=None, t_min=T_MIN, t_max=T_MAX,
             tol_lnl=TOL_LNL, tol_t=TOL_T, tol_newton=TOL_NEWTON,
             max_passes=MAX_PASSES, max_newton=MAX_NEWTON, prior_rate=0.0):
    """Coordinate-wise Newton; returns (objective, lengths, passes, converged).
    The objective is lnL, or with prior_rate > 0 lnL plus the log density of
    an exponential prior of that rate on every length (MAP lengths)."""
    e, b = _tree(edges, brlen)
    b = b.copy()
    m = None
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
    l = np.zeros(1)
    ps = np.zeros(1, np.int32)
    cv = np.zeros(1, np.int32)
    _check(lib().or_optimize(data.n, _i(e), _d(b), _u(m) if m is not None else None,
                             *data.args(), float(t_min), float(t_max), float(tol_lnl),
                             float(tol_t), float(tol_newton), int(max_passes), int(max_newton),
                             float(prior_rate), _d(l), _i(ps), _i(cv)))
    return float(l[0]), b, int(ps[0]), bool(cv[0])


# Bounds of the Gamma shape in per-topology model optimisation (the paper
# leaves them to its likelihood library; a reading).
ALPHA_MIN, ALPHA_MAX = 0.02, 100.0


def with_alpha(data: Data, alpha):
    """The same patterns and model with another Gamma shape."""
    return Data(data.tips, data.w, data.rates, data.freqs, alpha, data.K)


def optimize_alpha(data: Data, edges, brlen, alpha0, alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX,
                   tol_lnl=1e-11, max_rounds=500):
    """Joint maximum of lnL over the branch lengths and the Gamma shape alpha
    (the paper's optional per-topology model optimisation, Methods,
    "Phylogenetic Topographer"): rounds of a full branch-length optimisation
    at fixed alpha, then a bounded one-dimensional maximisation over log alpha
    at fixed lengths (scipy's bounded Brent minimiser as the primitive),
    until a round gains less than tol_lnl; then the lengths once more at the
    final alpha.  Returns (lnL, lengths, alpha, rounds)."""
    from scipy.optimize import minimize_scalar

    alpha = min(max(float(alpha0), alpha_min), alpha_max)
    b = np.asarray(brlen, dtype=np.float64).copy()
    prev = -np.inf
    cur = -np.inf
    rounds = 0
    for rounds in range(1, max_rounds + 1):
        cur, b, _, _ = optimize(with_alpha(data, alpha), edges, b)
        if data.K > 1:
            res = minimize_scalar(lambda x: -loglik(with_alpha(data, math.exp(x)), edges, b),
                                  bounds=(math.log(alpha_min), math.log(alpha_max)), method="bounded",
                                  options={"xatol": 1e-10})
            if -res.fun > cur:
                alpha, cur = math.exp(res.x), -res.fun
        if cur - prev < tol_lnl:
            break
        prev = cur
    cur, b, _, _ = optimize(with_alpha(data, alpha), edges, b)
    return cur, b, alpha, rounds
