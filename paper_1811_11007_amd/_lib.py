"""ctypes binding of libpt.so: the same entry points as include/pt.h.

Argument marshalling only; every step of the likelihood, its derivatives and
the branch-length optimisation runs in the library's HIP kernels.  There is
no CPU fallback: importing works without a GPU, but any call that needs one
raises if the library or the device is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpt.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_EUNSUPPORTED, PT_EINTERNAL = 0, -1, -2, -3, -4, -5
PT_FP64, PT_FP32 = 0, 1
PT_PLAN_LOGLIK, PT_PLAN_OPTIMIZE, PT_PLAN_GRAD = 1, 2, 4
PT_LOGLIK_REGISTERS, PT_LOGLIK_STORED = 0, 1

EXPORTS = [
    "pt_last_error", "pt_ctx_create", "pt_ctx_destroy", "pt_ctx_set_group_wait", "pt_aln_create", "pt_aln_destroy",
    "pt_opt_default", "pt_batch_loglik", "pt_batch_optimize_branches", "pt_batch_branch_grad",
    "pt_batch_loglik_noalloc",
    "pt_plan_create", "pt_plan_destroy", "pt_plan_set_graphs", "pt_plan_loglik",
    "pt_plan_optimize", "pt_plan_set_alpha", "pt_plan_optimize_alpha", "pt_plan_grad", "pt_plan_autotune",
    "pt_plan_traffic", "pt_plan_set_profile", "pt_plan_set_loglik_path", "pt_plan_info", "pt_plan_set_launch", "pt_plan_launch_shape",
    "pt_plan_set_tile_patterns", "pt_plan_tile_patterns", "pt_plan_autotune_tiles",
    "pt_model_info", "pt_tree_check", "pt_nni_neighbors", "pt_topology_key", "pt_topology_keys",
    "pt_nni_features", "pt_radius_masks", "pt_split_frequencies", "pt_majority_consensus",
    "pt_mlp_create", "pt_mlp_destroy", "pt_mlp_param_count", "pt_mlp_get_params", "pt_mlp_set_params",
    "pt_mlp_forward", "pt_mlp_warm_start", "pt_mlp_gradient", "pt_mlp_train_step",
]

PT_NNI_FEATURES = 14


class PTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class pt_model(ctypes.Structure):
    _fields_ = [("rates", ctypes.c_double * 6), ("freqs", ctypes.c_double * 4),
                ("alpha", ctypes.c_double), ("n_cats", ctypes.c_int32)]


class pt_trees(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("aln_index", ctypes.POINTER(ctypes.c_int32)),
                ("edge_offset", ctypes.POINTER(ctypes.c_int64)),
                ("edges", ctypes.POINTER(ctypes.c_int32))]


class pt_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class pt_opt(ctypes.Structure):
    _fields_ = [("t_min", ctypes.c_double), ("t_max", ctypes.c_double), ("tol_lnl", ctypes.c_double),
                ("tol_t", ctypes.c_double), ("tol_newton", ctypes.c_double),
                ("max_passes", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("prior_rate", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpt.so is not built: run paper_1811_11007_amd/build.py "
                               "(or __graft_entry__.build())")
        # One HIP runtime per process: when torch is present its bundled
        # runtime is loaded first and libpt binds to it by soname, so device
        # pointers and streams from torch are valid in the library's calls.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        L.pt_last_error.restype = ctypes.c_char_p
        L.pt_ctx_create.argtypes = [i32, P(vp)]
        L.pt_ctx_destroy.argtypes = [vp]
        L.pt_ctx_destroy.restype = None
        L.pt_aln_create.argtypes = [vp, i32, i32, vp, vp, P(pt_model), P(vp)]
        L.pt_aln_destroy.argtypes = [vp]
        L.pt_aln_destroy.restype = None
        L.pt_opt_default.argtypes = [i32, P(pt_opt)]
        L.pt_opt_default.restype = None
        L.pt_batch_loglik.argtypes = [vp, P(vp), i32, P(pt_trees), vp, i32, vp]
        L.pt_batch_optimize_branches.argtypes = [vp, P(vp), i32, P(pt_trees), vp, vp, P(pt_opt), i32,
                                                 vp, vp, vp]
        L.pt_batch_branch_grad.argtypes = [vp, P(vp), i32, P(pt_trees), vp, i32, vp, vp, vp]
        L.pt_batch_loglik_noalloc.argtypes = [vp, P(vp), i32, P(pt_trees), vp, i32, vp]
        L.pt_plan_create.argtypes = [vp, P(vp), i32, P(pt_trees), vp, i32, i32, P(vp)]
        L.pt_plan_destroy.argtypes = [vp]
        L.pt_plan_destroy.restype = None
        L.pt_plan_set_graphs.argtypes = [vp, i32]
        L.pt_plan_loglik.argtypes = [vp, vp, vp, vp]
        L.pt_plan_optimize.argtypes = [vp, vp, P(pt_opt), vp, vp, vp, vp]
        L.pt_plan_set_alpha.argtypes = [vp, vp, vp]
        L.pt_ctx_set_group_wait.argtypes = [vp, ctypes.c_int64]
        L.pt_plan_set_tile_patterns.argtypes = [vp, i32]
        L.pt_plan_tile_patterns.argtypes = [vp, P(i32)]
        L.pt_plan_autotune_tiles.argtypes = [vp, vp, P(i32)]
        L.pt_plan_set_launch.argtypes = [vp, i32, i32]
        L.pt_plan_launch_shape.argtypes = [vp, P(i32), P(i32), P(i32)]
        L.pt_plan_optimize_alpha.argtypes = [vp, vp, P(pt_opt), vp, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, i32, vp, P(i32), vp]
        L.pt_plan_grad.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pt_plan_autotune.argtypes = [vp, vp, P(pt_opt), P(i32), P(i32)]
        L.pt_plan_info.argtypes = [vp, P(i32), P(i64), P(i64)]
        L.pt_plan_traffic.argtypes = [vp, i32, vp, P(ctypes.c_double)]
        L.pt_plan_set_profile.argtypes = [vp, vp]
        L.pt_plan_set_loglik_path.argtypes = [vp, i32]
        L.pt_model_info.argtypes = [P(pt_model), vp, vp, vp, vp]
        L.pt_tree_check.argtypes = [i32, vp]
        L.pt_nni_neighbors.argtypes = [i32, vp, vp, vp, vp, vp]
        L.pt_topology_key.argtypes = [i32, vp, vp]
        L.pt_topology_keys.argtypes = [i32, i32, vp, vp]
        L.pt_nni_features.argtypes = [i32, vp, vp, vp]
        L.pt_radius_masks.argtypes = [i32, i32, vp, vp, i32, vp]
        L.pt_split_frequencies.argtypes = [i32, i32, vp, vp, i32, vp, vp, vp]
        L.pt_majority_consensus.argtypes = [i32, i32, vp, vp, vp, i32, vp]
        L.pt_mlp_create.argtypes = [vp, i32, i32, i32, vp, P(vp)]
        L.pt_mlp_destroy.argtypes = [vp]
        L.pt_mlp_destroy.restype = None
        L.pt_mlp_param_count.argtypes = [vp]
        L.pt_mlp_param_count.restype = i64
        L.pt_mlp_get_params.argtypes = [vp, vp]
        L.pt_mlp_set_params.argtypes = [vp, vp]
        L.pt_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.pt_mlp_warm_start.argtypes = [vp, vp, i32, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        vp, vp]
        L.pt_mlp_gradient.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.pt_mlp_train_step.argtypes = [vp, vp, vp, i32, P(pt_adam), vp, vp]
        for name in EXPORTS:
            if getattr(L, name).restype is ctypes.c_int:
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def check(code):
    if code != PT_OK:
        raise PTError(code, lib().pt_last_error().decode() or "pt error")


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def opt_default(precision=PT_FP64) -> pt_opt:
    o = pt_opt()
    lib().pt_opt_default(precision, ctypes.byref(o))
    return o


class Context:
    """One device: its stream, plans and tuning table."""

    def __init__(self, device: int = 0):
        self.h = ctypes.c_void_p()
        check(lib().pt_ctx_create(device, ctypes.byref(self.h)))

    def set_group_wait(self, cycles):
        """Shader clocks before a cross-block wait of the optimiser gives up
        (<= 0: the default); see pt_ctx_set_group_wait."""
        check(lib().pt_ctx_set_group_wait(self.h, int(cycles)))

    def close(self):
        if self.h:
            lib().pt_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Alignment:
    """Device-resident site patterns plus their GTR + Gamma model."""

    def __init__(self, ctx: Context, tips, weights, rates, freqs, alpha=1.0, n_cats=1):
        self.ctx = ctx
        self.tips = np.ascontiguousarray(tips, dtype=np.uint8)
        self.weights = np.ascontiguousarray(weights, dtype=np.float64)
        self.n_taxa, self.n_patterns = self.tips.shape
        m = make_model(rates, freqs, alpha, n_cats)
        self.h = ctypes.c_void_p()
        check(lib().pt_aln_create(ctx.h, self.n_taxa, self.n_patterns, _ptr(self.tips),
                                  _ptr(self.weights), ctypes.byref(m), ctypes.byref(self.h)))

    @classmethod
    def from_synth(cls, ctx, aln):
        return cls(ctx, aln.tips, aln.weights, aln.rates, aln.freqs, aln.alpha, aln.n_cats)

    def close(self):
        if self.h:
            lib().pt_aln_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trees:
    """A packed batch: per-tree alignment index, edge offsets and edges."""

    def __init__(self, edge_lists, aln_index=None):
        edge_lists = [np.asarray(e, dtype=np.int32).reshape(-1, 2) for e in edge_lists]
        n = len(edge_lists)
        self.aln_index = np.ascontiguousarray(
            np.zeros(n, np.int32) if aln_index is None else aln_index, dtype=np.int32)
        counts = [len(e) for e in edge_lists]
        self.edge_offset = np.zeros(n + 1, dtype=np.int64)
        self.edge_offset[1:] = np.cumsum(counts)
        self.edges = np.ascontiguousarray(
            np.concatenate(edge_lists) if n else np.zeros((0, 2), np.int32), dtype=np.int32)
        self.c = pt_trees(n, self.aln_index.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          self.edge_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))

    @property
    def n_trees(self):
        return len(self.aln_index)

    @property
    def n_edges(self):
        return int(self.edge_offset[-1])


def _aln_array(alns):
    arr = (ctypes.c_void_p * len(alns))(*[a.h for a in alns])
    return arr


def pt_batch_loglik(ctx, alns, trees: Trees, brlen, precision=PT_FP64):
    brlen = np.ascontiguousarray(brlen, dtype=np.float64)
    out = np.zeros(trees.n_trees)
    check(lib().pt_batch_loglik(ctx.h, _aln_array(alns), len(alns), ctypes.byref(trees.c),
                                _ptr(brlen), precision, _ptr(out)))
    return out


def pt_batch_loglik_noalloc(ctx, alns, trees: Trees, brlen, precision=PT_FP64):
    """pt_batch_loglik through the library's fixed workspace (no device
    allocation; see pt.h)."""
    brlen = np.ascontiguousarray(brlen, dtype=np.float64)
    out = np.zeros(trees.n_trees)
    check(lib().pt_batch_loglik_noalloc(ctx.h, _aln_array(alns), len(alns), ctypes.byref(trees.c),
                                        _ptr(brlen), precision, _ptr(out)))
    return out


def pt_batch_optimize_branches(ctx, alns, trees: Trees, brlen, mask=None, opt=None, precision=PT_FP64):
    """Returns (lnL[n_trees], optimised lengths, passes, status)."""
    b = np.array(brlen, dtype=np.float64, copy=True)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    lnl = np.zeros(trees.n_trees)
    ps = np.zeros(trees.n_trees, np.int32)
    st = np.zeros(trees.n_trees, np.int32)
    check(lib().pt_batch_optimize_branches(ctx.h, _aln_array(alns), len(alns), ctypes.byref(trees.c),
                                           _ptr(b), _ptr(m), ctypes.byref(opt) if opt else None,
                                           precision, _ptr(lnl), _ptr(ps), _ptr(st)))
    return lnl, b, ps, st


def pt_batch_branch_grad(ctx, alns, trees: Trees, brlen, precision=PT_FP64, hess=False):
    """Returns (lnL[n_trees], grad[n_edges], hessian diagonal or None)."""
    brlen = np.ascontiguousarray(brlen, dtype=np.float64)
    lnl = np.zeros(trees.n_trees)
    g = np.zeros(trees.n_edges)
    h = np.zeros(trees.n_edges) if hess else None
    check(lib().pt_batch_branch_grad(ctx.h, _aln_array(alns), len(alns), ctypes.byref(trees.c),
                                     _ptr(brlen), precision, _ptr(lnl), _ptr(g), _ptr(h)))
    return lnl, g, h


def make_model(rates, freqs, alpha=1.0, n_cats=1) -> pt_model:
    m = pt_model()
    m.rates[:] = [float(x) for x in rates]
    m.freqs[:] = [float(x) for x in freqs]
    m.alpha = float(alpha)
    m.n_cats = int(n_cats)
    return m


def pt_model_info(rates, freqs, alpha=1.0, n_cats=1):
    """(category rates, U, Uinv, lam) of the model, computed on the host."""
    m = make_model(rates, freqs, alpha, n_cats)
    r = np.zeros(max(int(n_cats), 1))
    U, Ui, lam = np.zeros(16), np.zeros(16), np.zeros(4)
    check(lib().pt_model_info(ctypes.byref(m), _ptr(r), _ptr(U), _ptr(Ui), _ptr(lam)))
    return r, U.reshape(4, 4), Ui.reshape(4, 4), lam


def pt_tree_check(n, edges):
    e = np.ascontiguousarray(edges, dtype=np.int32)
    check(lib().pt_tree_check(int(n), _ptr(e)))


def pt_nni_neighbors(n, edges, brlen=None):
    """Returns (edges[2(n-3)][2n-3][2], lengths or None, touched[2(n-3)][5])."""
    e = np.ascontiguousarray(edges, dtype=np.int32)
    E = len(e)
    k = 2 * (n - 3)
    oe = np.zeros((max(k, 0), E, 2), np.int32)
    ob = np.zeros((max(k, 0), E)) if brlen is not None else None
    ot = np.zeros((max(k, 0), 5), np.int32)
    b = None if brlen is None else np.ascontiguousarray(brlen, dtype=np.float64)
    check(lib().pt_nni_neighbors(n, _ptr(e), _ptr(b), _ptr(oe), _ptr(ob), _ptr(ot)))
    return oe, ob, ot


def pt_topology_key(n, edges):
    """uint64[n-3][W] sorted splits."""
    e = np.ascontiguousarray(edges, dtype=np.int32)
    W = (n + 63) // 64
    out = np.zeros((max(n - 3, 0), W), np.uint64)
    check(lib().pt_topology_key(n, _ptr(e), _ptr(out)))
    return out


def pt_topology_keys(n, edges):
    """Keys of a stack of trees: edges [count][2n-3][2] -> uint64[count][n-3][W]."""
    e = np.ascontiguousarray(edges, dtype=np.int32)
    count = e.shape[0]
    W = (n + 63) // 64
    out = np.zeros((count, max(n - 3, 0), W), np.uint64)
    check(lib().pt_topology_keys(int(n), int(count), _ptr(e), _ptr(out)))
    return out


def pt_nni_features(n, edges, brlen):
    """float32[2(n-3)][PT_NNI_FEATURES] features of each NNI move (pt_nni_neighbors order)."""
    e = np.ascontiguousarray(edges, dtype=np.int32)
    b = np.ascontiguousarray(brlen, dtype=np.float64)
    out = np.zeros((max(2 * (n - 3), 0), PT_NNI_FEATURES), np.float32)
    check(lib().pt_nni_features(int(n), _ptr(e), _ptr(b), _ptr(out)))
    return out


def pt_radius_masks(n, edges, centres, radius):
    """uint8[count][2n-3] radius-limited optimisation masks of a stack of
    trees (edges [count][2n-3][2]) around their centre edges."""
    e = np.ascontiguousarray(edges, dtype=np.int32)
    c = np.ascontiguousarray(centres, dtype=np.int32)
    if e.ndim != 3 or c.shape != (e.shape[0],):
        raise ValueError("edges must be [count][2n-3][2] and centres [count]")
    out = np.zeros((e.shape[0], e.shape[1]), np.uint8)
    check(lib().pt_radius_masks(int(n), int(e.shape[0]), _ptr(e), _ptr(c), int(radius), _ptr(out)))
    return out


def pt_split_frequencies(n, keys, lnl):
    """Split frequencies of a set of topologies (keys uint64[count][n-3][W]
    from pt_topology_keys, lnl[count]): returns (splits uint64[m][W],
    freq[m]) by decreasing frequency."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    lv = np.ascontiguousarray(lnl, dtype=np.float64)
    W = (n + 63) // 64
    if k.ndim != 3 or k.shape[1:] != (max(n - 3, 0), W) or lv.shape != (k.shape[0],):
        raise ValueError("keys must be [count][n-3][W] and lnl [count]")
    cap = max(1, k.shape[0] * max(n - 3, 0))
    splits = np.zeros((cap, W), np.uint64)
    freq = np.zeros(cap)
    m = ctypes.c_int32(0)
    check(lib().pt_split_frequencies(int(n), int(k.shape[0]), _ptr(k), _ptr(lv), int(cap), ctypes.byref(m),
                                     _ptr(splits), _ptr(freq)))
    return splits[:m.value].copy(), freq[:m.value].copy()


def pt_majority_consensus(n, splits, freq):
    """Majority-rule consensus tree (Newick, rooted at taxon 0, clade labels
    = split frequencies)."""
    s = np.ascontiguousarray(splits, dtype=np.uint64)
    f = np.ascontiguousarray(freq, dtype=np.float64)
    cap = 64 + 24 * int(n)
    buf = ctypes.create_string_buffer(cap)
    ln = ctypes.c_int32(0)
    check(lib().pt_majority_consensus(int(n), int(len(f)), _ptr(s), _ptr(f), buf, cap, ctypes.byref(ln)))
    return buf.value.decode()


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class MLP:
    """The warm-start perceptron (pt_mlp_*), driven with torch float32 tensors."""

    def __init__(self, ctx, n_in, n_hidden, n_out, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.shape = (int(n_in), int(n_hidden), int(n_out))
        self.h = ctypes.c_void_p()
        check(lib().pt_mlp_create(ctx.h, *self.shape, _ptr(p), ctypes.byref(self.h)))
        self.n_params = int(lib().pt_mlp_param_count(self.h))

    def params(self):
        out = np.zeros(self.n_params, np.float32)
        check(lib().pt_mlp_get_params(self.h, _ptr(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError("expected %d parameters" % self.n_params)
        check(lib().pt_mlp_set_params(self.h, _ptr(p)))

    def forward(self, d_x, d_y=None, stream=None):
        import torch
        if d_y is None:
            d_y = torch.empty((d_x.shape[0], self.shape[2]), dtype=torch.float32, device=d_x.device)
        check(lib().pt_mlp_forward(self.h, _dptr(d_x), int(d_x.shape[0]), _dptr(d_y), Plan._stream(stream)))
        return d_y

    def warm_start(self, d_x, d_pos, d_base, d_brlen, t_min=1e-8, t_max=100.0, shift=1e-4, stream=None):
        check(lib().pt_mlp_warm_start(self.h, _dptr(d_x), int(d_x.shape[0]), _dptr(d_pos), _dptr(d_base),
                                      float(shift), float(t_min), float(t_max), _dptr(d_brlen),
                                      Plan._stream(stream)))

    def gradient(self, d_x, d_t, d_grad, d_loss=None, stream=None):
        check(lib().pt_mlp_gradient(self.h, _dptr(d_x), _dptr(d_t), int(d_x.shape[0]), _dptr(d_grad),
                                    _dptr(d_loss), Plan._stream(stream)))

    def train_step(self, d_x, d_t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, d_loss=None, stream=None):
        a = pt_adam(lr, beta1, beta2, eps)
        check(lib().pt_mlp_train_step(self.h, _dptr(d_x), _dptr(d_t), int(d_x.shape[0]), ctypes.byref(a),
                                      _dptr(d_loss), Plan._stream(stream)))

    def close(self):
        if self.h:
            lib().pt_mlp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A compiled, device-resident batch (pt_plan_*), driven with torch tensors."""

    def __init__(self, ctx, alns, trees: Trees, kinds, precision=PT_FP64, mask=None):
        self.ctx, self.alns, self.trees, self.precision = ctx, list(alns), trees, precision
        self._mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.h = ctypes.c_void_p()
        check(lib().pt_plan_create(ctx.h, _aln_array(self.alns), len(self.alns), ctypes.byref(trees.c),
                                   _ptr(self._mask), precision, kinds, ctypes.byref(self.h)))

    def set_graphs(self, enable=True):
        check(lib().pt_plan_set_graphs(self.h, int(bool(enable))))

    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    def loglik(self, d_brlen, d_lnl, stream=None):
        check(lib().pt_plan_loglik(self.h, ctypes.c_void_p(d_brlen.data_ptr()),
                                   ctypes.c_void_p(d_lnl.data_ptr()), self._stream(stream)))

    def optimize(self, d_brlen, d_lnl, d_passes=None, d_status=None, opt=None, stream=None):
        check(lib().pt_plan_optimize(
            self.h, ctypes.c_void_p(d_brlen.data_ptr()), ctypes.byref(opt) if opt else None,
            ctypes.c_void_p(d_lnl.data_ptr()),
            ctypes.c_void_p(d_passes.data_ptr()) if d_passes is not None else None,
            ctypes.c_void_p(d_status.data_ptr()) if d_status is not None else None,
            self._stream(stream)))

    def set_alpha(self, alpha, stream=None):
        """Per-tree Gamma shapes (host array [n_trees]), or None for each
        alignment's own."""
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
        check(lib().pt_plan_set_alpha(self.h, _ptr(a), self._stream(stream)))

    def optimize_alpha(self, d_brlen, alpha, alpha_min=0.02, alpha_max=100.0, tol_alpha=1e-4, max_rounds=50,
                       opt=None, stream=None):
        """Joint lengths + Gamma-shape optimisation; returns (lnL, alpha,
        rounds) as numpy arrays / int; d_brlen is updated in place."""
        a = np.array(alpha, dtype=np.float64, copy=True)
        lnl = np.zeros(len(a))
        r = ctypes.c_int32(0)
        check(lib().pt_plan_optimize_alpha(self.h, ctypes.c_void_p(d_brlen.data_ptr()),
                                           ctypes.byref(opt) if opt else None, _ptr(a), float(alpha_min),
                                           float(alpha_max), float(tol_alpha), int(max_rounds), _ptr(lnl),
                                           ctypes.byref(r), self._stream(stream)))
        return lnl, a, r.value

    def grad(self, d_brlen, d_lnl, d_grad, d_hess=None, stream=None):
        check(lib().pt_plan_grad(self.h, ctypes.c_void_p(d_brlen.data_ptr()),
                                 ctypes.c_void_p(d_lnl.data_ptr()), ctypes.c_void_p(d_grad.data_ptr()),
                                 ctypes.c_void_p(d_hess.data_ptr()) if d_hess is not None else None,
                                 self._stream(stream)))

    def autotune(self, d_brlen, opt=None):
        b, i = ctypes.c_int32(), ctypes.c_int32()
        check(lib().pt_plan_autotune(self.h, ctypes.c_void_p(d_brlen.data_ptr()),
                                     ctypes.byref(opt) if opt else None, ctypes.byref(b), ctypes.byref(i)))
        return b.value, i.value

    def set_launch(self, block, groups=1):
        """Optimisation kernel shape: threads per block, blocks per tree."""
        check(lib().pt_plan_set_launch(self.h, int(block), int(groups)))

    def autotune_tiles(self, d_brlen):
        """Patterns per tile of the stored pass and gradient: the fastest of
        64, 128 and 256 on this plan (see pt.h)."""
        n = ctypes.c_int32()
        check(lib().pt_plan_autotune_tiles(self.h, ctypes.c_void_p(d_brlen.data_ptr()), ctypes.byref(n)))
        return n.value

    def set_tile_patterns(self, patterns):
        check(lib().pt_plan_set_tile_patterns(self.h, int(patterns)))

    def tile_patterns(self):
        n = ctypes.c_int32()
        check(lib().pt_plan_tile_patterns(self.h, ctypes.byref(n)))
        return n.value

    def set_loglik_path(self, path):
        """PT_LOGLIK_REGISTERS (default) or PT_LOGLIK_STORED; see pt.h."""
        check(lib().pt_plan_set_loglik_path(self.h, int(path)))

    def launch_shape(self):
        """(threads per block, patterns per thread, blocks per tree)."""
        b, i, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().pt_plan_launch_shape(self.h, ctypes.byref(b), ctypes.byref(i), ctypes.byref(g)))
        return b.value, i.value, g.value

    def traffic(self, kind, passes=None):
        """Algorithmic device bytes one run of `kind` moves."""
        ps = None if passes is None else np.ascontiguousarray(passes, dtype=np.int32)
        out = ctypes.c_double()
        check(lib().pt_plan_traffic(self.h, kind, _ptr(ps), ctypes.byref(out)))
        return out.value

    def set_profile(self, d_counters):
        """d_counters: device int64 tensor [n_trees, 8], or None to stop."""
        check(lib().pt_plan_set_profile(
            self.h, None if d_counters is None else ctypes.c_void_p(d_counters.data_ptr())))

    def info(self):
        n, e, by = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().pt_plan_info(self.h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(by)))
        return n.value, e.value, by.value

    def close(self):
        if self.h:
            lib().pt_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
