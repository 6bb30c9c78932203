// kernels.hip -- CDNA4 (gfx950) kernels of the tree likelihood.
//
// Work decomposition.  An item is one (site pattern, rate category) pair;
// the Kp items of a pattern occupy adjacent lanes of a 64-wide wavefront.
// A thread keeps the same category k for all its items, so the 4x4
// transition matrix it applies is the same for all of them and is read from
// LDS as a wave-uniform-per-k broadcast.  Partials are stored pattern-major,
// [slot][item][4], so one wavefront load of its 64 items is one contiguous
// 1 KiB (FP32) or 2 KiB (FP64) block.
//
// Numerics.  Partials may be stored in FP32; every product, transition
// matrix, logarithm and sum over patterns is FP64.  Per-pattern scaling
// multiplies a new partial by 2^S (S = 64 for FP32 storage, 256 for FP64)
// when its largest entry over categories and states falls below 2^-S, and
// counts the event in a per-pattern scaler; scaling by a power of two is
// exact, so it changes no value.
//
// Sums over patterns are fixed-order: butterfly within a wavefront, then the
// per-wave partials in wave order, then the tiles of a tree in tile order, so
// a rerun is bit-identical.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "pt.h"

namespace pt {
namespace {

constexpr double kLn2 = 0.69314718055994530942;

template <typename T>
struct Store;

template <>
struct Store<float> {
    static constexpr int kScaleExp = 64;
    __device__ static inline void load(const float *p, double x[4]) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    }
    __device__ static inline void store(float *p, const double x[4]) {
        *reinterpret_cast<float4 *>(p) =
            make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    }
};

template <>
struct Store<double> {
    static constexpr int kScaleExp = 256;
    __device__ static inline void load(const double *p, double x[4]) {
        double2 a = reinterpret_cast<const double2 *>(p)[0];
        double2 b = reinterpret_cast<const double2 *>(p)[1];
        x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
    }
    __device__ static inline void store(double *p, const double x[4]) {
        reinterpret_cast<double2 *>(p)[0] = make_double2(x[0], x[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(x[2], x[3]);
    }
};

// Model constants of the tree in flight, copied to LDS once per tree so the
// inner loops read them as broadcasts instead of holding them in registers.
struct ModelS {
    double pU[16];   // pi_i U_im
    double Ui[16];   // Uinv_mj
    double lam[4];
    double rate[kMaxCats];
};

__device__ inline void model_to_lds(const AlnDev *aln, ModelS *m) {
    for (int x = threadIdx.x; x < 16; x += blockDim.x) {
        m->pU[x] = aln->freqs[x >> 2] * aln->U[x];
        m->Ui[x] = aln->Uinv[x];
    }
    if (threadIdx.x < 4) m->lam[threadIdx.x] = aln->lam[threadIdx.x];
    if (threadIdx.x < kMaxCats) m->rate[threadIdx.x] = aln->rate[threadIdx.x];
}

// View of one tree's data for the device functions below.
template <typename T>
struct TreeView {
    const ModelS *m;     // LDS
    const double *pm;    // LDS: [E][Kp][16]
    const uint8_t *tips; // [n][P]
    const double *w;     // [P]
    T *clv;              // slot 0 of this tree
    uint16_t *cnt;       // slot 0 of this tree
    int P, K, Kp, kshift, items;
};

template <typename T>
__device__ inline void load_side(const TreeView<T> &v, int ref, int it, int p, double x[4], int &c) {
    if (ref < 0) {
        unsigned code = v.tips[(size_t)(-ref - 1) * v.P + p];
        x[0] = code & 1u; x[1] = (code >> 1) & 1u; x[2] = (code >> 2) & 1u; x[3] = (code >> 3) & 1u;
        c = 0;
    } else {
        Store<T>::load(v.clv + ((size_t)ref * v.items + it) * 4, x);
        c = v.cnt[(size_t)ref * v.P + p];
    }
}

__device__ inline double group_max(double x, int Kp) {
    for (int m = 1; m < Kp; m <<= 1) x = fmax(x, __shfl_xor(x, m, 64));
    return x;
}

__device__ inline double group_sum(double x, int Kp) {
    for (int m = 1; m < Kp; m <<= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Fixed-order block sum of three values; every thread receives the totals.
// `red` holds two buffers used alternately, so back-to-back sums need one
// barrier each.
template <int BS>
__device__ inline void block_sum3(double &a, double &b, double &c, double *red, int &parity) {
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m, 64);
        b += __shfl_xor(b, m, 64);
        c += __shfl_xor(c, m, 64);
    }
    constexpr int W = BS / 64;
    double *r = red + parity * W * 3;
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r[wave * 3 + 0] = a;
        r[wave * 3 + 1] = b;
        r[wave * 3 + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        a += r[w * 3 + 0];
        b += r[w * 3 + 1];
        c += r[w * 3 + 2];
    }
    parity ^= 1;
}

// Entry (i, j) of P(r_k t) = U diag(exp(lam r_k t)) Uinv.
__device__ inline double pm_entry(const AlnDev *aln, int k, int ij, double t) {
    const int i = ij >> 2, j = ij & 3;
    const double r = aln->rate[k];
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) s += aln->U[i * 4 + m] * exp(aln->lam[m] * r * t) * aln->Uinv[m * 4 + j];
    return s;
}

// OP_UPDATE over this thread's items:
//   dst = (P(t_ea) . side a) * (P(t_eb) . side b), elementwise over states,
// with per-pattern scaling.
// Returns p unchanged but opaque to the optimiser, so loads through it stay
// inside the op that needs them instead of being hoisted out of the op loop
// and pinned in registers for the whole kernel.
template <typename P>
__device__ inline P *opaque(P *p) {
    __asm__ volatile("" : "+s"(p));
    return p;
}

template <typename T, int BS, int NI>
__device__ inline void do_update(const TreeView<T> v, const Op op, int base) {
    const int tid = threadIdx.x;
    const int k = tid & (v.Kp - 1);
    const bool kval = k < v.K;
    const double *pm = opaque(v.pm);
    const double *Pa = pm + ((size_t)op.ea * v.Kp + k) * 16;
    const double *Pb = pm + ((size_t)op.eb * v.Kp + k) * 16;
    const double thr = ldexp(1.0, -Store<T>::kScaleExp);
    const double up = ldexp(1.0, Store<T>::kScaleExp);
#pragma unroll 1
    for (int j = 0; j < NI; ++j) {
        const int it = base + j * BS + tid;
        const bool valid = it < v.items;
        const int p = it >> v.kshift;
        double xa[4] = {0, 0, 0, 0}, xb[4] = {0, 0, 0, 0};
        int ca = 0, cb = 0;
        if (valid) {
            load_side(v, op.a, it, p, xa, ca);
            load_side(v, op.b, it, p, xb, cb);
        }
        double o[4], mx = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double sa = Pa[i * 4 + 0] * xa[0] + Pa[i * 4 + 1] * xa[1] + Pa[i * 4 + 2] * xa[2] + Pa[i * 4 + 3] * xa[3];
            double sb = Pb[i * 4 + 0] * xb[0] + Pb[i * 4 + 1] * xb[1] + Pb[i * 4 + 2] * xb[2] + Pb[i * 4 + 3] * xb[3];
            o[i] = kval ? sa * sb : 0.0;
            mx = fmax(mx, o[i]);
        }
        mx = group_max(mx, v.Kp);
        int c = ca + cb;
        if (mx < thr && mx > 0.0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] *= up;
            c += 1;
        }
        if (valid) {
            Store<T>::store(v.clv + ((size_t)op.dst * v.items + it) * 4, o);
            v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)c;  // every lane of the pattern writes the same value
        }
    }
}

// Per-edge eigenbasis table ("sumtable") of this thread's items across an
// edge with sides a and b:  s_m = (sum_i pi_i A_i U_im) (sum_j Uinv_mj B_j),
// so that L(t) = sum_m s_m exp(lam_m r_k t) for the item's category.
// wl = pattern weight on the first lane of a valid pattern, else 0;
// returns this thread's share of the t-independent part of lnL (scaler
// corrections and the 1/K category weight).
template <typename T, typename S, int BS, int NI>
__device__ inline double build_sumtable(const TreeView<T> &v, int a, int b, int base,
                                        S s[NI][4], double wl[NI]) {
    const ModelS *md = opaque(v.m);
    const int tid = threadIdx.x;
    const int k = tid & (v.Kp - 1);
    const double logK = log((double)v.K);
    double cterm = 0.0;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int it = base + j * BS + tid;
        const bool valid = it < v.items;
        const int p = it >> v.kshift;
        double xa[4] = {0, 0, 0, 0}, xb[4] = {0, 0, 0, 0};
        int ca = 0, cb = 0;
        if (valid) {
            load_side(v, a, it, p, xa, ca);
            load_side(v, b, it, p, xb, cb);
        }
        const bool live = valid && k < v.K;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double ua = 0.0, vb = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ua += md->pU[i * 4 + m] * xa[i];
                vb += md->Ui[m * 4 + i] * xb[i];
            }
            s[j][m] = live ? (S)(ua * vb) : (S)0;
        }
        const bool lead = valid && k == 0;
        const double w = lead ? v.w[p] : 0.0;
        wl[j] = w;
        cterm -= w * ((double)(ca + cb) * Store<T>::kScaleExp * kLn2 + logK);
    }
    return cterm;
}

// This thread's shares of lnL, d lnL/dt, d2 lnL/dt2 at length t.
template <typename S, int BS, int NI>
__device__ inline void eval_sumtable(const ModelS *md_in, int Kp, double t, const S s[NI][4],
                                     const double wl[NI], double &l0, double &l1, double &l2) {
    const ModelS *md = opaque(md_in);
    const int k = threadIdx.x & (Kp - 1);
    const double r = md->rate[k];
    double e[4], q1[4], q2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        q1[m] = md->lam[m] * r;
        q2[m] = q1[m] * q1[m];
        e[m] = exp(q1[m] * t);
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        double L = 0.0, L1 = 0.0, L2 = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double se = (double)s[j][m] * e[m];
            L += se;
            L1 += se * q1[m];
            L2 += se * q2[m];
        }
        L = group_sum(L, Kp);
        L1 = group_sum(L1, Kp);
        L2 = group_sum(L2, Kp);
        if (wl[j] != 0.0) {
            const double r1 = L1 / L;
            l0 += wl[j] * log(L);
            l1 += wl[j] * r1;
            l2 += wl[j] * (L2 / L - r1 * r1);
        }
    }
}

struct Sums3 {
    double l0, l1, l2;
    int parity;
};

// OP_EVAL: block totals of lnL and its first two derivatives across edge
// e at length t.
template <typename T, int BS, int NI>
__device__ inline Sums3 eval_edge(const TreeView<T> v, int a, int b, int base, double t, double *red,
                                        int parity) {
    T s[NI][4];
    double wl[NI];
    Sums3 r;
    r.l0 = build_sumtable<T, T, BS, NI>(v, a, b, base, s, wl);
    r.l1 = r.l2 = 0.0;
    eval_sumtable<T, BS, NI>(v.m, v.Kp, t, s, wl, r.l0, r.l1, r.l2);
    block_sum3<BS>(r.l0, r.l1, r.l2, red, parity);
    r.parity = parity;
    return r;
}

struct EdgeResult {
    double t, lnl;
    int parity;
};

// OP_NEWTON: safeguarded, projected Newton on the length of one edge.
//  - the bracket (lo, hi) starts as [t_min, t_max] and shrinks to t on the
//    side the first derivative points away from;
//  - a Newton step is taken when d2 < 0 and it stays in the bracket (the
//    original bounds count as inside), else the bracket is bisected
//    geometrically;
//  - a bound with the derivative pointing outwards is an optimum;
//  - a step of at most tol * max(t, 1e-6) is converged and not taken, so
//    the returned lnL is the one evaluated at the returned t.
// All threads hold identical block totals, so every thread takes the same
// decisions.
template <typename T, int BS, int NI>
__device__ inline EdgeResult newton_edge(const TreeView<T> v, int a, int b, double t, const OptParams opt,
                                               double *red, int parity) {
    T s[NI][4];
    double wl[NI];
    const double cterm = build_sumtable<T, T, BS, NI>(v, a, b, 0, s, wl);
    double lo = opt.t_min, hi = opt.t_max, lnl = 0.0;
    for (int it = 1;; ++it) {
        double l0 = cterm, d1 = 0.0, d2 = 0.0;
        eval_sumtable<T, BS, NI>(v.m, v.Kp, t, s, wl, l0, d1, d2);
        block_sum3<BS>(l0, d1, d2, red, parity);
        lnl = l0;
        if (it >= opt.max_newton) break;
        if (d1 > 0.0) lo = t;
        else if (d1 < 0.0) hi = t;
        else break;
        if ((t <= opt.t_min && d1 <= 0.0) || (t >= opt.t_max && d1 >= 0.0)) break;
        double tn = d2 < 0.0 ? t - d1 / d2 : NAN;
        if (tn < opt.t_min) tn = opt.t_min;
        if (tn > opt.t_max) tn = opt.t_max;
        const bool inside = !isnan(tn) && (tn > lo || (lo == opt.t_min && tn == opt.t_min)) &&
                            (tn < hi || (hi == opt.t_max && tn == opt.t_max));
        if (!inside) tn = sqrt(lo * hi);
        if (fabs(tn - t) <= opt.tol_newton * fmax(t, 1e-6)) break;
        t = tn;
    }
    EdgeResult r;
    r.t = t;
    r.lnl = lnl;
    r.parity = parity;
    return r;
}

template <typename T>
__device__ inline TreeView<T> make_view(const TreeDev &td, const AlnDev *aln, const BatchArgs &a,
                                        const ModelS *m, const double *pm_lds) {
    TreeView<T> v;
    v.m = m;
    v.pm = pm_lds;
    v.tips = aln->tips;
    v.w = aln->w;
    v.clv = reinterpret_cast<T *>(a.clv) + td.clv_off;
    v.cnt = a.cnt + td.cnt_off;
    v.P = aln->P;
    v.K = aln->K;
    v.Kp = aln->Kp;
    v.kshift = __ffs(aln->Kp) - 1;
    v.items = aln->P * aln->Kp;
    return v;
}

// ----------------------------------------------------------------- kernels

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Transition matrices of every flat edge: one thread per edge.
__global__ void k_pmat(const BatchArgs a, const double *brlen) {
    const int64_t fe = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (fe >= a.n_edges) return;
    const TreeDev &td = a.trees[a.edge_tree[fe]];
    const AlnDev *aln = a.alns + td.aln;
    const int Kp = aln->Kp;
    const double t = brlen[fe];
    double *out = a.pmat + td.pm_off + (fe - td.edge_off) * Kp * 16;
    for (int k = 0; k < Kp; ++k) {
        double e[4];
        for (int m = 0; m < 4; ++m) e[m] = exp(aln->lam[m] * aln->rate[k] * t);
        for (int ij = 0; ij < 16; ++ij) {
            const int i = ij >> 2, j = ij & 3;
            double s = 0.0;
            for (int m = 0; m < 4; ++m) s += aln->U[i * 4 + m] * e[m] * aln->Uinv[m * 4 + j];
            out[k * 16 + ij] = s;
        }
    }
}

// Pattern-tile kernel: each block runs its tree's program over one tile of
// items.  LOGLIK programs end in one EVAL (column 0); GRAD programs EVAL
// every edge.  Output: part[tile][col] = (lnL, d1, d2) partial sums.
template <typename T, int BS, int NI>
__global__ void __launch_bounds__(BS) k_tiles(const BatchArgs a, const double *brlen) {
    extern __shared__ double lds[];
    __shared__ double red[2 * (BS / 64) * 3];
    __shared__ ModelS model;
    const int tile = blockIdx.x;
    const TreeDev td = a.trees[a.tile_tree[tile]];
    const AlnDev *aln = a.alns + td.aln;
    const int n_pm = td.n_edges * aln->Kp * 16;
    for (int i = threadIdx.x; i < n_pm; i += BS) lds[i] = a.pmat[td.pm_off + i];
    model_to_lds(aln, &model);
    __syncthreads();
    const TreeView<T> v = make_view<T>(td, aln, a, &model, lds);
    const int base = (tile - td.tile_begin) * BS * NI;
    int parity = 0;
    for (int o = 0; o < td.n_first; ++o) {
        const Op op = a.ops[td.op_first + o];
        if (op.code == OP_UPDATE) {
            do_update<T, BS, NI>(v, op, base);
            continue;
        }
        const Sums3 r = eval_edge<T, BS, NI>(v, op.a, op.b, base, brlen[td.edge_off + op.dst], red, parity);
        parity = r.parity;
        if (threadIdx.x == 0) {
            double *out = a.part + ((size_t)tile * a.part_cols + op.ea) * 3;
            out[0] = r.l0;
            out[1] = r.l1;
            out[2] = r.l2;
        }
    }
}

// Sum the tile partials of every tree (LOGLIK) or every edge (GRAD) in
// tile order.
__global__ void k_reduce(const BatchArgs a, bool grad, double *lnl, double *gout, double *hout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!grad) {
        if (i >= a.n_trees) return;
        const TreeDev &td = a.trees[i];
        double s = 0.0;
        for (int t = 0; t < td.n_tiles; ++t) s += a.part[((size_t)(td.tile_begin + t) * a.part_cols) * 3];
        lnl[i] = s;
        return;
    }
    if (i >= a.n_edges) return;
    const int b = a.edge_tree[i];
    const TreeDev &td = a.trees[b];
    const int e = (int)(i - td.edge_off);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int t = 0; t < td.n_tiles; ++t) {
        const double *pp = a.part + ((size_t)(td.tile_begin + t) * a.part_cols + e) * 3;
        s0 += pp[0];
        s1 += pp[1];
        s2 += pp[2];
    }
    gout[i] = s1;
    if (hout) hout[i] = s2;
    if (e == 0 && lnl) lnl[b] = s0;
}

// Branch-length optimisation: one block owns one tree at a time, taken from
// a work counter in the order given (largest trees first), and runs the
// whole smoothing loop -- partial updates, per-edge Newton iterations with
// block reductions, pass-level convergence -- without leaving the kernel.
// Every wave exits once the counter passes the number of trees.
template <typename T, int BS, int NI>
__global__ void __launch_bounds__(BS) k_optimize(const BatchArgs a, double *brlen, const OptParams opt,
                                                 double *lnl_out, int32_t *passes_out,
                                                 int32_t *status_out) {
    extern __shared__ double lds[];
    __shared__ double red[2 * (BS / 64) * 3];
    __shared__ ModelS model;
    __shared__ int q_sh;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) q_sh = atomicAdd(a.queue, 1);
        __syncthreads();
        const int q = q_sh;
        if (q >= a.n_trees) break;
        const int b = a.order[q];
        const TreeDev td = a.trees[b];
        const AlnDev *aln = a.alns + td.aln;
        const int E = td.n_edges, Kp = aln->Kp;
        double *pm = lds;
        double *tl = lds + (size_t)E * Kp * 16;
        for (int e = tid; e < E; e += BS) tl[e] = fmin(fmax(brlen[td.edge_off + e], opt.t_min), opt.t_max);
        model_to_lds(aln, &model);
        __syncthreads();
        for (int x = tid; x < E * Kp * 16; x += BS) {
            const int e = x / (Kp * 16), r = x % (Kp * 16);
            pm[x] = pm_entry(aln, r >> 4, r & 15, tl[e]);
        }
        __syncthreads();
        const TreeView<T> v = make_view<T>(td, aln, a, &model, pm);
        int parity = 0;
        double prev = -INFINITY, cur = -INFINITY;
        int passes = 0;
        bool converged = false;
        for (;;) {
            const bool first = passes == 0;
            const int o0 = first ? td.op_first : td.op_steady;
            const int no = first ? td.n_first : td.n_steady;
            double max_rel = 0.0;
            for (int o = 0; o < no; ++o) {
                const Op op = a.ops[o0 + o];
                if (op.code == OP_UPDATE) {
                    do_update<T, BS, NI>(v, op, 0);
                    continue;
                }
                const int e = op.dst;
                const double t0 = tl[e];
                if (op.code == OP_EVAL) {
                    const Sums3 r = eval_edge<T, BS, NI>(v, op.a, op.b, 0, t0, red, parity);
                    parity = r.parity;
                    cur = r.l0;
                    continue;
                }
                const EdgeResult r = newton_edge<T, BS, NI>(v, op.a, op.b, t0, opt, red, parity);
                parity = r.parity;
                cur = r.lnl;
                max_rel = fmax(max_rel, fabs(r.t - t0) / fmax(t0, 1e-6));
                if (r.t != t0) {
                    if (tid == 0) tl[e] = r.t;
                    if (tid < Kp * 16) pm[(size_t)e * Kp * 16 + tid] = pm_entry(aln, tid >> 4, tid & 15, r.t);
                    __syncthreads();
                }
            }
            ++passes;
            if (td.n_steady == 0 || (cur - prev < opt.tol_lnl && max_rel < opt.tol_t)) {
                converged = true;
                break;
            }
            if (passes >= opt.max_passes) break;
            prev = cur;
        }
        for (int e = tid; e < E; e += BS) brlen[td.edge_off + e] = tl[e];
        if (tid == 0) {
            lnl_out[b] = cur;
            if (passes_out) passes_out[b] = passes;
            if (status_out) status_out[b] = converged ? 0 : 1;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- dispatch

template <typename T, int BS, int NI>
hipError_t launch_opt_t(int grid, const BatchArgs &a, double *brlen, const OptParams &opt, double *lnl,
                        int32_t *passes, int32_t *status, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_optimize<T, BS, NI>), dim3(grid), dim3(BS), lds, s, a, brlen, opt, lnl, passes,
                       status);
    return hipGetLastError();
}

template <typename T, int BS, int NI>
int occ_opt_t(size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_optimize<T, BS, NI>, BS, lds) != hipSuccess) return 0;
    return n;
}

#define PT_OPT_SHAPES(X) \
    X(256, 1) X(256, 2) X(256, 4) X(256, 8) X(256, 12) X(256, 16) \
    X(512, 1) X(512, 2) X(512, 4) X(512, 8) X(512, 12) X(512, 16) \
    X(1024, 1) X(1024, 2) X(1024, 4) X(1024, 8) X(1024, 12) X(1024, 16)

}  // namespace

bool optimize_shape_supported(int block, int items) {
#define X(B, N) if (block == B && items == N) return true;
    PT_OPT_SHAPES(X)
#undef X
    return false;
}

int optimize_blocks_per_cu(int precision, int block, int items, size_t lds) {
#define X(B, N)                                                               \
    if (block == B && items == N)                                             \
        return precision == PT_FP32 ? occ_opt_t<float, B, N>(lds) : occ_opt_t<double, B, N>(lds);
    PT_OPT_SHAPES(X)
#undef X
    return 0;
}

hipError_t launch_optimize(int precision, int block, int items, int grid, const BatchArgs &a, double *brlen,
                           const OptParams &opt, double *lnl, int32_t *passes, int32_t *status, size_t lds,
                           hipStream_t s) {
#define X(B, N)                                                                                      \
    if (block == B && items == N)                                                                    \
        return precision == PT_FP32                                                                  \
                   ? launch_opt_t<float, B, N>(grid, a, brlen, opt, lnl, passes, status, lds, s)     \
                   : launch_opt_t<double, B, N>(grid, a, brlen, opt, lnl, passes, status, lds, s);
    PT_OPT_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_pmat(const BatchArgs &a, const double *brlen, hipStream_t s) {
    if (a.n_edges <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pmat, dim3((unsigned)((a.n_edges + 127) / 128)), dim3(128), 0, s, a, brlen);
    return hipGetLastError();
}

hipError_t launch_tiles(int precision, bool grad, const BatchArgs &a, const double *brlen, size_t lds,
                        hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    dim3 g(a.n_tiles), b(kTileBlock);
    (void)grad;  // the program decides: one EVAL (lnL) or one per edge (gradient)
    if (precision == PT_FP32)
        hipLaunchKernelGGL((k_tiles<float, kTileBlock, kTileItems>), g, b, lds, s, a, brlen);
    else
        hipLaunchKernelGGL((k_tiles<double, kTileBlock, kTileItems>), g, b, lds, s, a, brlen);
    return hipGetLastError();
}

hipError_t launch_reduce(bool grad, const BatchArgs &a, double *lnl, double *gout, double *hout,
                         hipStream_t s) {
    const int64_t n = grad ? a.n_edges : a.n_trees;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, grad, lnl, gout, hout);
    return hipGetLastError();
}

}  // namespace pt
