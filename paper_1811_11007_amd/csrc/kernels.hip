// kernels.hip -- CDNA4 (gfx950) kernels of the tree likelihood.
//
// Work decomposition.  One thread owns one site pattern at a time and
// handles all of its rate categories, so the per-pattern scaling decision,
// the sum over categories and the logarithm stay inside the thread.  Partials
// are stored category-major per slot, [slot][Kp][P][4], so for a fixed
// category a wavefront's 64 patterns are one contiguous 1 KiB (FP32) or
// 2 KiB (FP64) block: every load and store is fully coalesced.  Transition
// matrices sit in LDS and are read with wave-uniform addresses (broadcast).
//
// Numerics.  Partials may be stored in FP32; every product, transition
// matrix, logarithm and sum over patterns is FP64.  Per-pattern scaling
// multiplies a new partial by 2^S (S = 64 for FP32 storage, 256 for FP64)
// when its largest entry over categories and states falls below 2^-S, and
// counts the event in a per-pattern scaler; scaling by a power of two is
// exact, so it changes no value.
//
// Sums over patterns are fixed-order: butterfly within a wavefront, then the
// per-wave partials in wave order, then the tiles of a tree in tile order (or,
// for a tree optimised by several blocks, the blocks in block order), so a
// rerun is bit-identical.
//
// Kernels: k_pmat (transition matrices), k_tiles32 / k_tiles64 (a tree's
// likelihood or gradient program over one pattern tile), k_reduce (tile sums
// in order), k_optimize (the whole branch-length smoothing loop of a tree,
// one block per tree or one tree split over several blocks).
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

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
    // one category's four states as loaded, widened when used
    using Raw = float4;
    __device__ static inline Raw load_raw(const float *p) { return *reinterpret_cast<const float4 *>(p); }
    __device__ static inline void widen(const Raw &v, double x[4]) {
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    }
    __device__ static inline double as_stored(double x) { return (double)(float)x; }
    __device__ static inline Raw pack(const double x[4]) {
        return make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    }
    __device__ static inline void store_raw(float *p, const Raw &r) { *reinterpret_cast<float4 *>(p) = r; }
    __device__ static inline void store(float *p, const double x[4]) { store_raw(p, pack(x)); }
};

template <>
struct Store<double> {
    static constexpr int kScaleExp = 256;
    struct Raw {
        double2 a, b;
    };
    __device__ static inline Raw load_raw(const double *p) {
        Raw r;
        r.a = reinterpret_cast<const double2 *>(p)[0];
        r.b = reinterpret_cast<const double2 *>(p)[1];
        return r;
    }
    __device__ static inline void widen(const Raw &v, double x[4]) {
        x[0] = v.a.x; x[1] = v.a.y; x[2] = v.b.x; x[3] = v.b.y;
    }
    __device__ static inline double as_stored(double x) { return x; }
    __device__ static inline Raw pack(const double x[4]) {
        Raw r;
        r.a = make_double2(x[0], x[1]);
        r.b = make_double2(x[2], x[3]);
        return r;
    }
    __device__ static inline void store_raw(double *p, const Raw &r) {
        reinterpret_cast<double2 *>(p)[0] = r.a;
        reinterpret_cast<double2 *>(p)[1] = r.b;
    }
    __device__ static inline void store(double *p, const double x[4]) {
        reinterpret_cast<double2 *>(p)[0] = make_double2(x[0], x[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(x[2], x[3]);
    }
};

// Model constants of the tree in flight, copied to LDS once per tree.
struct ModelS {
    double W[16];    // W_im = pi_i U_im = Uinv_mi
    double U[16];    // P(t) = U diag(exp(lam t)) Uinv
    double Uinv[16];
    double lam[4];
    double rate[kMaxCats];
    float Wf[16];    // W rounded to FP32 (the FP32 tables of the optimisation loop)
};

__device__ inline void model_to_lds(const AlnDev *aln, ModelS *m) {
    for (int x = threadIdx.x; x < 16; x += blockDim.x) {
        m->W[x] = aln->W[x];
        m->Wf[x] = (float)aln->W[x];
        m->U[x] = aln->U[x];
        m->Uinv[x] = aln->Uinv[x];
    }
    if (threadIdx.x < 4) m->lam[threadIdx.x] = aln->lam[threadIdx.x];
    if (threadIdx.x < kMaxCats) m->rate[threadIdx.x] = aln->rate[threadIdx.x];
}

// Load through a pointer known to address global memory (pointers read out
// of descriptors would otherwise be accessed with generic FLAT loads).
template <typename X>
__device__ inline X ldg(const X *p) {
    return *(const __attribute__((address_space(1))) X *)p;
}

// One op of a program.  Programs are never written during a launch, so they
// are read through the constant address space: scalar loads into SGPRs.
// (A kernel that stores partials would otherwise read its ops by vector
// loads, the global memory not being known constant, and wait on the vector
// memory counter before every branch on the opcode.)
__device__ inline Op load_op(const Op *ops, int64_t i) {
    static_assert(sizeof(Op) == 8 * sizeof(int32_t), "an op is eight words");
    const __attribute__((address_space(4))) int32_t *q = (const __attribute__((address_space(4))) int32_t *)(ops + i);
    Op op;
    op.code = q[0];
    op.dst = q[1];
    op.a = q[2];
    op.ea = q[3];
    op.b = q[4];
    op.eb = q[5];
    op.pad0 = q[6];
    op.pad1 = q[7];
    return op;
}

// View of one tree's data for the device functions below.
template <typename T>
struct TreeView {
    const ModelS *m;     // LDS
    const double *pm;    // LDS: [E][Kp][16] (or global, see PmPtr)
    const float *pmf;    // optional FP32 copy of pm in LDS
    const uint8_t *tips; // [n][P]
    const double *w;     // [P]
    T *clv;              // slot 0 of this tree: [slot][Kp][P][4]
    uint16_t *cnt;       // slot 0 of this tree: [slot][P]
    int P, K;            // P: the pattern stride of the layouts
    int np;              // patterns this block works on (tips, w, clv, cnt start at its first)
};

template <typename T, int KP>
__device__ inline T *slot_ptr(const TreeView<T> &v, int ref, int k, int p) {
    return v.clv + (((size_t)ref * KP + k) * v.P + p) * 4;
}

__device__ inline void tip_vec(unsigned code, double x[4]) {
    x[0] = code & 1u; x[1] = (code >> 1) & 1u; x[2] = (code >> 2) & 1u; x[3] = (code >> 3) & 1u;
}

// Entry (i, j) of P(r_k t) = U diag(exp(lam r_k t)) Uinv, from the block's
// LDS copy of the model (the optimisation loop recomputes an edge's matrices
// after every length change, and global loads there cost a round trip).
__device__ inline double pm_entry(const ModelS *md, int k, int ij, double t) {
    const int i = ij >> 2, j = ij & 3;
    const double r = md->rate[k];
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) s += md->U[i * 4 + m] * exp(md->lam[m] * r * t) * md->Uinv[m * 4 + j];
    return s;
}

// The same entry from the exponentials ex[k*4 + m] = exp(lam_m r_k t), each
// computed once (by the same expression) instead of once per entry.
__device__ inline double pm_entry_ex(const ModelS *md, const double *ex, int k, int ij) {
    const int i = ij >> 2, j = ij & 3;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) s += md->U[i * 4 + m] * ex[k * 4 + m] * md->Uinv[m * 4 + j];
    return s;
}

// 1 / x from the hardware estimate plus two Newton-Raphson steps.
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Moves a double across lanes with a DPP row shift; lanes whose source lies
// outside their row of 16 receive 0.
template <int CTRL>
__device__ inline double dpp_shr(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Wavefront sum in a fixed order: a prefix sum inside each row of 16 lanes
// (DPP row shifts by 1, 2, 4, 8), then the four row totals in row order.
// Every lane receives the total.
__device__ inline double wave_sum(double v) {
    v += dpp_shr<0x111>(v);
    v += dpp_shr<0x112>(v);
    v += dpp_shr<0x114>(v);
    v += dpp_shr<0x118>(v);
    return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// Fixed-order block sum of three values; every thread receives the totals.
// `red` holds two buffers used alternately, so back-to-back sums need one
// barrier each.
template <int BS>
__device__ inline void block_sum3(double &a, double &b, double &c, double *red, int &parity) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
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

// A tree optimised by G > 1 blocks, each over its own share of the patterns
// (k_optimize): every block sum is combined across the blocks.  Lane 0 of
// each block's first wave publishes the block's triple in its own entry of
// one of two alternating slots, each value carrying the reduction's number
// (mod 4) in its two lowest mantissa bits; lanes 0..G-1 of that wave then
// poll the G entries in parallel, one entry per lane, until every value of
// every entry carries the number, and the G triples are summed in block
// order with the tag bits cleared.  Every block sums the same bits in the
// same order, so all hold identical totals and take identical decisions;
// clearing the two bits perturbs a value by at most 2^-51 relative.  One
// store and one load round trip per reduction, with no counter.  The
// accesses are device-scope atomics (coherent across the XCDs).  A slot is
// rewritten two reductions later, by when every block has read it (a block
// publishes reduction s + 1 only after reading all of s), and the previous
// content of a slot carries another number (or is zero, which no reduction
// uses as its tag).  A wait is bounded in time: when it runs out the tree is
// marked broken, its blocks stop waiting, and its status reports the failure.
// (The blocks' own partials are a different matter: see k_optimize.)
// per-tree words (kGroupSyncWords): broken, then slots [2][G][3]
static_assert(1 + 2 * kGroupBlocksMax * 3 <= kGroupSyncWords, "cross-block state does not fit");
constexpr long long kGroupWaitCycles = 1ll << 27;  // shader clocks before a wait gives up

__device__ inline unsigned long long load_agent(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_agent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long tag_bits(double v, unsigned long long tag) {
    return ((unsigned long long)__double_as_longlong(v) & ~3ull) | tag;
}

__device__ inline double untag(unsigned long long b) { return __longlong_as_double((long long)(b & ~3ull)); }

__device__ inline unsigned long long lane_u64(unsigned long long v, int lane) {
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

struct GroupS {  // in LDS; written by lane 0 of the block's first wave
    int G, g;
    int seq, is_broken;
    unsigned long long *broken, *slots;
    long long wait;  // shader clocks before a wait gives up
    double tot[3];
};

// Called by the block's first wave (all 64 lanes) with the block's totals.
__device__ inline void group_exchange(GroupS *gs, double a, double b, double c) {
    const int G = gs->G, g = gs->g, s = gs->seq;
    const int lane = threadIdx.x & 63;
    unsigned long long *slot = gs->slots + (size_t)(s & 1) * G * 3;
    const unsigned long long want = (unsigned long long)((s + 1) & 3);
    const unsigned long long ta = tag_bits(a, want), tb = tag_bits(b, want), tc = tag_bits(c, want);
    if (lane == 0) {
        store_agent(slot + g * 3 + 0, ta);
        store_agent(slot + g * 3 + 1, tb);
        store_agent(slot + g * 3 + 2, tc);
    }
    unsigned long long va = ta, vb = tb, vc = tc;  // lane g keeps its own entry
    bool ok = lane >= G || lane == g;
    if (!gs->is_broken) {
        const long long t0 = clock64();
        for (;;) {
            if (!ok) {
                va = load_agent(slot + lane * 3 + 0);
                vb = load_agent(slot + lane * 3 + 1);
                vc = load_agent(slot + lane * 3 + 2);
                ok = (va & 3ull) == want && (vb & 3ull) == want && (vc & 3ull) == want;
            }
            if (__all(ok)) break;
            if (clock64() - t0 > gs->wait) {
                if (lane == 0) {
                    store_agent(gs->broken, 1ull);
                    gs->is_broken = 1;
                }
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int h = 0; h < G; ++h) {
        t0 += untag(lane_u64(va, h));
        t1 += untag(lane_u64(vb, h));
        t2 += untag(lane_u64(vc, h));
    }
    if (lane == 0) {
        gs->tot[0] = t0;
        gs->tot[1] = t1;
        gs->tot[2] = t2;
        gs->seq = s + 1;
    }
}

// Block sum of three values, then (gs set) the sum over the tree's blocks;
// every thread receives the totals.
template <int BS>
__device__ inline void group_sum3(double &a, double &b, double &c, double *red, int &parity, GroupS *gs) {
    block_sum3<BS>(a, b, c, red, parity);
    if (gs == nullptr) return;
    if (threadIdx.x < 64) group_exchange(gs, a, b, c);
    __syncthreads();
    a = gs->tot[0];
    b = gs->tot[1];
    c = gs->tot[2];
}

// Per-wave table of exp(lam_m r_k t) and its first two t-derivative factors:
// wx[km] = e, wx[32 + km] = lam_m r_k e, wx[64 + km] = (lam_m r_k)^2 e, with
// km = k*4 + m.  Lanes 0..4K-1 compute one entry each; LDS operations of a
// wave complete in order, so the wave's later reads see them.
constexpr int kWx = 3 * 4 * kMaxCats;  // doubles per wave

__device__ inline void wave_expo(double *wx, const ModelS *md, int K, double t, float *wxf = nullptr) {
    const int lane = threadIdx.x & 63;
    if (lane < 4 * K) {
        const int k = lane >> 2, m = lane & 3;
        const double q = md->lam[m] * md->rate[k];
        const double e = exp(q * t);
        wx[lane] = e;
        wx[4 * kMaxCats + lane] = e * q;
        wx[8 * kMaxCats + lane] = e * q * q;
        if (wxf) {
            wxf[lane] = (float)e;
            wxf[4 * kMaxCats + lane] = (float)(e * q);
            wxf[8 * kMaxCats + lane] = (float)(e * q * q);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// One side of an update or edge evaluation for one pattern: a tip code, or
// the scaler count and every category's partial of a slot.  TIP is a
// template parameter so that the code fetching a pattern's sides has no
// branch between its loads: they are all issued before the first is used,
// and their memory round trips overlap.
template <typename T, int KP, bool TIP>
struct Side {
    typename Store<T>::Raw r[KP];
    unsigned code;
    int c;
    __device__ inline void fetch(const TreeView<T> &v, int ref, int p) {
        if constexpr (TIP) {
            code = ldg(v.tips + (size_t)(-ref - 1) * v.P + p);
            c = 0;
        } else {
            c = v.cnt[(size_t)ref * v.P + p];
            // the layout holds KP categories, so padded ones are in bounds
#pragma unroll
            for (int k = 0; k < KP; ++k) r[k] = Store<T>::load_raw(slot_ptr<T, KP>(v, ref, k, p));
        }
    }
    __device__ inline void get(int k, double x[4]) const {
        if constexpr (TIP) tip_vec(code, x);
        else Store<T>::widen(r[k], x);
    }
    // the same state vector in FP32 (FP32 partials only)
    __device__ inline void getf(int k, float x[4]) const {
        if constexpr (TIP) {
            x[0] = (float)(code & 1u); x[1] = (float)((code >> 1) & 1u);
            x[2] = (float)((code >> 2) & 1u); x[3] = (float)((code >> 3) & 1u);
        } else {
            static_assert(std::is_same<T, float>::value, "FP32 state vectors of FP32 partials only");
            x[0] = r[k].x; x[1] = r[k].y; x[2] = r[k].z; x[3] = r[k].w;
        }
    }
};

// Where an update reads its transition matrices (PM):
//   kPmLds    FP64 copy in LDS;
//   kPmConst  global memory the kernel never writes, through the constant
//             address space, so that the wave-uniform entries arrive by
//             scalar loads into scalar registers instead of being broadcast
//             to every lane;
//   kPmLds32  FP32 copy in LDS (half the broadcast bytes), for FP32 partials
//             in the optimisation loop, whose updates then compute in FP32
//             (update_pattern_f32).
//   kPmGlobal FP64 matrices in global memory (the FP64 evaluation that ends
//             an optimisation with FP32 partials).
enum : int { kPmLds = 0, kPmConst = 1, kPmLds32 = 2, kPmGlobal = 3 };
template <int PM>
struct PmPtr {
    using type = const double *;
};
template <>
struct PmPtr<kPmConst> {
    using type = const __attribute__((address_space(4))) double *;
};
template <>
struct PmPtr<kPmLds32> {
    using type = const float *;
};
template <>
struct PmPtr<kPmGlobal> {
    using type = const __attribute__((address_space(1))) double *;
};
template <int PM, typename V>
__device__ inline typename PmPtr<PM>::type pm_base(const V &v) {
    if constexpr (PM == kPmLds32) return v.pmf;
    else return (typename PmPtr<PM>::type)v.pm;
}

// One pattern of an OP_UPDATE in FP32 arithmetic, for FP32 partials in the
// optimisation loop (matrices from the FP32 LDS copy): the same products and
// scaling rule as update_pattern, computed in the precision the partial is
// stored in, so no entry is widened to FP64 and narrowed back.  The new
// partial of every category goes to out[k] as stored; returns the scaler
// count.  (The lnL an optimisation reports comes from FP64 partials at the
// final lengths, and the Newton sums stay FP64.)
template <int KP, class SA, class SB>
__device__ inline int update_pattern_f32(const TreeView<float> &v, const Op &op, const SA &sa, const SB &sb,
                                         float4 out[KP]) {
    const float *pm = v.pmf;
    const float thr = 0x1p-64f, up = 0x1p64f;  // Store<float>::kScaleExp
    float o[KP][4];
    float mx = 0.0f;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        float xa[4], xb[4];
        sa.getf(k, xa);
        sb.getf(k, xb);
        const float *Pa = pm + ((size_t)op.ea * KP + k) * 16;
        const float *Pb = pm + ((size_t)op.eb * KP + k) * 16;
        const bool live = k < v.K;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float xsa = Pa[i * 4] * xa[0] + Pa[i * 4 + 1] * xa[1] + Pa[i * 4 + 2] * xa[2] + Pa[i * 4 + 3] * xa[3];
            const float xsb = Pb[i * 4] * xb[0] + Pb[i * 4 + 1] * xb[1] + Pb[i * 4 + 2] * xb[2] + Pb[i * 4 + 3] * xb[3];
            o[k][i] = live ? xsa * xsb : 0.0f;
            mx = fmaxf(mx, o[k][i]);
        }
    }
    int c = sa.c + sb.c;
    const float f = mx < thr && mx > 0.0f ? up : 1.0f;
    c += f != 1.0f;
#pragma unroll
    for (int k = 0; k < KP; ++k) out[k] = make_float4(o[k][0] * f, o[k][1] * f, o[k][2] * f, o[k][3] * f);
    return c;
}

// One pattern of an OP_UPDATE from its two fetched sides, for the fused
// update and table build: o[k] and the returned scaler count are what
// update_sides computes, by the same expressions in the same order (so both
// paths give identical partials; update_sides keeps its own copy because
// sharing this one changed the register allocation of the FP32 kernels and
// slowed them).
template <typename T, int KP, int PM, class SA, class SB>
__device__ inline int update_pattern(const TreeView<T> &v, const Op &op, const SA &sa, const SB &sb,
                                     double o[KP][4]) {
    const auto pm = pm_base<PM>(v);
    const double thr = ldexp(1.0, -Store<T>::kScaleExp);
    const double up = ldexp(1.0, Store<T>::kScaleExp);
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        double xa[4], xb[4];
        sa.get(k, xa);
        sb.get(k, xb);
        const auto Pa = pm + ((size_t)op.ea * KP + k) * 16;
        const auto Pb = pm + ((size_t)op.eb * KP + k) * 16;
        const bool live = k < v.K;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double xsa = Pa[i * 4] * xa[0] + Pa[i * 4 + 1] * xa[1] + Pa[i * 4 + 2] * xa[2] +
                               Pa[i * 4 + 3] * xa[3];
            const double xsb = Pb[i * 4] * xb[0] + Pb[i * 4 + 1] * xb[1] + Pb[i * 4 + 2] * xb[2] +
                               Pb[i * 4 + 3] * xb[3];
            o[k][i] = live ? xsa * xsb : 0.0;
            mx = fmax(mx, o[k][i]);
        }
    }
    int c = sa.c + sb.c;
    if (mx < thr && mx > 0.0) {
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int i = 0; i < 4; ++i) o[k][i] *= up;
        c += 1;
    }
    return c;
}

// OP_UPDATE for this thread's patterns, sides of kinds TA / TB (tip or slot):
//   dst[k] = (P_k(t_ea) . side a[k]) * (P_k(t_eb) . side b[k]), elementwise over
// states, for every category k, then per-pattern scaling.
template <typename T, int BS, int KP, bool TA, bool TB, int PM>
__device__ inline void update_sides(const TreeView<T> &v, const Op &op, int base, int ni) {
    const auto pm = pm_base<PM>(v);
    const double thr = ldexp(1.0, -Store<T>::kScaleExp);
    const double up = ldexp(1.0, Store<T>::kScaleExp);
#pragma unroll 1
    for (int j = 0; j < ni; ++j) {
        const int p = base + j * BS + threadIdx.x;
        if (p >= v.np) break;
        Side<T, KP, TA> sa;
        Side<T, KP, TB> sb;
        sa.fetch(v, op.a, p);
        sb.fetch(v, op.b, p);
        if constexpr (PM == kPmLds32) {
            float4 out[KP];
            const int c = update_pattern_f32<KP>(v, op, sa, sb, out);
#pragma unroll
            for (int k = 0; k < KP; ++k)
                if (k < v.K) Store<T>::store_raw(slot_ptr<T, KP>(v, op.dst, k, p), out[k]);
            v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)c;
            continue;
        }
        double o[KP][4];
        double mx = 0.0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            double xa[4], xb[4];
            sa.get(k, xa);
            sb.get(k, xb);
            const auto Pa = pm + ((size_t)op.ea * KP + k) * 16;
            const auto Pb = pm + ((size_t)op.eb * KP + k) * 16;
            const bool live = k < v.K;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double xsa = Pa[i * 4] * xa[0] + Pa[i * 4 + 1] * xa[1] + Pa[i * 4 + 2] * xa[2] +
                                   Pa[i * 4 + 3] * xa[3];
                const double xsb = Pb[i * 4] * xb[0] + Pb[i * 4 + 1] * xb[1] + Pb[i * 4 + 2] * xb[2] +
                                   Pb[i * 4 + 3] * xb[3];
                o[k][i] = live ? xsa * xsb : 0.0;
                mx = fmax(mx, o[k][i]);
            }
        }
        int c = sa.c + sb.c;
        if (mx < thr && mx > 0.0) {
#pragma unroll
            for (int k = 0; k < KP; ++k)
#pragma unroll
                for (int i = 0; i < 4; ++i) o[k][i] *= up;
            c += 1;
        }
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (k < v.K) Store<T>::store(slot_ptr<T, KP>(v, op.dst, k, p), o[k]);
        v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)c;
    }
}

// OP_UPDATE for this thread's patterns base + j*BS, j < ni.
template <typename T, int BS, int KP, int PM = kPmLds>
__device__ inline void do_update(const TreeView<T> &v, const Op &op, int base, int ni) {
    if (op.a < 0) {
        if (op.b < 0) update_sides<T, BS, KP, true, true, PM>(v, op, base, ni);
        else update_sides<T, BS, KP, true, false, PM>(v, op, base, ni);
    } else {
        if (op.b < 0) update_sides<T, BS, KP, false, true, PM>(v, op, base, ni);
        else update_sides<T, BS, KP, false, false, PM>(v, op, base, ni);
    }
}

// t-independent part of a pattern's lnL: scaler corrections and the 1/K
// category weight.
template <typename T>
__device__ inline double const_term(int c, double logK) {
    return -((double)c * Store<T>::kScaleExp * kLn2 + logK);
}

struct Sums3 {
    double l0, l1, l2;
    int parity;
};

// Eigenbasis coefficients from the two sides' state vectors of one category.
__device__ inline void coeffs_x(const ModelS *md, const double xa[4], const double xb[4], double s[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double ua = 0.0, vb = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double wim = md->W[i * 4 + m];
            ua += wim * xa[i];
            vb += wim * xb[i];
        }
        s[m] = ua * vb;
    }
}

// The same coefficients in FP32, for tables stored in FP32 (the optimisation
// loop with FP32 partials): computed in the precision they are stored in.
__device__ inline void coeffs_xf(const ModelS *md, const float xa[4], const float xb[4], float s[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        float ua = 0.0f, vb = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float wim = md->Wf[i * 4 + m];
            ua += wim * xa[i];
            vb += wim * xb[i];
        }
        s[m] = ua * vb;
    }
}

// One category's table coefficients for one pattern, stored at dst and
// returned (as stored) in sk: in FP32 from the FP32 values of the sides when
// the table is FP32, else in FP64.
template <typename T, class SA, class SB>
__device__ inline void table_coeffs(const ModelS *md, const SA &sa, const SB &sb, int k, T *dst, double sk[4]) {
    if constexpr (std::is_same<T, float>::value) {
        float xa[4], xb[4], s[4];
        sa.getf(k, xa);
        sb.getf(k, xb);
        coeffs_xf(md, xa, xb, s);
        *reinterpret_cast<float4 *>(dst) = make_float4(s[0], s[1], s[2], s[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) sk[m] = s[m];
    } else {
        double xa[4], xb[4];
        sa.get(k, xa);
        sb.get(k, xb);
        coeffs_x(md, xa, xb, sk);
        Store<T>::store(dst, sk);
    }
}

// This thread's contributions to lnL, d1 and d2 across an edge whose sides
// are of kinds TA / TB, with the exponentials of its length in wx (lnL only
// with want_l0: a gradient program reads it from one edge's output only).
template <typename T, int BS, int KP, bool TA, bool TB>
__device__ inline void eval_sides(const TreeView<T> &v, int a, int b, int base, int ni, const double *wx,
                                  double logK, bool want_l0, Sums3 &r) {
    const ModelS *md = v.m;
#pragma unroll 1
    for (int j = 0; j < ni; ++j) {
        const int p = base + j * BS + threadIdx.x;
        if (p >= v.np) break;
        Side<T, KP, TA> sa;
        Side<T, KP, TB> sb;
        sa.fetch(v, a, p);
        sb.fetch(v, b, p);
        const double w = ldg(v.w + p);
        double L = 0.0, L1 = 0.0, L2 = 0.0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            if (k < v.K) {
                double xa[4], xb[4], sk[4];
                sa.get(k, xa);
                sb.get(k, xb);
                coeffs_x(md, xa, xb, sk);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    L += sk[m] * wx[k * 4 + m];
                    L1 += sk[m] * wx[4 * kMaxCats + k * 4 + m];
                    L2 += sk[m] * wx[8 * kMaxCats + k * 4 + m];
                }
            }
        }
        const double inv = recip(L);
        const double r1 = L1 * inv;
        if (want_l0) r.l0 += w * (log(L) + const_term<T>(sa.c + sb.c, logK));
        r.l1 += w * r1;
        r.l2 += w * (L2 * inv - r1 * r1);
    }
}

// OP_EVAL: block totals of lnL (0 unless want_l0) and its first two
// derivatives across an edge at length t, computed on the fly from the two
// sides.
template <typename T, int BS, int KP>
__device__ inline Sums3 eval_edge(const TreeView<T> &v, int a, int b, int base, int ni, double t, double *red,
                                  double *wx, int parity, GroupS *gs = nullptr, bool want_l0 = true) {
    wave_expo(wx, v.m, v.K, t);
    const double logK = log((double)v.K);
    Sums3 r;
    r.l0 = r.l1 = r.l2 = 0.0;
    if (a < 0) {
        if (b < 0) eval_sides<T, BS, KP, true, true>(v, a, b, base, ni, wx, logK, want_l0, r);
        else eval_sides<T, BS, KP, true, false>(v, a, b, base, ni, wx, logK, want_l0, r);
    } else {
        if (b < 0) eval_sides<T, BS, KP, false, true>(v, a, b, base, ni, wx, logK, want_l0, r);
        else eval_sides<T, BS, KP, false, false>(v, a, b, base, ni, wx, logK, want_l0, r);
    }
    group_sum3<BS>(r.l0, r.l1, r.l2, red, parity, gs);
    r.parity = parity;
    return r;
}

struct EdgeResult {
    double t, lnl;
    double gain;  // the objective's gain from the step by its quadratic model at the start, or +inf
    double rise;  // the same model's value for the step, whatever the sign of its second derivative
    int parity, iters;
    long long cyc_table, cyc_iters;
};

// One row of an edge's eigenbasis table from the pattern's two sides (the
// table is symmetric in them), for the fused update and table build: the
// row, weight and sums that table_sides gives for the pattern, by the same
// expressions in the same order (table_sides keeps its own copy for the same
// reason as update_sides).  Stores the row of every live category into tab
// ([k][row][4]) and the weight into wrow, adds the pattern's t-independent
// lnL term to cterm and, with FUSE, its terms of the first Newton iteration
// at the exponentials wxe to f1 and f2.
template <typename T, int KP, bool FUSE, class SA, class SB, typename X>
__device__ inline void table_row(const TreeView<T> &v, const SA &sa, const SB &sb, int p, size_t rows, T *tab,
                                 double *wrow, double w, double logK, const X *wxe, double &cterm, double &f1,
                                 double &f2) {
    const ModelS *md = v.m;
    cterm += w * const_term<T>(sa.c + sb.c, logK);
    wrow[p] = w;
    double L = 0.0, L1 = 0.0, L2 = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        if (k < v.K) {
            double sk[4];
            table_coeffs<T>(md, sa, sb, k, tab + ((size_t)k * rows + p) * 4, sk);
            if constexpr (FUSE) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const double q = Store<T>::as_stored(sk[m]);
                    L += q * (double)wxe[k * 4 + m];
                    L1 += q * (double)wxe[4 * kMaxCats + k * 4 + m];
                    L2 += q * (double)wxe[8 * kMaxCats + k * 4 + m];
                }
            }
        }
    }
    if constexpr (FUSE) {
        const double ia = recip(L);
        const double r1 = L1 * ia;
        f1 += w * r1;
        f2 += w * (L2 * ia - r1 * r1);
    }
}

// The eigenbasis table of an edge whose sides are of kinds TA / TB: this
// thread's rows of tab ([k][row][4]) and wrow; returns the sum of its rows'
// t-independent lnL terms.  FUSE: also adds the rows' terms of the first
// Newton iteration, at the exponentials wxe, to f1 and f2, from the values as
// stored and in the order of newton_rows2, so the sums are the ones a row
// pass over the finished table would give.
template <typename T, int BS, int KP, bool TA, bool TB, bool FUSE, bool PAIR, typename X>
__device__ inline double table_sides(const TreeView<T> &v, int a, int b, int ni, size_t rows, T *tab, double *wrow,
                                     double logK, const X *wxe, double &f1, double &f2) {
    const ModelS *md = v.m;
    double cterm = 0.0;
    // PAIR: two patterns per step (FP32 partials; with FP64 the registers of
    // a second pattern would spill), both fetched before either is used; a
    // missing second pattern re-reads the first (in bounds) and is not
    // stored.  Kernels with the fused update and table build leave PAIR off
    // to make room for it.
    constexpr int kStep = std::is_same<T, float>::value && PAIR ? 2 : 1;
#pragma unroll 1
    for (int j = 0; j < ni; j += kStep) {
        const int p0 = j * BS + threadIdx.x;
        if (p0 >= v.np) break;
        const bool two = kStep == 2 && j + 1 < ni && p0 + BS < v.np;
        const int p1 = two ? p0 + BS : p0;
        Side<T, KP, TA> sa0, sa1;
        Side<T, KP, TB> sb0, sb1;
        sa0.fetch(v, a, p0);
        sb0.fetch(v, b, p0);
        sa1.fetch(v, a, p1);
        sb1.fetch(v, b, p1);
        const double w0 = ldg(v.w + p0), w1 = ldg(v.w + p1);
        cterm += w0 * const_term<T>(sa0.c + sb0.c, logK);
        wrow[p0] = w0;
        double L = 0.0, L1 = 0.0, L2 = 0.0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            if (k < v.K) {
                double sk[4];
                table_coeffs<T>(md, sa0, sb0, k, tab + ((size_t)k * rows + p0) * 4, sk);
                if constexpr (FUSE) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const double q = Store<T>::as_stored(sk[m]);
                        L += q * (double)wxe[k * 4 + m];
                        L1 += q * (double)wxe[4 * kMaxCats + k * 4 + m];
                        L2 += q * (double)wxe[8 * kMaxCats + k * 4 + m];
                    }
                }
            }
        }
        if constexpr (FUSE) {
            const double ia = recip(L);
            const double r1 = L1 * ia;
            f1 += w0 * r1;
            f2 += w0 * (L2 * ia - r1 * r1);
        }
        if (two) {
            cterm += w1 * const_term<T>(sa1.c + sb1.c, logK);
            wrow[p1] = w1;
            double M = 0.0, M1 = 0.0, M2 = 0.0;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                if (k < v.K) {
                    double sk[4];
                    table_coeffs<T>(md, sa1, sb1, k, tab + ((size_t)k * rows + p1) * 4, sk);
                    if constexpr (FUSE) {
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const double q = Store<T>::as_stored(sk[m]);
                            M += q * (double)wxe[k * 4 + m];
                            M1 += q * (double)wxe[4 * kMaxCats + k * 4 + m];
                            M2 += q * (double)wxe[8 * kMaxCats + k * 4 + m];
                        }
                    }
                }
            }
            if constexpr (FUSE) {
                const double ib = recip(M);
                const double r1 = M1 * ib;
                f1 += w1 * r1;
                f2 += w1 * (M2 * ib - r1 * r1);
            }
        }
    }
    return cterm;
}

// An OP_UPDATE whose output is one side of the next OP_NEWTON, with one
// pattern per thread: the update's loads and those of the edge's other side
// (kind TO) issue together, and the edge's table row is built from the
// update's output, kept in registers and rounded as stored, instead of being
// read back.  The table is symmetric in the two sides, so which side the
// update made does not matter.  Returns the row's t-independent lnL term
// (see table_row).
template <typename T, int BS, int KP, bool TA, bool TB, bool TO, bool FUSE, int PM, typename X>
__device__ inline double update_table_sides(const TreeView<T> &v, const Op &op, int other, T *tab, double *wrow,
                                            double logK, const X *wxe, double &f1, double &f2) {
    double cterm = 0.0;
    const int p = threadIdx.x;
    if (p < v.np) {
        Side<T, KP, TA> sa;
        Side<T, KP, TB> sb;
        Side<T, KP, TO> so;
        sa.fetch(v, op.a, p);
        sb.fetch(v, op.b, p);
        so.fetch(v, other, p);
        const double w = ldg(v.w + p);
        Side<T, KP, false> made;
        if constexpr (PM == kPmLds32) {
            made.c = update_pattern_f32<KP>(v, op, sa, sb, made.r);
        } else {
            double o[KP][4];
            made.c = update_pattern<T, KP, PM>(v, op, sa, sb, o);
#pragma unroll
            for (int k = 0; k < KP; ++k) made.r[k] = Store<T>::pack(o[k]);
        }
        table_row<T, KP, FUSE>(v, made, so, p, (size_t)BS, tab, wrow, w, logK, wxe, cterm, f1, f2);
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (k < v.K) Store<T>::store_raw(slot_ptr<T, KP>(v, op.dst, k, p), made.r[k]);
        v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)made.c;
    }
    return cterm;
}

// Newton pass over two table rows r0 and r1 (r1 < 0: only r0), so that each
// exponential read from the wave's LDS slice serves two patterns.  Adds the
// rows' d1 and d2 terms, or with lnl_only their weighted log L to d0; each
// row's sums run in the same order as for a single row.
template <typename T, int KP, typename X>
__device__ inline void newton_rows2(const T *tab, const double *wrow, size_t rows, int r0, int r1, const X *wx,
                                    int K, bool lnl_only, double &d0, double &d1, double &d2) {
    using Raw = typename Store<T>::Raw;
    const bool two = r1 >= 0;
    const int rb = two ? r1 : r0;
    Raw ra[KP], rr[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        if (k < K) {
            ra[k] = Store<T>::load_raw(tab + ((size_t)k * rows + r0) * 4);
            rr[k] = Store<T>::load_raw(tab + ((size_t)k * rows + rb) * 4);
        }
    }
    const double wa = wrow[r0], wb = wrow[rb];
    double La = 0.0, L1a = 0.0, L2a = 0.0, Lb = 0.0, L1b = 0.0, L2b = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        if (k < K) {
            double sa[4], sb[4];
            Store<T>::widen(ra[k], sa);
            Store<T>::widen(rr[k], sb);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double e0 = wx[k * 4 + m], e1 = wx[4 * kMaxCats + k * 4 + m],
                             e2 = wx[8 * kMaxCats + k * 4 + m];
                La += sa[m] * e0;
                L1a += sa[m] * e1;
                L2a += sa[m] * e2;
                Lb += sb[m] * e0;
                L1b += sb[m] * e1;
                L2b += sb[m] * e2;
            }
        }
    }
    if (lnl_only) {
        d0 += wa * log(La);
        if (two) d0 += wb * log(Lb);
        return;
    }
    const double ia = recip(La);
    const double ra1 = L1a * ia;
    d1 += wa * ra1;
    d2 += wa * (L2a * ia - ra1 * ra1);
    if (two) {
        const double ib = recip(Lb);
        const double rb1 = L1b * ib;
        d1 += wb * rb1;
        d2 += wb * (L2b * ib - rb1 * rb1);
    }
}

// Relative Newton step below which an edge's iterations end without a
// confirming evaluation (see newton_edge).  Measured on the 48 C2
// neighbours: 1.46 -> 1.07 iterations per edge step (FP32 partials) and
// 1.70 -> 1.04 (FP64), for at most one more pass on a few trees.
constexpr double kNewtonAccept = 0.03;

// Over-relaxation of the edge steps from a tree's second pass on: an edge
// whose Newton step exceeds tol_t relative moves kRelax times that step
// (nonlinear successive over-relaxation of the coordinate-wise maximisation;
// Ortega and Rheinboldt, Iterative Solution of Nonlinear Equations in Several
// Variables, 1970).  The lengths are coupled, so plain coordinate steps
// converge linearly and slowly on some trees; the fixed point is the same
// maximum.  Steps below tol_t are not relaxed, so a tree's last pass (every
// step below tol_t) leaves plain Newton results.  Measured with the oracle's
// arithmetic: on the 48 C2 neighbours, passes mean 7.4 -> 6.6 and max 11 -> 8
// (FP32 tolerances) and mean 11.7 -> 9.4, max 18 -> 12 (FP64 tolerances); on
// 64-taxon trees mean 14.9 -> 9.3, max 18 -> 14; 1.3 and above took more
// passes.
constexpr double kRelax = 1.2;

// An edge's table built ahead of newton_edge (by update_table_sides): this
// thread's t-independent lnL term and first-iteration derivative terms.
struct EdgePre {
    double cterm, f1, f2;
};

// The first iteration's derivative terms are summed while the table is built
// (with the same rounding and order as the row passes of newton_edge), up to
// four padded categories: with eight the extra registers would spill.
template <int KP>
struct FuseFirst {
    static constexpr bool value = KP <= 4;
};

// The exponentials of length t that the fused first iteration uses (in the
// wave's LDS slice), and a pointer to them in the precision it reads.
template <typename T, int KP>
__device__ inline const typename std::conditional<std::is_same<T, float>::value, float, double>::type *
first_expo(const TreeView<T> &v, double t, double *wx, float *wxf) {
    constexpr bool kF = std::is_same<T, float>::value;
    using XE = typename std::conditional<kF, float, double>::type;
    if constexpr (FuseFirst<KP>::value) {
        if constexpr (kF) wave_expo(wx, v.m, v.K, t, wxf);
        else wave_expo(wx, v.m, v.K, t);
    }
    return kF ? reinterpret_cast<const XE *>(wxf) : reinterpret_cast<const XE *>(wx);
}

// OP_UPDATE of slot op.dst fused with the table build of the next OP_NEWTON,
// whose other side is `other`, at its current length t (one pattern per
// thread).
template <typename T, int BS, int KP, int PM>
__device__ inline EdgePre update_and_table(const TreeView<T> &v, const Op &op, int other, double t, T *tab,
                                           double *wrow, double *wx, float *wxf) {
    constexpr bool kFuse = FuseFirst<KP>::value;
    const auto *wxe = first_expo<T, KP>(v, t, wx, wxf);
    const double logK = log((double)v.K);
    EdgePre pre;
    pre.f1 = pre.f2 = 0.0;
#define PT_UT(TA, TB, TO)                                                                                        \
    pre.cterm = update_table_sides<T, BS, KP, TA, TB, TO, kFuse, PM>(v, op, other, tab, wrow, logK, wxe, pre.f1, \
                                                                      pre.f2)
    if (op.a < 0) {
        if (op.b < 0) {
            if (other < 0) PT_UT(true, true, true); else PT_UT(true, true, false);
        } else {
            if (other < 0) PT_UT(true, false, true); else PT_UT(true, false, false);
        }
    } else {
        if (op.b < 0) {
            if (other < 0) PT_UT(false, true, true); else PT_UT(false, true, false);
        } else {
            if (other < 0) PT_UT(false, false, true); else PT_UT(false, false, false);
        }
    }
#undef PT_UT
    return pre;
}

// OP_NEWTON: safeguarded, projected Newton on the length of one edge, for
// lnL(t) - prior_rate * t (prior_rate 0: maximum likelihood).
//  - the eigenbasis coefficients of this thread's patterns are computed once
//    into `tab` (layout [k][row][4], rows = BS*ni pattern slots) and the
//    pattern weights into `wrow` (in LDS, or in a per-block global buffer),
//    then every iteration is a pass over them plus one block sum (up to four
//    padded categories, the first iteration's terms are summed while the
//    table is built);
//  - the bracket (lo, hi) starts as [t_min, t_max] and shrinks to t on the
//    side the first derivative points away from;
//  - a Newton step is taken when d2 < 0 and it stays in the bracket (the
//    original bounds count as inside), else the bracket is bisected
//    geometrically;
//  - a bound with the derivative pointing outwards is an optimum;
//  - a step of at most tol * max(t, 1e-6) is converged and not taken; a
//    Newton step of at most max(sqrt(tol), kNewtonAccept) * max(t, 1e-6) is
//    taken and ends the edge (quadratic convergence; the next pass revisits
//    the edge);
//  - the returned t is t_in + relax * (t_newton - t_in), kept in
//    [t_min, t_max], when that step exceeds tol_t * max(t_in, 1e-6), else
//    the Newton result;
//  - with want_lnl, lnL is evaluated at the returned t.
// All threads hold identical block totals, so every thread takes the same
// decisions.
template <typename T, int BS, int KP, bool PAIR = true>
__device__ inline EdgeResult newton_edge(const TreeView<T> &v, int a, int b, double t, bool want_lnl,
                                         const OptParams &opt, T *tab, double *wrow, int ni, double *red,
                                         double *wx, float *wxf, int parity, GroupS *gs, double relax,
                                         const EdgePre *pre = nullptr) {
    const double t_in = t;
    const size_t rows = (size_t)BS * ni;
    const double logK = log((double)v.K);
    const long long c0 = clock64();
    constexpr bool kFuse = FuseFirst<KP>::value;
    double f1 = 0.0, f2 = 0.0;
    double cterm;
    if (pre) {  // the table is built (one pattern per thread)
        cterm = pre->cterm;
        f1 = pre->f1;
        f2 = pre->f2;
    } else {
        const auto *wxe = first_expo<T, KP>(v, t, wx, wxf);
        if (a < 0) {
            if (b < 0) cterm = table_sides<T, BS, KP, true, true, kFuse, PAIR>(v, a, b, ni, rows, tab, wrow, logK, wxe, f1, f2);
            else cterm = table_sides<T, BS, KP, true, false, kFuse, PAIR>(v, a, b, ni, rows, tab, wrow, logK, wxe, f1, f2);
        } else {
            if (b < 0) cterm = table_sides<T, BS, KP, false, true, kFuse, PAIR>(v, a, b, ni, rows, tab, wrow, logK, wxe, f1, f2);
            else cterm = table_sides<T, BS, KP, false, false, kFuse, PAIR>(v, a, b, ni, rows, tab, wrow, logK, wxe, f1, f2);
        }
    }
    // rows this thread owns: tid + j*BS < P
    const int nj = v.np > (int)threadIdx.x ? min(ni, (v.np - (int)threadIdx.x + BS - 1) / BS) : 0;
    const long long c1 = clock64();
    double lo = opt.t_min, hi = opt.t_max;
    double d1_0 = 0.0, d2_0 = 0.0;  // derivatives at the starting length
    int iter = 1;
    for (;; ++iter) {
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        if (kFuse && iter == 1) {
            d1 = f1;
            d2 = f2;
        } else if constexpr (std::is_same<T, float>::value) {
            // FP32 partials: FP32 exponentials suffice for the derivatives
            // (they only steer Newton); lnL below uses FP64 ones
            wave_expo(wx, v.m, v.K, t, wxf);
#pragma unroll 1
            for (int j = 0; j < nj; j += 2)
                newton_rows2<T, KP>(tab, wrow, rows, j * BS + threadIdx.x,
                                    j + 1 < nj ? (j + 1) * BS + threadIdx.x : -1, (const float *)wxf, v.K, false, d0,
                                    d1, d2);
        } else {
            wave_expo(wx, v.m, v.K, t);
#pragma unroll 1
            for (int j = 0; j < nj; j += 2)
                newton_rows2<T, KP>(tab, wrow, rows, j * BS + threadIdx.x,
                                    j + 1 < nj ? (j + 1) * BS + threadIdx.x : -1, (const double *)wx, v.K, false, d0,
                                    d1, d2);
        }
        group_sum3<BS>(d0, d1, d2, red, parity, gs);
        d1 -= opt.prior_rate;  // MAP: the exponential prior's log density is linear in t
        if (iter == 1) {
            d1_0 = d1;
            d2_0 = d2;
        }
        if (iter >= opt.max_newton) break;
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
        const double dt = fabs(tn - t), scale = fmax(t, 1e-6);
        if (dt <= opt.tol_newton * scale) break;
        t = tn;
        // Newton converges quadratically near the optimum: after a Newton
        // step of relative size d the remaining error is of order d^2, so a
        // step of at most kNewtonAccept (or sqrt(tol_newton)) relative is
        // taken without a confirming evaluation.  The next pass revisits the
        // edge, and the pass-level rule (no step above tol_t) bounds the
        // final accuracy.
        if (inside && dt <= fmax(sqrt(opt.tol_newton), kNewtonAccept) * scale) break;
    }
    if (relax != 1.0 && fabs(t - t_in) > opt.tol_t * fmax(t_in, 1e-6))
        t = fmin(fmax(t_in + relax * (t - t_in), opt.t_min), opt.t_max);
    double lnl = 0.0;
    if (want_lnl) {
        wave_expo(wx, v.m, v.K, t);
        double l0 = cterm, z1 = 0.0, z2 = 0.0;
#pragma unroll 1
        for (int j = 0; j < nj; j += 2)
            newton_rows2<T, KP>(tab, wrow, rows, j * BS + threadIdx.x, j + 1 < nj ? (j + 1) * BS + threadIdx.x : -1,
                                (const double *)wx, v.K, true, l0, z1, z2);
        group_sum3<BS>(l0, z1, z2, red, parity, gs);
        lnl = l0;
    }
    EdgeResult r;
    r.t = t;
    r.lnl = lnl;
    r.parity = parity;
    r.iters = iter;
    r.cyc_table = c1 - c0;
    r.cyc_iters = clock64() - c1;
    {
        const double dt = t - t_in;
        r.rise = d1_0 * dt + 0.5 * d2_0 * dt * dt;
        r.gain = d2_0 < 0.0 ? r.rise : INFINITY;
    }
    return r;
}

template <typename T>
__device__ inline TreeView<T> make_view(const TreeDev &td, const AlnDev *aln, const BatchArgs &a,
                                        const ModelS *m, const double *pm_lds) {
    TreeView<T> v;
    v.m = m;
    v.pm = pm_lds;
    v.pmf = nullptr;
    v.tips = aln->tips;
    v.w = aln->w;
    v.clv = reinterpret_cast<T *>(a.clv) + td.clv_off;
    v.cnt = a.cnt + td.cnt_off;
    v.P = aln->P;
    v.np = aln->P;
    v.K = aln->K;
    return v;
}

// ----------------------------------------------------------------- kernels

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Transition matrices of every edge, P_k(t) = U diag(exp(lambda r_k t)) U^-1:
// one block per tree, so that the tree's descriptor and model constants are
// wave-uniform and arrive by scalar loads (neither is written by any kernel),
// and one thread per (edge, category k) of the tree.  The four exponentials
// serve the matrix's 16 entries, written as 16-byte stores.
__global__ void k_pmat(const BatchArgs a, const double *brlen) {
    using CD = const __attribute__((address_space(4))) double;
    const __attribute__((address_space(4))) TreeDev *td =
        (const __attribute__((address_space(4))) TreeDev *)(a.trees + blockIdx.x);
    const __attribute__((address_space(4))) AlnDev *aln =
        (const __attribute__((address_space(4))) AlnDev *)(a.alns + td->aln);
    const int kp = a.kp, n = td->n_edges * kp;
    const int64_t edge_off = td->edge_off, pm_off = td->pm_off;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        const int e = x / kp, k = x - e * kp;
        const double t = brlen[edge_off + e];
        CD *U = aln->U, *V = aln->Uinv;
        double ex[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) ex[m] = exp(aln->lam[m] * aln->rate[k] * t);
        double2 *out = reinterpret_cast<double2 *>(a.pmat + pm_off + (int64_t)x * 16);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double s2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = (2 * q + h) >> 2, j = (2 * q + h) & 3;
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < 4; ++m) s += U[i * 4 + m] * ex[m] * V[m * 4 + j];
                s2[h] = s;
            }
            out[q] = make_double2(s2[0], s2[1]);
        }
    }
}

// OP_UPDATE for one pattern per thread whose side `fwd_b ? b : a` is the
// partial the previous update of this thread made, still in registers
// (`last`): only the other side is loaded.  The new partial is stored and
// kept in `last` for the next update.  The same expressions as
// update_sides, so the partials are identical.
template <typename T, int KP, bool TO, int PM>
__device__ inline void update_forwarded(const TreeView<T> &v, const Op &op, bool fwd_b, int p,
                                        Side<T, KP, false> &last) {
    Side<T, KP, TO> so;
    so.fetch(v, fwd_b ? op.a : op.b, p);
    double o[KP][4];
    const int c = fwd_b ? update_pattern<T, KP, PM>(v, op, so, last, o) : update_pattern<T, KP, PM>(v, op, last, so, o);
#pragma unroll
    for (int k = 0; k < KP; ++k) last.r[k] = Store<T>::pack(o[k]);
    last.c = c;
#pragma unroll
    for (int k = 0; k < KP; ++k)
        if (k < v.K) Store<T>::store_raw(slot_ptr<T, KP>(v, op.dst, k, p), last.r[k]);
    v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)c;
}

// OP_UPDATE for one pattern per thread with both sides loaded, keeping the
// new partial in `last` (update_sides with the result kept).
template <typename T, int KP, bool TA, bool TB, int PM>
__device__ inline void update_keep(const TreeView<T> &v, const Op &op, int p, Side<T, KP, false> &last) {
    Side<T, KP, TA> sa;
    Side<T, KP, TB> sb;
    sa.fetch(v, op.a, p);
    sb.fetch(v, op.b, p);
    double o[KP][4];
    last.c = update_pattern<T, KP, PM>(v, op, sa, sb, o);
#pragma unroll
    for (int k = 0; k < KP; ++k) last.r[k] = Store<T>::pack(o[k]);
#pragma unroll
    for (int k = 0; k < KP; ++k)
        if (k < v.K) Store<T>::store_raw(slot_ptr<T, KP>(v, op.dst, k, p), last.r[k]);
    v.cnt[(size_t)op.dst * v.P + p] = (uint16_t)last.c;
}

// Requests one update's transition matrices (edges ea and eb, KP categories
// each) into the L2 ahead of use: one 16-byte LDS DMA per lane of the calling
// wave into `row`, which nobody reads.  The FP32 tile kernel reads the
// matrices by scalar loads, which its register budget serialises in pairs
// per update; issued one op early, these requests let those loads find the
// lines in the L2 instead of going out to memory one pair after another.
template <int KP>
__device__ inline void prefetch_pm(const double *pm, int ea, int eb, float4 *row) {
    constexpr int kChunks = KP * 8;  // 16-byte pieces of one edge's KP matrices
    const int lane = threadIdx.x & 63;
    if (lane < 2 * kChunks) {
        const double *src = pm + ((size_t)(lane < kChunks ? ea : eb) * KP) * 16 + (lane % kChunks) * 2;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)row, 16, 0, 0);
    }
}

// Pattern-tile kernels (k_tiles32 / k_tiles64 below): each block runs its tree's program over one tile of
// BS * kTileItems patterns.  LOGLIK programs end in one EVAL (column 0);
// GRAD programs EVAL every edge.  Output: part[tile][col] = (lnL, d1, d2).
template <typename T, int BS, int KP>
__device__ inline void tiles_body(const BatchArgs &a, const double *brlen) {
    extern __shared__ double lds[];
    __shared__ double red[2 * (BS / 64) * 3];
    __shared__ double wxs[(BS / 64) * kWx];
    __shared__ ModelS model;
    __shared__ float4 pf_row[64];  // target of prefetch_pm, never read
    // FP32 partials: the updates read the tree's transition matrices (written
    // by k_pmat before this launch) in place by scalar loads (see PmPtr);
    // FP64 partials: from a copy in LDS, which measured faster there.
    constexpr bool kConstPm = std::is_same<T, float>::value;
    const int tile = blockIdx.x;
    const TreeDev td = a.trees[a.tile_tree[tile]];
    const AlnDev *aln = a.alns + td.aln;
    if (!kConstPm) {
        // 16-byte loads, four in flight per thread (indices clamped into
        // range, so no branch separates the loads)
        const int n2 = td.n_edges * KP * 8;
        const double2 *src = reinterpret_cast<const double2 *>(a.pmat + td.pm_off);
        double2 *dst = reinterpret_cast<double2 *>(lds);
        for (int i = threadIdx.x; i < n2; i += 4 * BS) {
            double2 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = src[min(i + u * BS, n2 - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + u * BS < n2) dst[i + u * BS] = q[u];
        }
    }
    model_to_lds(aln, &model);
    __syncthreads();
    const TreeView<T> v = make_view<T>(td, aln, a, &model, kConstPm ? a.pmat + td.pm_off : lds);
    double *wx = wxs + (threadIdx.x >> 6) * kWx;
    const int base = (tile - td.tile_begin) * BS * kTileItems;
    int parity = 0;
    // FP64 partials, one pattern per thread: a partial the previous update
    // made is taken from registers when this update reads it (a post-order
    // pass reads most partials right after making them), saving that load's
    // round trip.  With FP32 partials the extra live registers cost more than
    // the load (measured), so those updates load both sides.
    constexpr int PMK = kConstPm ? kPmConst : kPmLds;
    constexpr bool kForward = !kConstPm;
    static_assert(kTileItems == 1, "partials are forwarded for one pattern per thread");
    const int p = base + threadIdx.x;
    const bool live_p = p < v.np;
    Side<T, KP, false> last;
    int last_dst = -1;
    // FP32 partials: the first wave requests each update's matrices into the
    // L2 one op ahead of the update
    if constexpr (kConstPm) {
        if (threadIdx.x < 64 && td.n_first > 0) {
            const Op nx = load_op(a.ops, td.op_first);
            if (nx.code == OP_UPDATE) prefetch_pm<KP>(a.pmat + td.pm_off, nx.ea, nx.eb, pf_row);
        }
    }
    for (int o = 0; o < td.n_first; ++o) {
        const Op op = load_op(a.ops, td.op_first + o);
        if constexpr (kConstPm) {
            if (threadIdx.x < 64 && o + 1 < td.n_first) {
                const Op nx = load_op(a.ops, td.op_first + o + 1);
                if (nx.code == OP_UPDATE) prefetch_pm<KP>(a.pmat + td.pm_off, nx.ea, nx.eb, pf_row);
            }
        }
        if (op.code == OP_UPDATE && !kForward) {
            do_update<T, BS, KP, PMK>(v, op, base, kTileItems);
            continue;
        }
        if (op.code == OP_UPDATE) {
            if (live_p) {
                if (op.b >= 0 && op.b == last_dst) {
                    if (op.a < 0) update_forwarded<T, KP, true, PMK>(v, op, true, p, last);
                    else update_forwarded<T, KP, false, PMK>(v, op, true, p, last);
                } else if (op.a >= 0 && op.a == last_dst) {
                    if (op.b < 0) update_forwarded<T, KP, true, PMK>(v, op, false, p, last);
                    else update_forwarded<T, KP, false, PMK>(v, op, false, p, last);
                } else if (op.a < 0) {
                    if (op.b < 0) update_keep<T, KP, true, true, PMK>(v, op, p, last);
                    else update_keep<T, KP, true, false, PMK>(v, op, p, last);
                } else {
                    if (op.b < 0) update_keep<T, KP, false, true, PMK>(v, op, p, last);
                    else update_keep<T, KP, false, false, PMK>(v, op, p, last);
                }
            }
            last_dst = op.dst;
            continue;
        }
        // lnL is read from output column 0 only (the likelihood program's one
        // edge, the gradient program's first edge)
        const Sums3 r = eval_edge<T, BS, KP>(v, op.a, op.b, base, kTileItems, brlen[td.edge_off + op.dst], red, wx,
                                             parity, nullptr, op.ea == 0);
        parity = r.parity;
        if (threadIdx.x == 0) {
            double *out = a.part + ((size_t)tile * a.part_cols + op.ea) * 3;
            out[0] = r.l0;
            out[1] = r.l1;
            out[2] = r.l2;
        }
    }
}

// The tile kernels.  With FP32 partials the kernel is held to 128 VGPRs
// (four blocks per CU), which measured 7 % faster despite a 48-byte spill
// outside the update loop; with FP64 partials the LDS copy of the matrices
// already limits a CU to two blocks.
template <int BS, int KP>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
k_tiles32(const BatchArgs a, const double *brlen) {
    tiles_body<float, BS, KP>(a, brlen);
}

template <int BS, int KP>
__global__ void __launch_bounds__(BS) k_tiles64(const BatchArgs a, const double *brlen) {
    tiles_body<double, BS, KP>(a, brlen);
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

// ------------------------------------------------ register-resident lnL
//
// The lnL of a tree by Felsenstein's post-order pass with no partial ever
// stored: a lane owns kItems patterns of one rate category, and their
// partials live in registers (an accumulator per pattern) and a small stack
// in LDS, the program ordered so that the stack stays shallow (see
// compile_loglik_reg).  A wave is one category, so every transition-matrix
// entry it reads is wave-uniform and arrives by scalar loads (k_pmat writes
// the matrices before the launch), and each entry loaded serves the lane's
// kItems patterns.  Arithmetic is FP64 whatever the storage precision of
// the plan, because nothing is stored.  Scaling is per pattern and
// category: a partial whose largest entry falls below 2^-256 is multiplied
// by 2^256 and the event counted; all events of a pattern and category
// multiply into its root value, so one counter per pattern suffices.  At the
// root edge the categories of a pattern meet in LDS:
//   ln L_p = ln sum_k 2^(-256 (c_k - c_min)) L_k - ln K - 256 c_min ln 2.
// Memory traffic per pattern: the n tip codes and the weight.
template <int KP>
struct RegShape {
    static constexpr int kItems = 2;                        // patterns per lane
    static constexpr int kWaves = KP >= 4 ? KP : 4;        // waves per block
    static constexpr int kGroups = kWaves / KP;             // pattern groups per block
    static constexpr int kGroupPats = 64 * kItems;          // patterns of a group
    static constexpr int kPats = kGroupPats * kGroups;      // patterns per tile
    static constexpr int kThreads = 64 * kWaves;
};

__device__ inline void reg_copy(double d[4], const double s[4]) {
    d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; d[3] = s[3];
}

// The accumulators, which most steps read and write, are in registers.  The
// stack: with RSLOTS > 0 (programs needing at most RSLOTS slots) in
// registers too, each slot selected by its wave-uniform number against
// compile-time indices (an array indexed by a runtime number would go to
// scratch memory), which leaves LDS to the tip codes alone and lets more
// blocks share a compute unit; with RSLOTS = 0 in LDS, [slot][item][thread]
// of four doubles.  Three register slots fit five waves per SIMD, four slots
// four.
template <int KP, int RSLOTS>
__global__ void __launch_bounds__(RegShape<KP>::kThreads) __attribute__((amdgpu_waves_per_eu(RSLOTS == 3 ? 5 : 4)))
k_loglik_reg(const BatchArgs a) {
    using RS = RegShape<KP>;
    constexpr int NI = RS::kItems;
    // dynamic LDS: with RSLOTS = 0 the stack [reg_depth][kItems][kThreads] of
    // double4; then the tile's tip codes [n][kPats]
    extern __shared__ double4 stack_lds[];
    const int lds_slots = RSLOTS > 0 ? 0 : a.reg_depth;
    uint8_t *tip_lds = reinterpret_cast<uint8_t *>(stack_lds + (size_t)lds_slots * NI * RS::kThreads);
    __shared__ double cat_l[RS::kWaves][RS::kGroupPats];
    __shared__ int cat_c[RS::kWaves][RS::kGroupPats];
    __shared__ double grp_sum[RS::kGroups];
    const int tile = blockIdx.x;
    const TreeDev td = a.trees[a.tile_tree[tile]];
    const AlnDev *aln = a.alns + td.aln;
    const int P = aln->P, n = aln->n_taxa, K = aln->K;
    // the wave index is wave-uniform, so the matrix addresses below are too
    // and their entries arrive by scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int k = wave % KP, grp = wave / KP;
    const int p0 = (tile - td.tile_begin) * RS::kPats;
    // tips of the tile into LDS (a pattern past the end reads as all states)
    for (int x = threadIdx.x; x < n * RS::kPats; x += RS::kThreads) {
        const int tx = x / RS::kPats, q = p0 + x % RS::kPats;
        tip_lds[x] = q < P ? ldg(aln->tips + (size_t)tx * P + q) : (uint8_t)15;
    }
    __syncthreads();
    // item j of this lane: pattern p0 + grp * kGroupPats + j * 64 + lane
    const uint8_t *tips = tip_lds + grp * RS::kGroupPats + lane;
    // this wave's category of every edge: P(r_k t_e) at pm + e * KP * 16
    const __attribute__((address_space(4))) double *pm =
        (const __attribute__((address_space(4))) double *)(a.pmat + td.pm_off) + k * 16;
    // the 4x4 identity, the matrix of an OP_REVAL's side a (1 x and 0 x are
    // exact, so I . x = x bit for bit): the plan keeps one after the last
    // tree's matrices
    const __attribute__((address_space(4))) double *ident =
        (const __attribute__((address_space(4))) double *)a.ident;
    const double thr = ldexp(1.0, -256), up = ldexp(1.0, 256);
    double acc[NI][4];
    int cnt[NI];
    double L[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        reg_copy(acc[j], (const double[4]){0.0, 0.0, 0.0, 0.0});
        cnt[j] = 0;
        L[j] = 0.0;
    }
    double4 *stk = stack_lds + threadIdx.x;  // item j, slot s at stk[(s * NI + j) * kThreads]
    double4 rstk[RSLOTS > 0 ? RSLOTS : 1][NI];  // slot s, item j (RSLOTS > 0)
    // One step for item j.  The compiler emits three side forms (see
    // compile_loglik_reg): two tips; the accumulator and a tip; a stack slot
    // and the accumulator.  Each form has its own straight-line code so that
    // the step's scalar matrix loads and LDS reads all issue before the one
    // wait for them.  (An OP_REVAL's side a takes the identity matrix: ea < 0.)
    auto step = [&](int j, const double xa[4], const double xb[4], const double *ma, const double *mb, bool upd) {
        double y[4], mx = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double ya = ma[i * 4] * xa[0] + ma[i * 4 + 1] * xa[1] + ma[i * 4 + 2] * xa[2] +
                              ma[i * 4 + 3] * xa[3];
            const double yb = mb[i * 4] * xb[0] + mb[i * 4 + 1] * xb[1] + mb[i * 4 + 2] * xb[2] +
                              mb[i * 4 + 3] * xb[3];
            y[i] = ya * yb;
            mx = fmax(mx, y[i]);
        }
        if (!upd) {
            L[j] = aln->freqs[0] * y[0] + aln->freqs[1] * y[1] + aln->freqs[2] * y[2] + aln->freqs[3] * y[3];
            return;
        }
        const bool scale = mx < thr && mx > 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] = scale ? y[i] * up : y[i];
        cnt[j] += scale ? 1 : 0;
    };
    // each op is loaded one step ahead, so its scalar load's round trip
    // overlaps the previous step
    Op nx = load_op(a.ops, td.op_first);
    for (int o = 0; o < td.n_first; ++o) {
        const Op op = nx;
        if (o + 1 < td.n_first) nx = load_op(a.ops, td.op_first + o + 1);
        if (op.code == OP_RPUSH) {
#pragma unroll
            for (int j = 0; j < NI; ++j)
            {
                const double4 x = make_double4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
                if constexpr (RSLOTS > 0) {
#pragma unroll
                    for (int q = 0; q < RSLOTS; ++q)
                        if (q == op.dst) rstk[q][j] = x;
                } else {
                    stk[((size_t)op.dst * NI + j) * RS::kThreads] = x;
                }
            }
            continue;
        }
        // both matrices are used on every path, so their loads issue together
        const bool upd = op.code == OP_RUPDATE;
        const auto Pa = op.ea >= 0 ? pm + (size_t)op.ea * KP * 16 : ident;
        const auto Pb = pm + (size_t)op.eb * KP * 16;
        double ma[16], mb[16];
        if (op.a >= 0) {  // two tips
            unsigned ca[NI], cb[NI];
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                ca[j] = tips[op.a * RS::kPats + j * 64];
                cb[j] = tips[op.b * RS::kPats + j * 64];
            }
#pragma unroll
            for (int x = 0; x < 16; ++x) {
                ma[x] = Pa[x];
                mb[x] = Pb[x];
            }
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                double xa[4], xb[4];
                tip_vec(ca[j], xa);
                tip_vec(cb[j], xb);
                step(j, xa, xb, ma, mb, upd);
            }
        } else if (op.a == REF_ACC) {  // the accumulator and a tip
            unsigned cb[NI];
#pragma unroll
            for (int j = 0; j < NI; ++j) cb[j] = tips[op.b * RS::kPats + j * 64];
#pragma unroll
            for (int x = 0; x < 16; ++x) {
                ma[x] = Pa[x];
                mb[x] = Pb[x];
            }
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                double xa[4], xb[4];
                reg_copy(xa, acc[j]);
                tip_vec(cb[j], xb);
                step(j, xa, xb, ma, mb, upd);
            }
        } else {  // a stack slot and the accumulator
            double4 v[NI];
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                const int slot = REF_STACK0 - op.a;
                if constexpr (RSLOTS > 0) {
                    v[j] = rstk[0][j];
#pragma unroll
                    for (int q = 1; q < RSLOTS; ++q)
                        if (q == slot) v[j] = rstk[q][j];
                } else {
                    v[j] = stk[((size_t)slot * NI + j) * RS::kThreads];
                }
            }
#pragma unroll
            for (int x = 0; x < 16; ++x) {
                ma[x] = Pa[x];
                mb[x] = Pb[x];
            }
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                double xa[4] = {v[j].x, v[j].y, v[j].z, v[j].w}, xb[4];
                reg_copy(xb, acc[j]);
                step(j, xa, xb, ma, mb, upd);
            }
        }
    }
    // the categories of each pattern meet in LDS
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        cat_l[wave][j * 64 + lane] = L[j];
        cat_c[wave][j * 64 + lane] = cnt[j];
    }
    __syncthreads();
    if (k == 0) {
        double term = 0.0;
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int q = j * 64 + lane, p = p0 + grp * RS::kGroupPats + q;
            if (p < P) {
                int cmin = cat_c[wave][q];
                for (int c = 1; c < K; ++c) cmin = min(cmin, cat_c[wave + c][q]);
                double sum = 0.0;
                for (int c = 0; c < K; ++c) sum += ldexp(cat_l[wave + c][q], -256 * (cat_c[wave + c][q] - cmin));
                term += ldg(aln->w + p) * (log(sum) - log((double)K) - (double)cmin * 256.0 * kLn2);
            }
        }
        term = wave_sum(term);
        if (lane == 0) grp_sum[grp] = term;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int g = 0; g < RS::kGroups; ++g) sum += grp_sum[g];
        a.part[(size_t)tile * a.part_cols * 3] = sum;
    }
}

// Log density of independent Exponential(rate) priors on the E lengths in
// LDS, sum_e (log rate - rate t_e); 0 for rate 0.  Every thread reads all
// lengths in the same order, so all hold the same value.
__device__ inline double log_prior(const double *tl, int E, double rate) {
    if (!(rate > 0.0)) return 0.0;
    const double lr = log(rate);
    double s = 0.0;
    for (int e = 0; e < E; ++e) s += lr - rate * tl[e];
    return s;
}

// Branch-length optimisation: one block owns one tree at a time, taken from
// a work counter in the order given (largest trees first), and runs the
// whole smoothing loop -- partial updates, per-edge Newton iterations with
// block reductions, pass-level convergence -- without leaving the kernel.
// Every wave exits once the counter passes the number of trees.
// With a.groups = G > 1 (a small batch: G blocks per tree, all resident at
// once), G blocks on one XCD own tree order[q] instead (see below), each
// over its own contiguous share of the patterns, and every reduction spans the G blocks
// (group_sum3); they take identical decisions, and block 0 of the group
// writes the tree's outputs.
// Each thread owns patterns tid + j*BS, j < ni, of its block's share
// (ni*BS >= the share of every tree).  TAB_LDS: the per-edge eigenbasis
// table lives in LDS after the transition matrices; otherwise in a
// per-block slice of a.tab.  GRP: compiled for a.groups > 1 (the
// one-block-per-tree instantiations carry none of the cross-block code).
template <typename T, int BS, int KP, bool TAB_LDS, bool GRP>
__global__ void __launch_bounds__(BS) k_optimize(const BatchArgs a, double *brlen, const OptParams opt, int ni,
                                                 int pm_lds_doubles, double *lnl_out, int32_t *passes_out,
                                                 int32_t *status_out) {
    extern __shared__ double lds[];
    __shared__ double red[2 * (BS / 64) * 3];
    __shared__ double wxs[(BS / 64) * kWx];
    __shared__ float wxfs[(BS / 64) * kWx];
    __shared__ ModelS model;
    __shared__ int q_sh;
    __shared__ GroupS gsh;
    __shared__ double pm_ex[4 * kMaxCats];
    const int tid = threadIdx.x;
    const int G = GRP ? a.groups : 1;
    // grouped: the hardware deals blocks to the XCDs in turn, so block i
    // runs on XCD i % kXcds; the G blocks of a tree are taken from one XCD
    // (trees x, x + kXcds, ... on XCD x), keeping their cross-block traffic
    // within one L2
    const unsigned xcd = blockIdx.x % (unsigned)kXcds, xslot = blockIdx.x / (unsigned)kXcds;
    const int g = GRP ? (int)(xslot % (unsigned)G) : 0;
    GroupS *gs = GRP ? &gsh : nullptr;
    double *wx = wxs + (tid >> 6) * kWx;
    float *wxf = wxfs + (tid >> 6) * kWx;
    // per block: the table [KP][BS*ni][4] of T, then the weights [BS*ni]
    const size_t tab_bytes = (size_t)BS * ni * KP * 4 * sizeof(T);
    char *tab_base = TAB_LDS ? reinterpret_cast<char *>(lds + pm_lds_doubles)
                             : reinterpret_cast<char *>(a.tab) + (size_t)blockIdx.x * (tab_bytes + (size_t)BS * ni * 8);
    T *tab = reinterpret_cast<T *>(tab_base);
    double *wrow = reinterpret_cast<double *>(tab_base + tab_bytes);
    for (int round = 0;; ++round) {
        int q;
        if (GRP) {
            q = (int)((xslot / (unsigned)G) * (unsigned)kXcds + xcd);
            if (round > 0 || q >= a.n_trees) break;
        } else {
            if (tid == 0) q_sh = atomicAdd(a.queue, 1);
            __syncthreads();
            q = q_sh;
            if (q >= a.n_trees) break;
        }
        const int b = a.order[q];
        const TreeDev td = a.trees[b];
        const AlnDev *aln = a.alns + td.aln;
        const int E = td.n_edges;
        // FP64 partials: the matrices, then the lengths, in LDS.  FP32
        // partials: the lengths, then (16-byte aligned) an FP32 copy of the
        // matrices for the loop's updates in LDS, while the FP64 matrices,
        // read only by the final FP64 evaluation, are written once before it
        // to this tree's slice of the global matrix buffer (so a 64-taxon
        // tree's table still fits in LDS beside the FP32 copy).
        constexpr bool kF32 = std::is_same<T, float>::value;
        constexpr bool kFuseUpd = GRP && TAB_LDS && FuseFirst<KP>::value && BS == 256;
        double *pm = kF32 ? a.pmat + td.pm_off : lds;
        double *tl = kF32 ? lds : lds + (size_t)E * KP * 16;
        float *pmf = reinterpret_cast<float *>(lds + (((size_t)E + 1) & ~(size_t)1));
        for (int e = tid; e < E; e += BS) tl[e] = fmin(fmax(brlen[td.edge_off + e], opt.t_min), opt.t_max);
        model_to_lds(aln, &model);
        if (GRP && tid == 0) {
            unsigned long long *base = a.gsync + (size_t)b * kGroupSyncWords;
            gsh.G = G;
            gsh.g = g;
            gsh.seq = 0;
            gsh.is_broken = 0;
            gsh.broken = base;
            gsh.slots = base + 1;
            gsh.wait = a.wait_cycles > 0 ? a.wait_cycles : kGroupWaitCycles;
        }
        __syncthreads();
        for (int x = tid; x < E * KP * 16; x += BS) {
            const int e = x / (KP * 16), r = x % (KP * 16);
            const double pe = pm_entry(&model, r >> 4, r & 15, tl[e]);
            if (kF32) pmf[x] = (float)pe;
            else pm[x] = pe;
        }
        __syncthreads();
        TreeView<T> v = make_view<T>(td, aln, a, &model, pm);
        v.pmf = pmf;
        // this block's share of the patterns
        const int chunk = (v.P + G - 1) / G;
        const int lo = min(v.P, g * chunk);
        v.np = min(v.P - lo, chunk);
        v.tips += lo;
        v.w += lo;
        v.clv += (size_t)lo * 4;
        v.cnt += lo;
        int parity = 0;
        double prev = -INFINITY, cur = -INFINITY;
        int passes = 0;
        bool converged = false;
        long long pc[PROF_FIELDS] = {0, 0, 0, 0, 0, 0, 0, 0};
        const long long t_start = clock64();
        for (;;) {
            const bool first = passes == 0;
            const int o0 = first ? td.op_first : td.op_steady;
            const int no = first ? td.n_first : td.n_steady;
            double max_rel = 0.0;
            double pass_gain = 0.0;  // the steps' predicted gains (FP32 partials)
            EdgePre pre;
            bool have_pre = false;
            for (int o = 0; o < no; ++o) {
                const Op op = load_op(a.ops, o0 + o);
                if (op.code == OP_UPDATE) {
                    const long long u0 = a.prof ? clock64() : 0;
                    bool fused = false;
                    // (256 threads per block only: with two waves per SIMD
                    // the extra registers would spill)
                    if constexpr (kFuseUpd) {
                        // an update making one side of the next edge step:
                        // build that edge's table from it directly
                        if (ni == 1 && o + 1 < no) {
                            const Op nx = load_op(a.ops, o0 + o + 1);
                            if (nx.code == OP_NEWTON && (nx.a == op.dst || nx.b == op.dst)) {
                                pre = update_and_table<T, BS, KP, kF32 ? kPmLds32 : kPmLds>(
                                    v, op, nx.a == op.dst ? nx.b : nx.a, tl[nx.dst], tab, wrow, wx, wxf);
                                have_pre = fused = true;
                            }
                        }
                    }
                    if (!fused) do_update<T, BS, KP, kF32 ? kPmLds32 : kPmLds>(v, op, 0, ni);
                    if (a.prof) {
                        pc[PROF_UPDATES] += 1;
                        pc[PROF_CYC_UPDATE] += clock64() - u0;
                    }
                    continue;
                }
                const int e = op.dst;
                const double t0 = tl[e];
                if (op.code == OP_EVAL) {
                    const Sums3 r = eval_edge<T, BS, KP>(v, op.a, op.b, 0, ni, t0, red, wx, parity, gs);
                    parity = r.parity;
                    cur = r.l0;
                    continue;
                }
                // the pass's lnL comes from its last edge step (op.ea = 1)
                const EdgeResult r =
                    newton_edge<T, BS, KP, !kFuseUpd>(v, op.a, op.b, t0, op.ea != 0, opt, tab, wrow, ni, red, wx, wxf,
                                                      parity, gs, passes >= 1 ? kRelax : 1.0, have_pre ? &pre : nullptr);
                have_pre = false;
                parity = r.parity;
                if (op.ea) cur = r.lnl;
                pc[PROF_EDGE_STEPS] += 1;
                pc[PROF_NEWTON_ITERS] += r.iters;
                pc[PROF_CYC_TABLE] += r.cyc_table;
                pc[PROF_CYC_ITERS] += r.cyc_iters;
                // A step counts against convergence when it moves the length
                // by more than tol_t relative, unless it starts or ends at a
                // bound and its gain by the quadratic model at the start is
                // negligible (below tol_lnl / E; the bound is then optimal to
                // within that gain).  With FP32 partials a length whose
                // optimum lies at t_min otherwise never settles: the
                // derivative there is at the noise level, and Newton keeps
                // moving the length on and off the bound by amounts tiny in
                // absolute terms but large relative to the 1e-6 floor of the
                // relative change, for no gain.
                //
                // With FP32 partials the same holds away from the bounds: a
                // pass's lnL is resolved only to about 1e-4 (rounding of the
                // stored partials; measured on the 27-taxon trees), above
                // tol_lnl, and a short length keeps moving by about tol_t
                // relative on derivative noise for gains near 1e-9.  There a
                // step counts against convergence only when its gain is not
                // negligible, and the pass's lnL increase is taken as the sum
                // over its steps of the quadratic model's value (which sees
                // no rounding noise) instead of the difference of two noisy
                // lnL values.  A step not concave at its start still counts
                // its model value there (a flat long length settles with a
                // second derivative at the noise level, of either sign), and
                // always counts against convergence by its length change.
                const bool at_bound = t0 <= opt.t_min || t0 >= opt.t_max || r.t <= opt.t_min || r.t >= opt.t_max;
                if (!((kF32 || at_bound) && r.gain < opt.tol_lnl / E))
                    max_rel = fmax(max_rel, fabs(r.t - t0) / fmax(t0, 1e-6));
                pass_gain += r.rise;
                if (r.t != t0) {
                    if (tid == 0) tl[e] = r.t;
                    if constexpr (KP * 16 <= 64) {
                        // the edge's matrices are one wave's work: its first
                        // 4 KP lanes take the exponentials, then every lane
                        // one entry (LDS operations of a wave complete in order)
                        if (tid < 4 * KP) pm_ex[tid] = exp(model.lam[tid & 3] * model.rate[tid >> 2] * r.t);
                        __builtin_amdgcn_wave_barrier();
                        if (tid < KP * 16) {
                            const double pe = pm_entry_ex(&model, pm_ex, tid >> 4, tid & 15);
                            if (kF32) pmf[(size_t)e * KP * 16 + tid] = (float)pe;
                            else pm[(size_t)e * KP * 16 + tid] = pe;
                        }
                    } else {
                        if (tid < KP * 16) {
                            const double pe = pm_entry(&model, tid >> 4, tid & 15, r.t);
                            if (kF32) pmf[(size_t)e * KP * 16 + tid] = (float)pe;
                            else pm[(size_t)e * KP * 16 + tid] = pe;
                        }
                    }
                    __syncthreads();
                }
            }
            ++passes;
            cur += log_prior(tl, E, opt.prior_rate);
            const double rise = kF32 ? pass_gain : cur - prev;
            if (td.n_steady == 0 || (rise < opt.tol_lnl && max_rel < opt.tol_t)) {
                converged = true;
                break;
            }
            if (passes >= opt.max_passes) break;
            prev = cur;
        }
        if (kF32 && td.n_final > 0) {
            // The FP64 matrices at the final lengths, for the FP64 pass below
            // (the loop's updates read only the FP32 copy in LDS, so no FP64
            // matrix is stored during the loop).  Every block of a tree
            // computes the same values from the same lengths.
            for (int x = tid; x < E * KP * 16; x += BS) {
                const int e = x / (KP * 16), r = x % (KP * 16);
                pm[x] = pm_entry(&model, r >> 4, r & 15, tl[e]);
            }
            if (!GRP) __syncthreads();
        }
        if (GRP && kF32 && td.n_final > 0) {
            // The FP64 pass below reuses the tree's buffer in another layout,
            // so a block writes bytes that another block wrote as FP32
            // partials.  The XCDs' L2 caches are not coherent: a dirty FP32
            // line left in another XCD's L2 could later be written back over
            // the new FP64 values.  Every wave writes back its L2 (release at
            // device scope) and the group meets once before any FP64 write.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            double z0 = 0.0, z1 = 0.0, z2 = 0.0;
            group_sum3<BS>(z0, z1, z2, red, parity, gs);
        }
        if (std::is_same<T, float>::value && td.n_final > 0) {
            // Report lnL from FP64 partials at the final lengths: one post-order
            // pass over the same buffer (dense slots; the FP32 partials are no
            // longer needed, and each thread touches only its own patterns).
            TreeView<double> vd;
            vd.m = v.m;
            vd.pm = v.pm;
            vd.tips = v.tips;
            vd.w = v.w;
            // the same share in the FP64 layout: every block of the tree has
            // finished reading FP32 partials (their reads preceded the
            // arrivals at the last reduction)
            vd.clv = reinterpret_cast<double *>(reinterpret_cast<T *>(a.clv) + td.clv_off) + (size_t)lo * 4;
            vd.cnt = v.cnt;
            vd.P = v.P;
            vd.np = v.np;
            vd.K = v.K;
            for (int o = 0; o < td.n_final; ++o) {
                const Op op = load_op(a.ops, td.op_final + o);
                if (op.code == OP_UPDATE) {
                    do_update<double, BS, KP, kPmGlobal>(vd, op, 0, ni);
                } else {
                    const Sums3 r =
                        eval_edge<double, BS, KP>(vd, op.a, op.b, 0, ni, tl[op.dst], red, wx, parity, gs);
                    parity = r.parity;
                    cur = r.l0 + log_prior(tl, E, opt.prior_rate);
                }
            }
        }
        if (g == 0) {
            for (int e = tid; e < E; e += BS) brlen[td.edge_off + e] = tl[e];
            if (tid == 0 && a.prof) {
                pc[PROF_PASSES] = passes;
                pc[PROF_CYC_TOTAL] = clock64() - t_start;
                for (int f = 0; f < PROF_FIELDS; ++f) a.prof[(size_t)b * PROF_FIELDS + f] = pc[f];
            }
            if (tid == 0) {
                // a timed-out wait anywhere in the group: status 2, lnL NaN
                const bool broken = GRP && load_agent(gsh.broken) != 0ull;
                lnl_out[b] = broken ? NAN : cur;
                if (passes_out) passes_out[b] = passes;
                if (status_out) status_out[b] = broken ? 2 : (converged ? 0 : 1);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- dispatch

template <typename T, int BS, int KP, bool L, bool GRP>
hipError_t launch_opt_t(int grid, const BatchArgs &a, double *brlen, const OptParams &opt, int ni, int pm_doubles,
                        double *lnl, int32_t *passes, int32_t *status, size_t lds, hipStream_t s) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_optimize<T, BS, KP, L, GRP>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_optimize<T, BS, KP, L, GRP>), dim3(grid), dim3(BS), lds, s, a, brlen, opt, ni,
                       pm_doubles, lnl, passes, status);
    return hipGetLastError();
}

template <typename T, int BS, int KP, bool L, bool GRP>
int occ_opt_t(size_t lds) {
    int n = 0;
    if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void *>(k_optimize<T, BS, KP, L, GRP>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_optimize<T, BS, KP, L, GRP>, BS, lds) != hipSuccess)
        return 0;
    return n;
}

template <typename T, int BS, int KP, bool L, bool GRP>
size_t spill_opt_t() {
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(k_optimize<T, BS, KP, L, GRP>)) != hipSuccess)
        return ~size_t(0);
    return at.localSizeBytes;
}

// Runtime (precision, block, padded categories, table placement, grouped)
// to the matching instantiation of FN.
#define PT_OPT_CALL_T(FN, T, BSZ, ...)                                                        \
    do {                                                                                      \
        if (grouped)                                                                          \
            return tab_lds ? FN<T, BSZ, KP, true, true>(__VA_ARGS__) : FN<T, BSZ, KP, false, true>(__VA_ARGS__); \
        return tab_lds ? FN<T, BSZ, KP, true, false>(__VA_ARGS__) : FN<T, BSZ, KP, false, false>(__VA_ARGS__); \
    } while (0)
#define PT_OPT_CALL(FN, ...)                                                                  \
    do {                                                                                      \
        if (block == 256 && precision == PT_FP32) PT_OPT_CALL_T(FN, float, 256, __VA_ARGS__);  \
        if (block == 256) PT_OPT_CALL_T(FN, double, 256, __VA_ARGS__);                        \
        if (block == 512 && precision == PT_FP32) PT_OPT_CALL_T(FN, float, 512, __VA_ARGS__);  \
        if (block == 512) PT_OPT_CALL_T(FN, double, 512, __VA_ARGS__);                        \
    } while (0)

#define PT_KP_SWITCH(...)                                   \
    switch (kp) {                                           \
    case 1: { constexpr int KP = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int KP = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int KP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int KP = 8; __VA_ARGS__; } break;   \
    default: break;                                         \
    }

template <typename T, int BS, int KP>
hipError_t launch_tiles_t(const BatchArgs &a, const double *brlen, size_t lds, hipStream_t s) {
    if (std::is_same<T, float>::value) {
        hipLaunchKernelGGL((k_tiles32<BS, KP>), dim3(a.n_tiles), dim3(BS), 0, s, a, brlen);
        return hipGetLastError();
    }
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_tiles64<BS, KP>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tiles64<BS, KP>), dim3(a.n_tiles), dim3(BS), lds, s, a, brlen);
    return hipGetLastError();
}

}  // namespace

bool optimize_shape_supported(int block, int items) {
    return (block == 256 || block == 512) && items >= 1 && items <= 64;
}

int optimize_blocks_per_cu(int precision, int block, int kp, bool tab_lds, bool grouped, size_t lds) {
    PT_KP_SWITCH(PT_OPT_CALL(occ_opt_t, lds));
    return 0;
}

size_t optimize_spill_bytes(int precision, int block, int kp, bool tab_lds, bool grouped) {
    PT_KP_SWITCH(PT_OPT_CALL(spill_opt_t));
    return ~size_t(0);
}

hipError_t launch_optimize(int precision, int block, int kp, int items, bool tab_lds, int pm_doubles, int grid,
                           const BatchArgs &a, double *brlen, const OptParams &opt, double *lnl, int32_t *passes,
                           int32_t *status, size_t lds, hipStream_t s) {
    const bool grouped = a.groups > 1;
    PT_KP_SWITCH(PT_OPT_CALL(launch_opt_t, grid, a, brlen, opt, items, pm_doubles, lnl, passes, status, lds, s));
    return hipErrorInvalidValue;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_pmat(const BatchArgs &a, const double *brlen, hipStream_t s) {
    if (a.n_edges <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pmat, dim3((unsigned)a.n_trees), dim3(256), 0, s, a, brlen);
    return hipGetLastError();
}

bool tile_patterns_supported(int pats) { return pats == 64 || pats == 128 || pats == 256; }

hipError_t launch_tiles(int precision, int kp, int tile_pats, const BatchArgs &a, const double *brlen, size_t lds,
                        hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
#define PT_TILES_BS(BSZ)                                                                             \
    PT_KP_SWITCH(return precision == PT_FP32 ? launch_tiles_t<float, BSZ, KP>(a, brlen, lds, s) \
                                             : launch_tiles_t<double, BSZ, KP>(a, brlen, lds, s))
    if (tile_pats == 64) PT_TILES_BS(64);
    if (tile_pats == 128) PT_TILES_BS(128);
    if (tile_pats == 256) PT_TILES_BS(256);
#undef PT_TILES_BS
    return hipErrorInvalidValue;
}

int loglik_reg_tile_patterns(int kp) {
    PT_KP_SWITCH(return RegShape<KP>::kPats);
    return 0;
}

size_t loglik_reg_lds(int kp, int n, int depth) {
    // programs of at most kRegStackRegs slots keep their stack in registers
    const int lds_slots = depth <= kRegStackRegs ? 0 : depth;
    PT_KP_SWITCH(return (size_t)lds_slots * RegShape<KP>::kItems * RegShape<KP>::kThreads * sizeof(double4) +
                        (size_t)n * RegShape<KP>::kPats);
    return 0;
}

hipError_t launch_loglik_reg(int kp, const BatchArgs &a, size_t lds_bytes, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
#define PT_REG_LAUNCH(RSL)                                                                                  \
    do {                                                                                                    \
        if (lds_bytes > 48 * 1024) {                                                                        \
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_loglik_reg<KP, RSL>),       \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes); \
            if (e != hipSuccess) return e;                                                                  \
        }                                                                                                   \
        hipLaunchKernelGGL((k_loglik_reg<KP, RSL>), dim3(a.n_tiles), dim3(RegShape<KP>::kThreads), lds_bytes, s, a); \
        return hipGetLastError();                                                                           \
    } while (0)
    PT_KP_SWITCH({
        static_assert(kRegStackRegs == 4, "register stacks of three and four slots");
        if (a.reg_depth <= 3) PT_REG_LAUNCH(3);
        if (a.reg_depth <= 4) PT_REG_LAUNCH(4);
        PT_REG_LAUNCH(0);
    });
#undef PT_REG_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(bool grad, const BatchArgs &a, double *lnl, double *gout, double *hout,
                         hipStream_t s) {
    const int64_t n = grad ? a.n_edges : a.n_trees;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, grad, lnl, gout, hout);
    return hipGetLastError();
}

}  // namespace pt
