// pt_device.hpp -- descriptors shared by the host runtime and the kernels.
//
// Device memory layout of one batch ("plan"):
//   partials  T[slot][Kp][pattern][4]  Kp = the largest category count of the
//             batch padded to a power of two; a tree owns 3 (n-2)
//             directional slots (one per internal node and neighbour: the
//             partial of that node's side of the edge to the neighbour).
//   scalers   uint16[slot][pattern]  power-of-two scaling events.
//   pmat      double[edge][Kp][4][4] transition matrices P(r_k t_e).
// A thread owns a pattern and loops over its categories; for a fixed
// category, consecutive patterns are consecutive 16- or 32-byte rows.
#pragma once
#include <stdint.h>

namespace pt {

constexpr int kMaxCats = 8;

// Program opcodes.  A side reference `ref` is a slot index (>= 0) or a tip
// -(leaf + 1).
enum : int32_t {
    OP_UPDATE = 1,  // dst = (P(ea) . side a) * (P(eb) . side b), then scaling
    OP_NEWTON = 2,  // optimise the length of edge e between sides a and b
    OP_EVAL = 3,    // lnL (and derivatives) across edge e; out = output column
    // Register programs (the lnL with every partial kept in registers):
    OP_RUPDATE = 4,  // acc = (P(ea) . side a) * (P(eb) . side b), then scaling
    OP_RPUSH = 5,    // stack slot dst = acc
    OP_REVAL = 6,    // lnL across edge eb: pi . (side a * (P(eb) . side b)); ea = -1
};

// Side references of register programs: a leaf's tip (>= 0), the
// accumulator, or stack slot REF_STACK0 - ref.
constexpr int32_t REF_ACC = -1;
constexpr int32_t REF_STACK0 = -2;
constexpr int kRegStack = 8;      // stack slots of the register kernel
constexpr int kRegStackRegs = 4;  // programs of at most this many slots keep the stack in registers

struct Op {
    int32_t code;
    int32_t dst;    // UPDATE: destination slot;  NEWTON/EVAL: edge
    int32_t a;      // side a
    int32_t ea;     // UPDATE: edge of side a;  EVAL: output column;
                    // NEWTON: 1 when this step reports the tree's lnL
    int32_t b;      // side b
    int32_t eb;     // UPDATE: edge of side b
    int32_t pad0, pad1;
};

struct AlnDev {
    const uint8_t *tips;   // [n_taxa][P]
    const double *w;       // [P]
    int32_t n_taxa, P, K, Kp;
    double freqs[4];
    double U[16];          // P(t) = U diag(exp(lam t)) Uinv
    double Uinv[16];
    double W[16];          // W_im = pi_i U_im = Uinv_mi = sqrt(pi_i) V_im
    double lam[4];
    double rate[kMaxCats]; // category rates (0 for padded categories)
};

struct TreeDev {
    int32_t aln;
    int32_t n_edges;
    int32_t n_slots;
    int32_t n_tiles;       // tile kernels: pattern tiles of this tree
    int32_t op_first, n_first;    // loglik/grad program, or first optimisation pass
    int32_t op_steady, n_steady;  // later optimisation passes
    int64_t clv_off;       // element offset of slot 0 in the partials buffer
    int64_t cnt_off;       // element offset of slot 0 in the scaler buffer
    int64_t edge_off;      // first edge in the flat per-edge arrays
    int64_t pm_off;        // first double of this tree's transition matrices
    int32_t tile_begin;    // first global tile index of this tree
    int32_t op_final;      // FP32 optimisation: FP64 lnL program run at the end
    int32_t n_final;       //   (slots renumbered densely, see tree.cpp)
    int32_t pad;
};

struct OptParams {
    double t_min, t_max, tol_lnl, tol_t, tol_newton;
    int32_t max_passes, max_newton;
    double prior_rate;  // 0: maximum likelihood; > 0: exponential prior (MAP)
};

}  // namespace pt
