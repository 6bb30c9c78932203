// kernels.hpp -- launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "pt_device.hpp"

namespace pt {

// Pointers and sizes a batch hands to its kernels.
struct BatchArgs {
    const TreeDev *trees;
    const AlnDev *alns;
    const Op *ops;
    const int32_t *tile_tree;   // tile kernels: owning tree of each tile
    const int32_t *edge_tree;   // owning tree of each flat edge
    const int32_t *order;       // optimisation: tree order (largest first)
    void *clv;                  // float or double partials
    uint16_t *cnt;
    double *pmat;               // [sum_b E_b * Kp_b * 16]
    double *part;               // tile partial sums [tile][part_cols][3]
    void *tab;                  // optimisation: per-block eigenbasis tables when not in LDS
    int32_t *queue;             // optimisation work counter
    int32_t n_trees;
    int32_t n_tiles;
    int64_t n_edges;            // total flat edges
    int32_t part_cols;
    int32_t kp;                 // padded category count of every layout in the batch
    long long *prof;            // optimisation: per-tree phase counters [n_trees][8], or null
    int32_t groups;             // optimisation: blocks per tree (1: one block per tree, work queue)
    unsigned long long *gsync;  // optimisation with groups > 1: per-tree cross-block words, zeroed
    int32_t reg_depth;          // register-resident lnL: stack slots of the deepest tree
    const double *ident;        // register-resident lnL: the 4x4 identity (16 doubles)
    long long wait_cycles;      // optimisation with groups > 1: shader clocks before a
                                // cross-block wait gives up (0: kGroupWaitCycles)
};

// Optimisation with several blocks per tree: at most kGroupBlocksMax blocks,
// and kGroupSyncWords words of cross-block state per tree.
constexpr int kGroupBlocksMax = 8;
constexpr int kGroupSyncWords = 64;
// XCDs of the device, to which consecutive blocks are dealt in turn; a
// grouped launch has kXcds * groups * ceil(trees / kXcds) blocks.
constexpr int kXcds = 8;

// Per-tree optimisation counters (when BatchArgs::prof is set).  Where an
// edge step's last update and its table build run fused, the table's cycles
// count as the update's.
enum : int { PROF_PASSES, PROF_EDGE_STEPS, PROF_NEWTON_ITERS, PROF_UPDATES, PROF_CYC_UPDATE,
             PROF_CYC_TABLE, PROF_CYC_ITERS, PROF_CYC_TOTAL, PROF_FIELDS };

// Patterns per tile of the tile kernels (threads per block x patterns per thread).
constexpr int kTileBlock = 256;
constexpr int kTileItems = 1;

// Optimisation kernel shapes: threads per block 256 or 512, patterns per
// thread 1..64 (a runtime loop bound); kp = padded categories 1, 2, 4, 8;
// grouped: the instantiation for several blocks per tree.
bool optimize_shape_supported(int block, int items);
int optimize_blocks_per_cu(int precision, int block, int kp, bool tab_lds, bool grouped, size_t lds_bytes);
// Private (spill) bytes per thread of an optimisation kernel instantiation.
size_t optimize_spill_bytes(int precision, int block, int kp, bool tab_lds, bool grouped);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_pmat(const BatchArgs &a, const double *brlen, hipStream_t s);
// lds_bytes: the largest tree's transition matrices (used with FP64 partials).
// tile_pats: patterns per tile (= threads per block, one pattern each): 64,
// 128 or 256 (kTileBlock, the default).
bool tile_patterns_supported(int pats);
hipError_t launch_tiles(int precision, int kp, int tile_pats, const BatchArgs &a, const double *brlen,
                        size_t lds_bytes, hipStream_t s);
// Register-resident lnL (k_loglik_reg): patterns per tile for a padded
// category count, its LDS for n taxa and a stack of `depth` slots, and the
// launch (one block per tile; a.tile_tree, a.part, a.n_tiles and
// a.reg_depth describe the register tiles; lds_bytes from loglik_reg_lds).
int loglik_reg_tile_patterns(int kp);
size_t loglik_reg_lds(int kp, int n, int depth);
hipError_t launch_loglik_reg(int kp, const BatchArgs &a, size_t lds_bytes, hipStream_t s);
// The fixed device workspace of pt_batch_loglik_noalloc (noalloc.hip):
// kNoAllocBytes on each device; its address on `device`, looked up once per
// device (with that device current) and kept.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
hipError_t noalloc_workspace(int device, void **out);
hipError_t launch_reduce(bool grad, const BatchArgs &a, double *lnl, double *grad_out,
                         double *hess_out, hipStream_t s);
// With a.groups > 1, grid = trees x groups and a.gsync zeroed beforehand.
hipError_t launch_optimize(int precision, int block, int kp, int items, bool tab_lds, int pm_doubles, int grid,
                           const BatchArgs &a, double *brlen, const OptParams &opt, double *lnl,
                           int32_t *passes, int32_t *status, size_t lds_bytes, hipStream_t s);

}  // namespace pt
