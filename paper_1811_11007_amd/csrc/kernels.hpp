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
    int32_t *queue;             // optimisation work counter
    int32_t n_trees;
    int32_t n_tiles;
    int64_t n_edges;            // total flat edges
    int32_t part_cols;
};

// Items per tile of the tile kernels (threads per block x items per thread).
constexpr int kTileBlock = 256;
constexpr int kTileItems = 2;

bool optimize_shape_supported(int block, int items);
int optimize_blocks_per_cu(int precision, int block, int items, size_t lds_bytes);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_pmat(const BatchArgs &a, const double *brlen, hipStream_t s);
hipError_t launch_tiles(int precision, bool grad, const BatchArgs &a, const double *brlen,
                        size_t lds_bytes, hipStream_t s);
hipError_t launch_reduce(bool grad, const BatchArgs &a, double *lnl, double *grad_out,
                         double *hess_out, hipStream_t s);
hipError_t launch_optimize(int precision, int block, int items, int grid, const BatchArgs &a,
                           double *brlen, const OptParams &opt, double *lnl, int32_t *passes,
                           int32_t *status, size_t lds_bytes, hipStream_t s);

}  // namespace pt
