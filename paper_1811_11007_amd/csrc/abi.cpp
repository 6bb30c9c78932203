// abi.cpp -- the C ABI: contexts, alignments, plans and batch entry points.
//
// A plan is one compiled batch: every tree validated, its programs emitted
// (tree.cpp), descriptors and programs uploaded, partial buffers allocated.
// The host-pointer batch calls build a plan (split to respect the arena cap),
// run it once and free it; the device-pointer plan calls run it repeatedly,
// optionally through captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "mlp.hpp"
#include "pt_internal.hpp"

using pt::AlnDev;
using pt::Op;
using pt::TreeDev;

namespace {

thread_local std::string g_err;

pt_status fail(pt_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define PT_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(e_ == hipErrorOutOfMemory ? PT_ENOMEM : PT_EDEVICE,                     \
                        std::string(#call) + ": " + hipGetErrorString(e_));                    \
    } while (0)

constexpr int kMaxOptPatterns = 512 * 64;

int64_t arena_cap() {
    const char *s = std::getenv("PT_ARENA_CAP_BYTES");
    if (!s || !*s) return -1;
    char *end = nullptr;
    long long v = std::strtoll(s, &end, 10);
    return (end && *end == 0 && v > 0) ? (int64_t)v : -1;
}

}  // namespace

// Device blocks of destroyed plans, kept for later plans (size -> block).
// Shared by a context and its plans, so a plan destroyed after its context
// still has somewhere to return its memory; the last owner frees the blocks.
struct DevicePool {
    int device = 0;
    std::multimap<size_t, void *> blocks;
    size_t bytes = 0;
    ~DevicePool() {
        if (blocks.empty()) return;
        (void)hipSetDevice(device);
        for (auto &b : blocks) (void)hipFree(b.second);
    }
};

struct pt_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_per_block = 65536;
    hipStream_t stream = nullptr;
    // tuned (threads per block, blocks per tree) of the optimisation kernel,
    // per (precision, padded categories, largest pattern count)
    std::map<std::tuple<int, int, int>, std::pair<int, int>> tuned;
    // tuned patterns per tile of the stored pass and gradient, per
    // (precision, padded categories, largest pattern count, largest edge count)
    std::map<std::tuple<int, int, int, int>, int> tuned_tiles;
    // device memory of destroyed plans: a search creates a plan of the same
    // size for every batch, and a fresh hipMalloc / hipFree of tens of GB
    // each time cost far more than the optimisation itself
    std::shared_ptr<DevicePool> pool = std::make_shared<DevicePool>();
    // shader clocks before a cross-block wait of the optimisation kernel
    // gives up (pt_ctx_set_group_wait; 0: the kernel's default)
    long long group_wait = 0;
    // this device's no-allocation workspace (pt_batch_loglik_noalloc)
    void *noalloc = nullptr;
    std::string noalloc_err;
};

struct pt_aln {
    pt_ctx *ctx = nullptr;
    int n_taxa = 0, P = 0;
    AlnDev desc{};
    uint8_t *d_tips = nullptr;
    double *d_w = nullptr;
};

struct pt_plan {
    pt_ctx *ctx = nullptr;
    int precision = 0, kinds = 0;
    int n_trees = 0;
    int64_t n_edges = 0;
    int max_P = 0, max_E = 0, n_tiles = 0, kp = 1;
    int tile_pats = pt::kTileBlock;      // patterns per tile of the stored pass and gradient
    size_t tile_cap = 0, part_cap = 0;   // allocated entries of d_tile_tree and d_part
    std::vector<int> tree_E;
    AlnDev *d_alns = nullptr;
    Op *d_ops = nullptr;
    TreeDev *d_trees_ll = nullptr, *d_trees_gr = nullptr, *d_trees_opt = nullptr;
    int32_t *d_tile_tree = nullptr, *d_edge_tree = nullptr, *d_order = nullptr, *d_queue = nullptr;
    // the register-resident lnL (k_loglik_reg): its descriptors, tiles and
    // tile sums; reg_ok when every tree of the plan fits it
    bool reg_ok = false, stored_ok = true;
    int ll_stored = 0;  // pt_plan_set_loglik_path: 1 = the stored post-order pass
    TreeDev *d_trees_reg = nullptr;
    int32_t *d_tile_tree_reg = nullptr;
    double *d_part_reg = nullptr;
    int n_tiles_reg = 0, reg_depth = 0;
    size_t lds_reg = 0;
    const double *ident = nullptr;  // the 4x4 identity, after the matrices
    void *d_clv = nullptr;
    uint16_t *d_cnt = nullptr;
    double *d_pmat = nullptr, *d_part = nullptr, *d_scratch = nullptr;
    size_t lds_tiles = 0, lds_opt = 0;
    int opt_block = 0, opt_items = 0, opt_grid = 0, pm_doubles = 0;
    int opt_groups = 1;                      // blocks per tree of the optimisation kernel
    unsigned long long *d_gsync = nullptr;   // their cross-block state, per tree
    bool opt_tab_lds = true;
    void *d_tab = nullptr;
    size_t tab_bytes = 0;
    long long *d_prof = nullptr;
    int64_t device_bytes = 0;
    bool graphs = false;
    std::map<std::vector<uint64_t>, hipGraphExec_t> execs;
    std::vector<std::pair<void *, size_t>> allocs;  // device blocks and their sizes
    std::shared_ptr<DevicePool> pool;                // where they go when the plan is destroyed
    // host copies for traffic accounting
    std::vector<Op> ops_h;
    std::vector<TreeDev> tll_h, tgr_h, top_h, treg_h;
    std::vector<AlnDev> alns_h;       // per tree, as on the device
    std::vector<AlnDev> alns_base_h;  // per tree, the alignment's own model
    double *d_alpha_lnl = nullptr;    // per tree, for the Gamma-shape search
};

namespace {

// Bytes the context keeps in its pool of released device blocks
// (PT_POOL_CAP_BYTES, default 64 GiB); beyond it the largest are freed.
size_t pool_cap() {
    const char *s = std::getenv("PT_POOL_CAP_BYTES");
    if (s && *s) {
        char *end = nullptr;
        long long v = std::strtoll(s, &end, 10);
        if (end && *end == 0 && v >= 0) return (size_t)v;
    }
    return (size_t)64 << 30;
}

void pool_trim(DevicePool *pool, size_t cap) {
    while (pool->bytes > cap && !pool->blocks.empty()) {
        auto it = std::prev(pool->blocks.end());
        (void)hipFree(it->second);
        pool->bytes -= it->first;
        pool->blocks.erase(it);
    }
}

// A device block for a plan: the smallest pooled block of 1x to 2x the size,
// else a new one (after emptying the pool if the device is full).  Plans
// initialise everything they read, so a reused block needs no clearing.
template <typename P>
pt_status dev_alloc(pt_plan *pl, P **out, size_t bytes) {
    DevicePool *pool = pl->pool.get();
    bytes = std::max<size_t>(bytes, 16);
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    size_t got = bytes;
    auto it = pool->blocks.lower_bound(bytes);
    if (it != pool->blocks.end() && it->first <= 2 * bytes) {
        p = it->second;
        got = it->first;
        pool->bytes -= got;
        pool->blocks.erase(it);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess && !pool->blocks.empty()) {
            (void)hipGetLastError();
            pool_trim(pool, 0);
            e = hipMalloc(&p, bytes);
        }
        if (e != hipSuccess) return fail(PT_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    pl->allocs.push_back({p, got});
    pl->device_bytes += (int64_t)got;
    *out = reinterpret_cast<P *>(p);
    return PT_OK;
}

// Destroys a plan; its device blocks go to the pool once the device has
// finished any work that may still use them (the pool outlives the plan's
// context if need be).
void free_plan(pt_plan *pl) {
    if (!pl) return;
    for (auto &kv : pl->execs) (void)hipGraphExecDestroy(kv.second);
    if (!pl->allocs.empty()) {
        DevicePool *pool = pl->pool.get();
        (void)hipSetDevice(pool->device);
        (void)hipDeviceSynchronize();
        for (const auto &a : pl->allocs) {
            pool->blocks.emplace(a.second, a.first);
            pool->bytes += a.second;
        }
        pool_trim(pool, pool_cap());
    }
    delete pl;
}

pt_status check_opt(const pt_opt &o) {
    if (!(o.t_min > 0.0) || !(o.t_max > o.t_min) || !std::isfinite(o.t_max))
        return fail(PT_EINVAL, "pt_opt: need 0 < t_min < t_max < inf");
    if (!(o.tol_lnl >= 0.0) || !(o.tol_t >= 0.0) || !(o.tol_newton >= 0.0))
        return fail(PT_EINVAL, "pt_opt: tolerances must be >= 0");
    if (o.max_passes < 1 || o.max_newton < 1) return fail(PT_EINVAL, "pt_opt: max_passes and max_newton must be >= 1");
    if (!(o.prior_rate >= 0.0) || !std::isfinite(o.prior_rate))
        return fail(PT_EINVAL, "pt_opt: prior_rate must be finite and >= 0");
    return PT_OK;
}

pt::OptParams to_params(const pt_opt &o) {
    pt::OptParams p;
    p.t_min = o.t_min;
    p.t_max = o.t_max;
    p.tol_lnl = o.tol_lnl;
    p.tol_t = o.tol_t;
    p.tol_newton = o.tol_newton;
    p.max_passes = o.max_passes;
    p.max_newton = o.max_newton;
    p.prior_rate = o.prior_rate;
    return p;
}

// Validates the batch description and returns per-tree taxon counts.
pt_status check_trees(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                      std::vector<int> &n_taxa) {
    if (!ctx) return fail(PT_EINVAL, "ctx is NULL");
    if (!trees) return fail(PT_EINVAL, "trees is NULL");
    if (trees->n_trees < 0) return fail(PT_EINVAL, "n_trees < 0");
    if (trees->n_trees > 0 && (!trees->aln_index || !trees->edge_offset || !trees->edges))
        return fail(PT_EINVAL, "trees: NULL array");
    if (n_alns < 1 || !alns) return fail(PT_EINVAL, "need at least one alignment");
    for (int i = 0; i < n_alns; ++i) {
        if (!alns[i]) return fail(PT_EINVAL, "alns[" + std::to_string(i) + "] is NULL");
        if (alns[i]->ctx != ctx) return fail(PT_EINVAL, "alignment belongs to another context");
    }
    if (trees->n_trees > 0 && trees->edge_offset[0] != 0) return fail(PT_EINVAL, "edge_offset[0] must be 0");
    n_taxa.resize(trees->n_trees);
    for (int b = 0; b < trees->n_trees; ++b) {
        int ai = trees->aln_index[b];
        if (ai < 0 || ai >= n_alns) return fail(PT_EINVAL, "tree " + std::to_string(b) + ": aln_index out of range");
        int n = alns[ai]->n_taxa;
        int64_t want = n == 2 ? 1 : 2 * n - 3;
        if (trees->edge_offset[b + 1] - trees->edge_offset[b] != want)
            return fail(PT_EINVAL, "tree " + std::to_string(b) + ": edge count must be 2n-3 = " + std::to_string(want));
        n_taxa[b] = n;
    }
    return PT_OK;
}

pt_status check_lengths(const double *brlen, int64_t n) {
    if (n > 0 && !brlen) return fail(PT_EINVAL, "brlen is NULL");
    for (int64_t i = 0; i < n; ++i)
        if (!(brlen[i] >= 0.0) || !std::isfinite(brlen[i]))
            return fail(PT_EINVAL, "branch length " + std::to_string(i) + " is negative or not finite");
    return PT_OK;
}

size_t store_bytes(int precision) { return precision == PT_FP32 ? 4 : 8; }

// Device bytes a one-tree plan of this shape needs (for the arena cap).
int64_t tree_bytes(int n, const AlnDev &a, int precision, int kinds) {
    const int E = n == 2 ? 1 : 2 * n - 3, slots = n >= 3 ? 3 * (n - 2) : 0;
    const int64_t items = (int64_t)a.P * a.Kp;
    int64_t b = (int64_t)slots * items * 4 * store_bytes(precision) + (int64_t)slots * a.P * 2;
    b += (int64_t)E * a.Kp * 16 * 8 + 64 * E + 256;
    if (kinds & (PT_PLAN_LOGLIK | PT_PLAN_GRAD)) {
        int64_t tiles = (a.P + 63) / 64;  // the smallest tile (pt_plan_set_tile_patterns)
        b += tiles * (int64_t)E * 3 * 8 + tiles * 4;
    }
    return b;
}

// Static LDS of the optimisation kernel at 512 threads (reduction buffers,
// per-wave exponential tables, model, counter), rounded up.
constexpr size_t kOptStaticLds = 12288;

// Doubles of the optimisation kernel's per-tree LDS before its table: with
// FP64 partials the FP64 matrices then the lengths; with FP32 partials the
// lengths then (16-byte aligned) an FP32 copy of the matrices.
size_t opt_pm_doubles(int precision, int E, int kp) {
    return precision == PT_FP32 ? (((size_t)E + 1) & ~(size_t)1) + (size_t)E * kp * 8
                                : (size_t)E * (kp * 16 + 1);
}

// LDS of the stored post-order pass for one tree: FP64 partials read the
// matrices from an LDS copy, FP32 partials by scalar loads (none).
size_t stored_lds(int precision, int E, int kp) {
    return precision == PT_FP64 ? (size_t)E * kp * 16 * 8 : 0;
}

// Sets the optimisation launch shape for `block` threads per block: patterns
// per thread, where the eigenbasis table lives (LDS when it fits, else a
// per-block global buffer), dynamic LDS, grid.  Refuses shapes whose kernel
// needs private (spill) memory.
// Optimisation launch shape: `block` threads per block, `groups` blocks per
// tree.  Several blocks per tree need every block of the grid resident at
// once (they wait for each other), so groups > 1 is refused unless
// trees x groups blocks fit on the device at the kernel's occupancy.
pt_status configure_shape(pt_plan *pl, int block, int groups = 1) {
    if (groups < 1 || groups > pt::kGroupBlocksMax)
        return fail(PT_EUNSUPPORTED, "blocks per tree must be in 1.." + std::to_string(pt::kGroupBlocksMax));
    const bool grouped = groups > 1;
    const int share = (pl->max_P + groups - 1) / groups;
    const int ni = (share + block - 1) / block;
    if (!pt::optimize_shape_supported(block, ni))
        return fail(PT_EUNSUPPORTED, "patterns x padded categories too large for the optimisation kernel");
    const size_t esz = store_bytes(pl->precision);
    const size_t tab_lds = (size_t)block * ni * pl->kp * 4 * esz + (size_t)block * ni * 8;
    const size_t pm_bytes = (size_t)pl->pm_doubles * 8;
    const bool lds_ok = pm_bytes + tab_lds + kOptStaticLds <= pl->ctx->lds_per_block;
    if (pt::optimize_spill_bytes(pl->precision, block, pl->kp, lds_ok, grouped) != 0)
        return fail(PT_EUNSUPPORTED, "optimisation kernel shape needs register spills");
    const size_t lds = pm_bytes + (lds_ok ? tab_lds : 0);
    int per_cu = pt::optimize_blocks_per_cu(pl->precision, block, pl->kp, lds_ok, grouped, lds);
    if (per_cu < 1) return fail(PT_EUNSUPPORTED, "optimisation kernel does not fit on a compute unit");
    const long resident = (long)per_cu * std::max(1, pl->ctx->n_cu);
    // grouped: whole trees per XCD (the kernel's block-to-tree mapping), so
    // the grid rounds the trees up to a multiple of the XCD count and each
    // XCD must hold its share
    const long grouped_grid = (long)pt::kXcds * groups * ((pl->n_trees + pt::kXcds - 1) / pt::kXcds);
    if (grouped && grouped_grid > resident)
        return fail(PT_EUNSUPPORTED, "trees x blocks per tree exceed the blocks resident at once");
    const int grid = grouped ? (int)grouped_grid : (int)std::max(1L, std::min<long>(pl->n_trees, resident));
    if (grouped && !pl->d_gsync) {
        pt_status st = dev_alloc(pl, &pl->d_gsync, sizeof(unsigned long long) * pt::kGroupSyncWords *
                                                       (size_t)std::max(1, pl->n_trees));
        if (st) return st;
    }
    if (!lds_ok) {
        size_t need = (size_t)grid * tab_lds;
        if (need > pl->tab_bytes) {
            char *p = nullptr;
            pt_status st = dev_alloc(pl, &p, need);
            if (st) return st;
            pl->d_tab = p;
            pl->tab_bytes = need;
        }
    }
    pl->opt_block = block;
    pl->opt_items = ni;
    pl->opt_groups = groups;
    pl->opt_tab_lds = lds_ok;
    pl->lds_opt = lds;
    pl->opt_grid = grid;
    return PT_OK;
}

// Re-tiles the stored pass and the gradient at `pats` patterns per tile:
// each tree's tile count, the tiles of the longest programs first (as at
// build time), the tile-to-tree map and the per-tile sums, reallocated when
// they grow.  Captured graphs are dropped.
pt_status set_tile_pats(pt_plan *pl, int pats) {
    if (!pt::tile_patterns_supported(pats)) return fail(PT_EINVAL, "patterns per tile must be 64, 128 or 256");
    if (!(pl->kinds & (PT_PLAN_LOGLIK | PT_PLAN_GRAD)) || pl->n_trees == 0) {
        pl->tile_pats = pats;
        return PT_OK;
    }
    const int B = pl->n_trees;
    std::vector<int> order(B);
    for (int b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pl->tree_E[x] > pl->tree_E[y]; });
    std::vector<int32_t> tile_tree;
    std::vector<TreeDev> tll = pl->tll_h, tgr = pl->tgr_h;
    int tiles = 0;
    for (int b : order) {
        const int nt = (pl->alns_h[b].P + pats - 1) / pats;
        tll[b].n_tiles = tgr[b].n_tiles = nt;
        tll[b].tile_begin = tgr[b].tile_begin = tiles;
        for (int x = 0; x < nt; ++x) tile_tree.push_back(b);
        tiles += nt;
    }
    const size_t part = 3 * (size_t)tiles * std::max(1, pl->max_E);
    PT_HIP(hipSetDevice(pl->ctx->device));
    PT_HIP(hipDeviceSynchronize());  // no launch of this plan may still read the old tiles
    if ((size_t)tiles > pl->tile_cap) {
        int32_t *p = nullptr;
        pt_status st = dev_alloc(pl, &p, sizeof(int32_t) * tiles);
        if (st) return st;
        pl->d_tile_tree = p;
        pl->tile_cap = (size_t)tiles;
    }
    if (part > pl->part_cap) {
        double *p = nullptr;
        pt_status st = dev_alloc(pl, &p, sizeof(double) * part);
        if (st) return st;
        pl->d_part = p;
        pl->part_cap = part;
    }
    PT_HIP(hipMemcpy(pl->d_tile_tree, tile_tree.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice));
    if (pl->kinds & PT_PLAN_LOGLIK)
        PT_HIP(hipMemcpy(pl->d_trees_ll, tll.data(), sizeof(TreeDev) * B, hipMemcpyHostToDevice));
    if (pl->kinds & PT_PLAN_GRAD)
        PT_HIP(hipMemcpy(pl->d_trees_gr, tgr.data(), sizeof(TreeDev) * B, hipMemcpyHostToDevice));
    pl->tll_h = tll;
    pl->tgr_h = tgr;
    pl->n_tiles = tiles;
    pl->tile_pats = pats;
    for (auto &kv : pl->execs) (void)hipGraphExecDestroy(kv.second);
    pl->execs.clear();
    return PT_OK;
}

// Padded category count of a plan: that of the widest alignment its trees use.
int kp_of_plan(pt_aln *const *alns, const pt_trees *trees) {
    int kp = 1;
    for (int b = 0; b < trees->n_trees; ++b) kp = std::max(kp, alns[trees->aln_index[b]]->desc.Kp);
    return kp;
}

pt_status plan_build(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                     const uint8_t *mask, int precision, int kinds, pt_plan **out) {
    if (precision != PT_FP32 && precision != PT_FP64) return fail(PT_EINVAL, "precision must be PT_FP64 or PT_FP32");
    if (kinds <= 0 || kinds > 7) return fail(PT_EINVAL, "kinds must be a non-empty OR of PT_PLAN_*");
    std::vector<int> ntx;
    pt_status st = check_trees(ctx, alns, n_alns, trees, ntx);
    if (st) return st;
    const int B = trees->n_trees;
    const int64_t NE = B ? trees->edge_offset[B] : 0;
    if (mask)
        for (int64_t i = 0; i < NE; ++i)
            if (mask[i] > 1) return fail(PT_EINVAL, "opt_mask entries must be 0 or 1");

    std::unique_ptr<pt_plan, void (*)(pt_plan *)> pl(new pt_plan, free_plan);
    pl->ctx = ctx;
    pl->pool = ctx->pool;
    pl->precision = precision;
    pl->kinds = kinds;
    pl->n_trees = B;
    pl->n_edges = NE;

    std::vector<Op> ops;
    std::vector<TreeDev> tll(B), tgr(B), top(B);
    std::vector<int32_t> tile_tree, edge_tree(NE);
    std::vector<double> cost(B);
    int64_t clv_off = 0, cnt_off = 0, pm_off = 0;
    int tiles = 0;
    const int64_t tile_pats = (int64_t)pt::kTileBlock * pt::kTileItems;
    const int kp = kp_of_plan(alns, trees);
    pl->kp = kp;
    // Trees compile independently, on up to 16 host threads (a search
    // builds a plan of about a thousand trees for every batch); offsets and
    // the concatenated program follow in tree order.
    struct Compiled {
        pt_status st = PT_OK;
        std::string err;
        int E = 0, n_slots = 0, reg_depth = 0;
        bool any = true, stored_ok = true;
        std::vector<Op> ll, gr, p1, p2, p3, rg;
    };
    const bool want_reg = (kinds & PT_PLAN_LOGLIK) || ((kinds & PT_PLAN_GRAD) && precision == PT_FP32);
    std::vector<Compiled> cp(B);
    auto compile_tree = [&](int b) {
        Compiled &c = cp[b];
        const AlnDev &ad = alns[trees->aln_index[b]]->desc;
        pt::Tree t;
        const int32_t *ed = trees->edges + 2 * trees->edge_offset[b];
        std::string err;
        c.st = pt::build_tree(ntx[b], ed, t, err);
        if (c.st) { c.err = "tree " + std::to_string(b) + ": " + err; return; }
        c.E = t.n_edges;
        c.n_slots = t.n_slots();
        // transition matrices the kernels keep in LDS, per tree
        if ((kinds & PT_PLAN_OPTIMIZE) && opt_pm_doubles(precision, c.E, kp) * 8 + kOptStaticLds > ctx->lds_per_block) {
            c.st = PT_EUNSUPPORTED;
            c.err = "tree " + std::to_string(b) + ": (2n-3) x padded categories transition matrices exceed the "
                    "LDS of a block for branch optimisation (" + std::to_string(ctx->lds_per_block) + " bytes)";
            return;
        }
        c.stored_ok = stored_lds(precision, c.E, kp) <= ctx->lds_per_block;
        if ((kinds & PT_PLAN_GRAD) && !c.stored_ok) {
            c.st = PT_EUNSUPPORTED;
            c.err = "tree " + std::to_string(b) + ": (2n-3) x padded categories FP64 transition matrices exceed the "
                    "LDS of a block (" + std::to_string(ctx->lds_per_block) + " bytes)";
            return;
        }
        if ((kinds & PT_PLAN_OPTIMIZE) && ad.P > kMaxOptPatterns) {
            c.st = PT_EUNSUPPORTED;
            c.err = "tree " + std::to_string(b) + ": more than 32768 patterns for branch optimisation";
            return;
        }
        if (want_reg) c.reg_depth = pt::compile_loglik_reg(t, c.rg);
        if (kinds & PT_PLAN_LOGLIK) pt::compile_loglik(t, c.ll);
        if (kinds & PT_PLAN_GRAD) pt::compile_grad(t, c.gr);
        if (kinds & PT_PLAN_OPTIMIZE) {
            const uint8_t *m = mask ? mask + trees->edge_offset[b] : nullptr;
            c.any = !m;
            for (int e = 0; m && e < c.E; ++e) c.any |= m[e] != 0;
            if (c.any) pt::compile_optimize(t, m, c.p1, c.p2);
            else pt::compile_loglik(t, c.p1);
            if (precision == PT_FP32) pt::compile_loglik_dense(t, c.p3);
        }
    };
    {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        const int nt = std::max(1, std::min({hw, 16, (B + 31) / 32}));
        if (nt == 1) {
            for (int b = 0; b < B; ++b) compile_tree(b);
        } else {
            std::vector<std::thread> pool;
            for (int w = 0; w < nt; ++w)
                pool.emplace_back([&, w]() {
                    for (int b = w; b < B; b += nt) compile_tree(b);
                });
            for (auto &th : pool) th.join();
        }
    }
    for (int b = 0; b < B; ++b)
        if (cp[b].st) return fail(cp[b].st, cp[b].err);
    // the register-resident lnL needs every tree within its stack and the
    // tile's tip codes within the LDS of a block
    const int reg_pats = pt::loglik_reg_tile_patterns(kp);
    pl->reg_ok = want_reg && B > 0;
    int reg_depth = 0, reg_n = 0;
    for (int b = 0; b < B; ++b) {
        reg_depth = std::max(reg_depth, cp[b].reg_depth);
        reg_n = std::max(reg_n, ntx[b]);
    }
    if (reg_depth > pt::kRegStack || pt::loglik_reg_lds(kp, reg_n, reg_depth) > ctx->lds_per_block)
        pl->reg_ok = false;
    pl->reg_depth = reg_depth;
    pl->stored_ok = true;
    for (int b = 0; b < B; ++b) pl->stored_ok = pl->stored_ok && cp[b].stored_ok;
    if ((kinds & PT_PLAN_LOGLIK) && !pl->reg_ok && !pl->stored_ok)
        return fail(PT_EUNSUPPORTED, "a tree exceeds the LDS of a block on both likelihood passes");
    if (!pl->reg_ok) pl->ll_stored = 1;
    std::vector<TreeDev> treg(B);
    for (int b = 0; b < B; ++b) {
        Compiled &c = cp[b];
        const AlnDev &ad = alns[trees->aln_index[b]]->desc;
        const int E = c.E;
        pl->max_P = std::max(pl->max_P, ad.P);
        pl->max_E = std::max(pl->max_E, E);
        pl->tree_E.push_back(E);
        TreeDev base{};
        base.aln = b;  // every tree has a descriptor of its own (per-tree Gamma shape)
        base.n_edges = E;
        base.n_slots = c.n_slots;
        base.clv_off = clv_off;
        base.cnt_off = cnt_off;
        base.edge_off = trees->edge_offset[b];
        base.pm_off = pm_off;
        base.n_tiles = (int)((ad.P + tile_pats - 1) / tile_pats);
        base.tile_begin = 0;  // assigned below, longest programs first
        clv_off += (int64_t)c.n_slots * kp * ad.P * 4;
        cnt_off += (int64_t)c.n_slots * ad.P;
        pm_off += (int64_t)E * kp * 16;
        for (int64_t i = 0; i < E; ++i) edge_tree[base.edge_off + i] = b;
        tll[b] = tgr[b] = top[b] = base;
        auto append = [&](const std::vector<Op> &v, int32_t &first, int32_t &count) {
            first = (int32_t)ops.size();
            count = (int32_t)v.size();
            ops.insert(ops.end(), v.begin(), v.end());
        };
        if (pl->reg_ok) {
            treg[b] = base;
            treg[b].n_tiles = (ad.P + reg_pats - 1) / reg_pats;
            append(c.rg, treg[b].op_first, treg[b].n_first);
        }
        if (kinds & PT_PLAN_LOGLIK) append(c.ll, tll[b].op_first, tll[b].n_first);
        if (kinds & PT_PLAN_GRAD) append(c.gr, tgr[b].op_first, tgr[b].n_first);
        if (kinds & PT_PLAN_OPTIMIZE) {
            append(c.p1, top[b].op_first, top[b].n_first);
            append(c.p2, top[b].op_steady, top[b].n_steady);
            if (precision == PT_FP32) append(c.p3, top[b].op_final, top[b].n_final);
            cost[b] = (double)ad.P * ad.K * (double)(c.p2.size() + 1);
        }
        std::vector<Op>().swap(c.ll);
        std::vector<Op>().swap(c.gr);
        std::vector<Op>().swap(c.p1);
        std::vector<Op>().swap(c.p2);
        std::vector<Op>().swap(c.p3);
        std::vector<Op>().swap(c.rg);
    }
    std::vector<int32_t> tile_tree_reg;
    if (pl->reg_ok) {
        // register tiles of the longest programs first, as below
        std::vector<int> order(B);
        for (int b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pl->tree_E[x] > pl->tree_E[y]; });
        for (int b : order) {
            treg[b].tile_begin = (int32_t)tile_tree_reg.size();
            for (int x = 0; x < treg[b].n_tiles; ++x) tile_tree_reg.push_back(b);
        }
        pl->lds_reg = pt::loglik_reg_lds(kp, reg_n, reg_depth);
        pl->n_tiles_reg = (int)tile_tree_reg.size();
    }
    if (kinds & (PT_PLAN_LOGLIK | PT_PLAN_GRAD)) {
        // Tiles of the trees with the longest programs first: the hardware
        // dispatches blocks in index order, so long tiles start early and the
        // launch does not end on a tail of them.
        std::vector<int> order(B);
        for (int b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pl->tree_E[x] > pl->tree_E[y]; });
        for (int b : order) {
            tll[b].tile_begin = tgr[b].tile_begin = top[b].tile_begin = tiles;
            for (int x = 0; x < tll[b].n_tiles; ++x) tile_tree.push_back(b);
            tiles += tll[b].n_tiles;
        }
    }
    pl->n_tiles = tiles;
    pl->ops_h = ops;
    pl->tll_h = tll;
    pl->tgr_h = tgr;
    pl->top_h = top;
    pl->treg_h = treg;
    for (int b = 0; b < B; ++b) pl->alns_h.push_back(alns[trees->aln_index[b]]->desc);
    pl->alns_base_h = pl->alns_h;

    // arena cap
    int64_t need = clv_off * (int64_t)store_bytes(precision) + cnt_off * 2 + (pm_off + 16) * 8 +
                   (int64_t)ops.size() * sizeof(Op) + (int64_t)tiles * std::max(1, pl->max_E) * 24 +
                   (int64_t)NE * 16 + (int64_t)B * 4 * sizeof(TreeDev) + (int64_t)pl->n_tiles_reg * 28;
    int64_t cap = arena_cap();
    if (cap > 0 && need > cap)
        return fail(PT_ENOMEM, "batch needs " + std::to_string(need) + " device bytes, over PT_ARENA_CAP_BYTES");

    int dev_prev = 0;
    PT_HIP(hipGetDevice(&dev_prev));
    PT_HIP(hipSetDevice(ctx->device));
    // descriptors, one per tree
    if ((st = dev_alloc(pl.get(), &pl->d_alns, sizeof(AlnDev) * std::max(1, B)))) return st;
    if (B) PT_HIP(hipMemcpy(pl->d_alns, pl->alns_h.data(), sizeof(AlnDev) * B, hipMemcpyHostToDevice));
    if ((st = dev_alloc(pl.get(), &pl->d_ops, sizeof(Op) * ops.size()))) return st;
    if (!ops.empty()) PT_HIP(hipMemcpy(pl->d_ops, ops.data(), sizeof(Op) * ops.size(), hipMemcpyHostToDevice));
    auto up_trees = [&](std::vector<TreeDev> &v, TreeDev **d) -> pt_status {
        pt_status s2 = dev_alloc(pl.get(), d, sizeof(TreeDev) * std::max(1, B));
        if (s2) return s2;
        if (B) PT_HIP(hipMemcpy(*d, v.data(), sizeof(TreeDev) * B, hipMemcpyHostToDevice));
        return PT_OK;
    };
    if (kinds & PT_PLAN_LOGLIK) if ((st = up_trees(tll, &pl->d_trees_ll))) return st;
    if (kinds & PT_PLAN_GRAD) if ((st = up_trees(tgr, &pl->d_trees_gr))) return st;
    if (kinds & PT_PLAN_OPTIMIZE) if ((st = up_trees(top, &pl->d_trees_opt))) return st;
    if (pl->reg_ok) {
        if ((st = up_trees(treg, &pl->d_trees_reg))) return st;
        if ((st = dev_alloc(pl.get(), &pl->d_tile_tree_reg, sizeof(int32_t) * pl->n_tiles_reg))) return st;
        PT_HIP(hipMemcpy(pl->d_tile_tree_reg, tile_tree_reg.data(), sizeof(int32_t) * pl->n_tiles_reg,
                         hipMemcpyHostToDevice));
        if ((st = dev_alloc(pl.get(), &pl->d_part_reg, sizeof(double) * 3 * (size_t)pl->n_tiles_reg))) return st;
    }
    if ((st = dev_alloc(pl.get(), &pl->d_edge_tree, sizeof(int32_t) * std::max<int64_t>(1, NE)))) return st;
    if (NE) PT_HIP(hipMemcpy(pl->d_edge_tree, edge_tree.data(), sizeof(int32_t) * NE, hipMemcpyHostToDevice));
    if (tiles) {
        if ((st = dev_alloc(pl.get(), &pl->d_tile_tree, sizeof(int32_t) * tiles))) return st;
        PT_HIP(hipMemcpy(pl->d_tile_tree, tile_tree.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice));
        if ((st = dev_alloc(pl.get(), &pl->d_part, sizeof(double) * 3 * (size_t)tiles * std::max(1, pl->max_E)))) return st;
        pl->tile_cap = (size_t)tiles;
        pl->part_cap = 3 * (size_t)tiles * std::max(1, pl->max_E);
    }
    if (kinds & PT_PLAN_OPTIMIZE) {
        std::vector<int32_t> order(B);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        if ((st = dev_alloc(pl.get(), &pl->d_order, sizeof(int32_t) * std::max(1, B)))) return st;
        if (B) PT_HIP(hipMemcpy(pl->d_order, order.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice));
        if ((st = dev_alloc(pl.get(), &pl->d_queue, sizeof(int32_t) * 4))) return st;
        if ((st = dev_alloc(pl.get(), &pl->d_scratch, sizeof(double) * std::max<int64_t>(1, NE)))) return st;
    }
    if ((st = dev_alloc(pl.get(), &pl->d_clv, (size_t)clv_off * store_bytes(precision)))) return st;
    if ((st = dev_alloc(pl.get(), &pl->d_cnt, (size_t)cnt_off * 2))) return st;
    // the trees' matrices, then the 4x4 identity the register-resident pass
    // applies to one side at the root edge
    if ((st = dev_alloc(pl.get(), &pl->d_pmat, (size_t)(pm_off + 16) * 8))) return st;
    {
        const double ident[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
        PT_HIP(hipMemcpy(pl->d_pmat + pm_off, ident, sizeof(ident), hipMemcpyHostToDevice));
    }
    pl->ident = pl->d_pmat + pm_off;
    PT_HIP(hipSetDevice(dev_prev));

    pl->lds_tiles = 0;
    for (int b = 0; b < B; ++b) {
        const AlnDev &a2 = alns[trees->aln_index[b]]->desc;
        (void)a2;
        pl->lds_tiles = std::max(pl->lds_tiles, (size_t)pl->tree_E[b] * kp * 16 * 8);
        pl->pm_doubles = std::max(pl->pm_doubles, (int)opt_pm_doubles(precision, pl->tree_E[b], kp));
    }
    pl->pm_doubles = (pl->pm_doubles + 3) / 4 * 4;  // 32-byte aligned table rows after it
    if (kinds & PT_PLAN_OPTIMIZE) {
        auto it = ctx->tuned.find(std::make_tuple(precision, pl->kp, pl->max_P));
        st = PT_EUNSUPPORTED;
        if (it != ctx->tuned.end()) {
            st = configure_shape(pl.get(), it->second.first, it->second.second);
            if (st && it->second.second > 1) st = configure_shape(pl.get(), it->second.first, 1);
        }
        // default: a batch that leaves at least half the compute units idle
        // splits each tree over up to 4 blocks of 256 threads (the fastest
        // shape measured on such batches), if they fit at once; otherwise
        // the widest block that needs no spills
        const int n_cu = std::max(1, ctx->n_cu);
        if (st && B > 0 && 2 * B <= n_cu) st = configure_shape(pl.get(), 256, std::min(4, n_cu / B));
        for (int bs : {512, 256})
            if (st) st = configure_shape(pl.get(), bs);
        if (st) return st;
    }
    if (kinds & (PT_PLAN_LOGLIK | PT_PLAN_GRAD)) {
        auto it = ctx->tuned_tiles.find(std::make_tuple(precision, pl->kp, pl->max_P, pl->max_E));
        if (it != ctx->tuned_tiles.end() && it->second != pl->tile_pats)
            if ((st = set_tile_pats(pl.get(), it->second))) return st;
    }
    *out = pl.release();
    return PT_OK;
}

pt::BatchArgs batch_args(const pt_plan *pl, const TreeDev *trees, int part_cols) {
    pt::BatchArgs a{};
    a.trees = trees;
    a.alns = pl->d_alns;
    a.ops = pl->d_ops;
    a.tile_tree = pl->d_tile_tree;
    a.edge_tree = pl->d_edge_tree;
    a.order = pl->d_order;
    a.clv = pl->d_clv;
    a.cnt = pl->d_cnt;
    a.pmat = pl->d_pmat;
    a.part = pl->d_part;
    a.queue = pl->d_queue;
    a.n_trees = pl->n_trees;
    a.n_tiles = pl->n_tiles;
    a.n_edges = pl->n_edges;
    a.part_cols = part_cols;
    a.kp = pl->kp;
    return a;
}

// Enqueue the kernels of one plan call.
pt_status enqueue(pt_plan *pl, int kind, const double *brlen_c, double *brlen, const pt::OptParams *op,
                  double *lnl, int32_t *passes, int32_t *status, double *grad, double *hess, hipStream_t s) {
    if (pl->n_trees == 0) return PT_OK;
    hipError_t e = hipSuccess;
    if (kind == PT_PLAN_LOGLIK || kind == PT_PLAN_GRAD) {
        const bool g = kind == PT_PLAN_GRAD;
        const bool reg_ll = !g && pl->reg_ok && !pl->ll_stored;
        pt::BatchArgs a = batch_args(pl, g ? pl->d_trees_gr : pl->d_trees_ll, g ? std::max(1, pl->max_E) : 1);
        if ((e = pt::launch_pmat(a, brlen_c, s)) != hipSuccess) goto bad;
        if (!reg_ll) {
            if ((e = pt::launch_tiles(pl->precision, pl->kp, pl->tile_pats, a, brlen_c, pl->lds_tiles, s)) != hipSuccess)
                goto bad;
            if ((e = pt::launch_reduce(g, a, lnl, grad, hess, s)) != hipSuccess) goto bad;
        }
        // lnL with every partial in FP64 registers: the likelihood call
        // itself, and the lnL a gradient call with FP32 partials reports
        // (FP32 storage puts ~1e-4 of rounding noise into lnL at a few
        // thousand sites; the gradient keeps its stored partials)
        if (reg_ll || (g && pl->reg_ok && pl->precision == PT_FP32)) {
            pt::BatchArgs r = batch_args(pl, pl->d_trees_reg, 1);
            r.tile_tree = pl->d_tile_tree_reg;
            r.part = pl->d_part_reg;
            r.n_tiles = pl->n_tiles_reg;
            r.reg_depth = pl->reg_depth;
            r.ident = pl->ident;
            if ((e = pt::launch_loglik_reg(pl->kp, r, pl->lds_reg, s)) != hipSuccess) goto bad;
            if (lnl && (e = pt::launch_reduce(false, r, lnl, nullptr, nullptr, s)) != hipSuccess) goto bad;
        }
        return PT_OK;
    }
    {
        pt::BatchArgs a = batch_args(pl, pl->d_trees_opt, 1);
        a.tab = pl->d_tab;
        a.prof = pl->d_prof;
        a.groups = pl->opt_groups;
        a.gsync = pl->d_gsync;
        a.wait_cycles = pl->ctx->group_wait;
        if ((e = pt::launch_fill_i32(pl->d_queue, 0, 1, s)) != hipSuccess) goto bad;
        if (pl->opt_groups > 1 &&
            (e = pt::launch_fill_i32(reinterpret_cast<int32_t *>(pl->d_gsync), 0,
                                     (int64_t)pl->n_trees * pt::kGroupSyncWords * 2, s)) != hipSuccess)
            goto bad;
        if ((e = pt::launch_optimize(pl->precision, pl->opt_block, pl->kp, pl->opt_items, pl->opt_tab_lds, pl->pm_doubles,
                                     pl->opt_grid, a, brlen, *op, lnl, passes, status, pl->lds_opt, s)) != hipSuccess)
            goto bad;
        return PT_OK;
    }
bad:
    return fail(PT_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Run directly, or through a graph captured once per argument set.
pt_status run(pt_plan *pl, int kind, const double *brlen_c, double *brlen, const pt::OptParams *op, double *lnl,
              int32_t *passes, int32_t *status, double *grad, double *hess, hipStream_t s) {
    PT_HIP(hipSetDevice(pl->ctx->device));
    if (!pl->graphs || s == nullptr) return enqueue(pl, kind, brlen_c, brlen, op, lnl, passes, status, grad, hess, s);
    std::vector<uint64_t> key = {(uint64_t)kind, (uint64_t)(uintptr_t)brlen_c, (uint64_t)(uintptr_t)brlen,
                                 (uint64_t)(uintptr_t)lnl, (uint64_t)(uintptr_t)passes, (uint64_t)(uintptr_t)status,
                                 (uint64_t)(uintptr_t)grad, (uint64_t)(uintptr_t)hess, (uint64_t)(uintptr_t)s};
    if (op) {
        const uint64_t *w = reinterpret_cast<const uint64_t *>(op);
        key.insert(key.end(), w, w + sizeof(pt::OptParams) / 8);
    }
    auto it = pl->execs.find(key);
    if (it == pl->execs.end()) {
        hipGraph_t g = nullptr;
        PT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        pt_status st = enqueue(pl, kind, brlen_c, brlen, op, lnl, passes, status, grad, hess, s);
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (st) { if (g) (void)hipGraphDestroy(g); return st; }
        if (e2 != hipSuccess) return fail(PT_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
        hipGraphExec_t ex = nullptr;
        hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(PT_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
        it = pl->execs.emplace(key, ex).first;
    }
    PT_HIP(hipGraphLaunch(it->second, s));
    return PT_OK;
}

// Groups the trees of a host-pointer batch into chunks: one group per padded
// category count (every layout of a plan uses its widest alignment's), each
// group split so that no chunk's plan exceeds the arena cap.
pt_status make_chunks(pt_aln *const *alns, const pt_trees *trees, const std::vector<int> &ntx, int precision,
                      int kinds, std::vector<std::vector<int>> &out) {
    const int64_t cap = arena_cap();
    const int B = trees->n_trees;
    for (int kp : {1, 2, 4, 8}) {
        std::vector<int> cur;
        int64_t used = 0;
        for (int b = 0; b < B; ++b) {
            const AlnDev &ad = alns[trees->aln_index[b]]->desc;
            if (ad.Kp != kp) continue;
            if (cap > 0) {
                int64_t need = tree_bytes(ntx[b], ad, precision, kinds) + 4096;
                if (need > cap) return fail(PT_ENOMEM, "tree " + std::to_string(b) + " alone exceeds PT_ARENA_CAP_BYTES");
                if (used + need > cap && !cur.empty()) {
                    out.push_back(cur);
                    cur.clear();
                    used = 0;
                }
                used += need;
            }
            cur.push_back(b);
        }
        if (!cur.empty()) out.push_back(cur);
    }
    return PT_OK;
}

// Host-pointer batch driver shared by the three batch calls: validate, split
// into chunks, run each chunk as its own plan, scatter results; outputs are
// written only after every chunk has succeeded.
pt_status host_batch(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees, double *brlen_io,
                     const double *brlen_in, const uint8_t *mask, const pt_opt *opt, int precision, int kind,
                     double *lnl_out, int32_t *passes_out, int32_t *status_out, double *grad_out, double *hess_out) {
    std::vector<int> ntx;
    pt_status st = check_trees(ctx, alns, n_alns, trees, ntx);
    if (st) return st;
    if (precision != PT_FP32 && precision != PT_FP64) return fail(PT_EINVAL, "precision must be PT_FP64 or PT_FP32");
    const int B = trees->n_trees;
    const int64_t NE = B ? trees->edge_offset[B] : 0;
    const double *lens = brlen_io ? brlen_io : brlen_in;
    if ((st = check_lengths(lens, NE))) return st;
    if (B > 0 && !lnl_out) return fail(PT_EINVAL, "lnl_out is NULL");
    if (kind == PT_PLAN_GRAD && NE > 0 && !grad_out) return fail(PT_EINVAL, "grad_out is NULL");
    if (mask)
        for (int64_t i = 0; i < NE; ++i)
            if (mask[i] > 1) return fail(PT_EINVAL, "opt_mask entries must be 0 or 1");
    pt_opt o;
    if (kind == PT_PLAN_OPTIMIZE) {
        if (opt) o = *opt; else pt_opt_default(precision, &o);
        if ((st = check_opt(o))) return st;
    }
    std::vector<std::vector<int>> chunks;
    if ((st = make_chunks(alns, trees, ntx, precision, kind, chunks))) return st;

    std::vector<double> lnl(B), lens_out(lens, lens + NE), grad(kind == PT_PLAN_GRAD ? NE : 0),
        hess(kind == PT_PLAN_GRAD && hess_out ? NE : 0);
    std::vector<int32_t> passes(B), status(B);
    for (const std::vector<int> &ch : chunks) {
        const int nb = (int)ch.size();
        // contiguous copies of the chunk's trees
        std::vector<int32_t> ai(nb), ed;
        std::vector<int64_t> off(nb + 1, 0);
        std::vector<double> cl;
        std::vector<uint8_t> cm;
        for (int i = 0; i < nb; ++i) {
            const int b = ch[i];
            const int64_t e0 = trees->edge_offset[b], e1 = trees->edge_offset[b + 1];
            ai[i] = trees->aln_index[b];
            off[i + 1] = off[i] + (e1 - e0);
            ed.insert(ed.end(), trees->edges + 2 * e0, trees->edges + 2 * e1);
            cl.insert(cl.end(), lens + e0, lens + e1);
            if (mask) cm.insert(cm.end(), mask + e0, mask + e1);
        }
        const int64_t ne = off[nb];
        pt_trees sub;
        sub.n_trees = nb;
        sub.aln_index = ai.data();
        sub.edge_offset = off.data();
        sub.edges = ed.data();
        pt_plan *raw = nullptr;
        st = plan_build(ctx, alns, n_alns, &sub, mask ? cm.data() : nullptr, precision, kind, &raw);
        if (st) return st;
        std::unique_ptr<pt_plan, void (*)(pt_plan *)> pl(raw, free_plan);
        PT_HIP(hipSetDevice(ctx->device));
        double *d_len = nullptr, *d_lnl = nullptr, *d_g = nullptr, *d_h = nullptr;
        int32_t *d_ps = nullptr, *d_st = nullptr;
        if ((st = dev_alloc(pl.get(), &d_len, sizeof(double) * std::max<int64_t>(1, ne)))) return st;
        if ((st = dev_alloc(pl.get(), &d_lnl, sizeof(double) * std::max(1, nb)))) return st;
        if (ne) PT_HIP(hipMemcpyAsync(d_len, cl.data(), sizeof(double) * ne, hipMemcpyHostToDevice, ctx->stream));
        pt::OptParams op{};
        if (kind == PT_PLAN_OPTIMIZE) {
            op = to_params(o);
            if ((st = dev_alloc(pl.get(), &d_ps, sizeof(int32_t) * std::max(1, nb)))) return st;
            if ((st = dev_alloc(pl.get(), &d_st, sizeof(int32_t) * std::max(1, nb)))) return st;
            st = enqueue(pl.get(), kind, nullptr, d_len, &op, d_lnl, d_ps, d_st, nullptr, nullptr, ctx->stream);
            if (!st && pl->opt_groups > 1) {
                // A tree split over several blocks needs all of them resident
                // at once; when other work holds compute units a cross-block
                // wait times out (status 2).  The chunk is then optimised
                // again from its starting lengths with one block per tree.
                std::vector<int32_t> h_st(nb);
                PT_HIP(hipMemcpyAsync(h_st.data(), d_st, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, ctx->stream));
                PT_HIP(hipStreamSynchronize(ctx->stream));
                if (std::find(h_st.begin(), h_st.end(), 2) != h_st.end()) {
                    st = configure_shape(pl.get(), 512, 1);
                    if (st) st = configure_shape(pl.get(), 256, 1);
                    if (st) return st;
                    if (ne)
                        PT_HIP(hipMemcpyAsync(d_len, cl.data(), sizeof(double) * ne, hipMemcpyHostToDevice,
                                              ctx->stream));
                    st = enqueue(pl.get(), kind, nullptr, d_len, &op, d_lnl, d_ps, d_st, nullptr, nullptr,
                                 ctx->stream);
                }
            }
        } else if (kind == PT_PLAN_GRAD) {
            if ((st = dev_alloc(pl.get(), &d_g, sizeof(double) * std::max<int64_t>(1, ne)))) return st;
            if (hess_out && (st = dev_alloc(pl.get(), &d_h, sizeof(double) * std::max<int64_t>(1, ne)))) return st;
            st = enqueue(pl.get(), kind, d_len, nullptr, nullptr, d_lnl, nullptr, nullptr, d_g, d_h, ctx->stream);
        } else {
            st = enqueue(pl.get(), kind, d_len, nullptr, nullptr, d_lnl, nullptr, nullptr, nullptr, nullptr, ctx->stream);
        }
        if (st) return st;
        std::vector<double> r_lnl(nb), r_len(kind == PT_PLAN_OPTIMIZE ? ne : 0), r_g(kind == PT_PLAN_GRAD ? ne : 0),
            r_h(d_h ? ne : 0);
        std::vector<int32_t> r_ps(nb), r_st(nb);
        PT_HIP(hipMemcpyAsync(r_lnl.data(), d_lnl, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
        if (kind == PT_PLAN_OPTIMIZE) {
            if (ne) PT_HIP(hipMemcpyAsync(r_len.data(), d_len, sizeof(double) * ne, hipMemcpyDeviceToHost, ctx->stream));
            PT_HIP(hipMemcpyAsync(r_ps.data(), d_ps, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, ctx->stream));
            PT_HIP(hipMemcpyAsync(r_st.data(), d_st, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, ctx->stream));
        }
        if (kind == PT_PLAN_GRAD && ne) {
            PT_HIP(hipMemcpyAsync(r_g.data(), d_g, sizeof(double) * ne, hipMemcpyDeviceToHost, ctx->stream));
            if (d_h) PT_HIP(hipMemcpyAsync(r_h.data(), d_h, sizeof(double) * ne, hipMemcpyDeviceToHost, ctx->stream));
        }
        PT_HIP(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < nb; ++i) {
            const int b = ch[i];
            const int64_t e0 = trees->edge_offset[b];
            lnl[b] = r_lnl[i];
            passes[b] = r_ps[i];
            status[b] = r_st[i];
            for (int64_t x = off[i]; x < off[i + 1]; ++x) {
                if (kind == PT_PLAN_OPTIMIZE) lens_out[e0 + x - off[i]] = r_len[x];
                if (kind == PT_PLAN_GRAD) {
                    grad[e0 + x - off[i]] = r_g[x];
                    if (d_h) hess[e0 + x - off[i]] = r_h[x];
                }
            }
        }
    }
    if (kind == PT_PLAN_OPTIMIZE)
        for (int b = 0; b < B; ++b)
            if (status[b] == 2)
                return fail(PT_EINTERNAL, "tree " + std::to_string(b) + ": a cross-block wait of the "
                                          "optimisation kernel timed out");
    std::copy(lnl.begin(), lnl.end(), lnl_out);
    if (kind == PT_PLAN_OPTIMIZE) {
        std::copy(lens_out.begin(), lens_out.end(), brlen_io);
        if (passes_out) std::copy(passes.begin(), passes.end(), passes_out);
        if (status_out) std::copy(status.begin(), status.end(), status_out);
    }
    if (kind == PT_PLAN_GRAD) {
        std::copy(grad.begin(), grad.end(), grad_out);
        if (hess_out) std::copy(hess.begin(), hess.end(), hess_out);
    }
    return PT_OK;
}

}  // namespace

extern "C" {

const char *pt_last_error(void) { return g_err.c_str(); }

pt_status pt_ctx_create(int32_t device, pt_ctx **out) {
    if (!out) return fail(PT_EINVAL, "out is NULL");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(PT_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(PT_EINVAL, "device index out of range");
    auto *c = new pt_ctx;
    c->device = device;
    c->pool->device = device;
    hipDeviceProp_t prop;
    if ((e = hipSetDevice(device)) != hipSuccess || (e = hipGetDeviceProperties(&prop, device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete c;
        return fail(PT_EDEVICE, std::string("device set-up: ") + hipGetErrorString(e));
    }
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    if ((e = pt::noalloc_workspace(device, &c->noalloc)) != hipSuccess) {
        c->noalloc = nullptr;
        c->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
    }
    *out = c;
    return PT_OK;
}

void pt_ctx_destroy(pt_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    pool_trim(ctx->pool.get(), 0);  // plans still alive keep the pool itself
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

pt_status pt_aln_create(pt_ctx *ctx, int32_t n_taxa, int32_t n_patterns, const uint8_t *tips, const double *weights,
                        const pt_model *model, pt_aln **out) {
    if (!ctx || !tips || !weights || !model || !out) return fail(PT_EINVAL, "NULL argument");
    if (n_taxa < 2) return fail(PT_EINVAL, "n_taxa must be >= 2");
    if (n_patterns < 1) return fail(PT_EINVAL, "n_patterns must be >= 1");
    for (int64_t i = 0; i < (int64_t)n_taxa * n_patterns; ++i)
        if (tips[i] == 0 || tips[i] > 15) return fail(PT_EINVAL, "tip codes must be in 1..15");
    for (int p = 0; p < n_patterns; ++p)
        if (!(weights[p] > 0.0) || !std::isfinite(weights[p])) return fail(PT_EINVAL, "weights must be finite and > 0");
    AlnDev d{};
    std::string err;
    pt_status st = pt::build_model(*model, d, err);
    if (st) return fail(st, err);
    d.n_taxa = n_taxa;
    d.P = n_patterns;
    auto *a = new pt_aln;
    a->ctx = ctx;
    a->n_taxa = n_taxa;
    a->P = n_patterns;
    hipError_t e;
    size_t tb = (size_t)n_taxa * n_patterns;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess || (e = hipMalloc(&a->d_tips, tb)) != hipSuccess ||
        (e = hipMalloc(&a->d_w, sizeof(double) * n_patterns)) != hipSuccess ||
        (e = hipMemcpy(a->d_tips, tips, tb, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(a->d_w, weights, sizeof(double) * n_patterns, hipMemcpyHostToDevice)) != hipSuccess) {
        pt_aln_destroy(a);
        return fail(e == hipErrorOutOfMemory ? PT_ENOMEM : PT_EDEVICE, std::string("alignment upload: ") + hipGetErrorString(e));
    }
    d.tips = a->d_tips;
    d.w = a->d_w;
    a->desc = d;
    *out = a;
    return PT_OK;
}

void pt_aln_destroy(pt_aln *aln) {
    if (!aln) return;
    if (aln->d_tips) (void)hipFree(aln->d_tips);
    if (aln->d_w) (void)hipFree(aln->d_w);
    delete aln;
}

void pt_opt_default(int32_t precision, pt_opt *out) {
    if (!out) return;
    out->t_min = 1e-8;
    out->t_max = 100.0;
    out->max_passes = 200;
    out->max_newton = 32;
    out->prior_rate = 0.0;
    if (precision == PT_FP32) {
        out->tol_lnl = 1e-5;
        out->tol_t = 1e-3;
        out->tol_newton = 1e-6;
    } else {
        out->tol_lnl = 1e-8;
        out->tol_t = 1e-5;
        out->tol_newton = 1e-9;
    }
}

pt_status pt_batch_loglik(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees, const double *brlen,
                          int32_t precision, double *lnl_out) {
    return host_batch(ctx, alns, n_alns, trees, nullptr, brlen, nullptr, nullptr, precision, PT_PLAN_LOGLIK, lnl_out,
                      nullptr, nullptr, nullptr, nullptr);
}

pt_status pt_batch_optimize_branches(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                                     double *brlen_inout, const uint8_t *opt_mask, const pt_opt *opt,
                                     int32_t precision, double *lnl_out, int32_t *passes_out, int32_t *status_out) {
    if (!brlen_inout && trees && trees->n_trees > 0) return fail(PT_EINVAL, "brlen_inout is NULL");
    return host_batch(ctx, alns, n_alns, trees, brlen_inout, nullptr, opt_mask, opt, precision, PT_PLAN_OPTIMIZE,
                      lnl_out, passes_out, status_out, nullptr, nullptr);
}

pt_status pt_batch_branch_grad(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                               const double *brlen, int32_t precision, double *lnl_out, double *grad_out,
                               double *hess_diag_out) {
    return host_batch(ctx, alns, n_alns, trees, nullptr, brlen, nullptr, nullptr, precision, PT_PLAN_GRAD, lnl_out,
                      nullptr, nullptr, grad_out, hess_diag_out);
}

pt_status pt_batch_loglik_noalloc(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                                  const double *brlen, int32_t precision, double *lnl_out) {
    std::vector<int> ntx;
    pt_status st = check_trees(ctx, alns, n_alns, trees, ntx);
    if (st) return st;
    if (precision != PT_FP32 && precision != PT_FP64) return fail(PT_EINVAL, "precision must be PT_FP64 or PT_FP32");
    const int B = trees->n_trees;
    const int64_t NE = B ? trees->edge_offset[B] : 0;
    if ((st = check_lengths(brlen, NE))) return st;
    if (B > 0 && !lnl_out) return fail(PT_EINVAL, "lnl_out is NULL");
    if (B == 0) return PT_OK;
    if (!ctx->noalloc) return fail(PT_EDEVICE, "no-allocation workspace unavailable: " + ctx->noalloc_err);
    const int kp = kp_of_plan(alns, trees);
    const int reg_pats = pt::loglik_reg_tile_patterns(kp);
    // programs and descriptors on the host (host memory only)
    std::vector<Op> ops;
    std::vector<TreeDev> td(B);
    std::vector<AlnDev> ad(B);
    std::vector<int32_t> edge_tree(NE), tile_tree;
    std::vector<int> tree_E(B);
    int depth = 0, n_max = 0;
    int64_t pm_off = 0;
    for (int b = 0; b < B; ++b) {
        pt::Tree t;
        std::string err;
        if ((st = pt::build_tree(ntx[b], trees->edges + 2 * trees->edge_offset[b], t, err)))
            return fail(st, "tree " + std::to_string(b) + ": " + err);
        const AlnDev &a = alns[trees->aln_index[b]]->desc;
        TreeDev d{};
        d.aln = b;
        d.n_edges = t.n_edges;
        d.edge_off = trees->edge_offset[b];
        d.pm_off = pm_off;
        d.op_first = (int32_t)ops.size();
        depth = std::max(depth, pt::compile_loglik_reg(t, ops));
        d.n_first = (int32_t)ops.size() - d.op_first;
        d.n_tiles = (a.P + reg_pats - 1) / reg_pats;
        td[b] = d;
        ad[b] = a;
        tree_E[b] = t.n_edges;
        n_max = std::max(n_max, ntx[b]);
        pm_off += (int64_t)t.n_edges * kp * 16;
        for (int e = 0; e < t.n_edges; ++e) edge_tree[d.edge_off + e] = b;
    }
    if (depth > pt::kRegStack) return fail(PT_EUNSUPPORTED, "a tree needs more than 8 stack slots");
    const size_t lds = pt::loglik_reg_lds(kp, n_max, depth);
    if (lds > ctx->lds_per_block) return fail(PT_EUNSUPPORTED, "a tree exceeds the LDS of a block");
    {   // tiles of the trees with the most edges first
        std::vector<int> order(B);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tree_E[x] > tree_E[y]; });
        for (int b : order) {
            td[b].tile_begin = (int32_t)tile_tree.size();
            for (int x = 0; x < td[b].n_tiles; ++x) tile_tree.push_back(b);
        }
    }
    const int tiles = (int)tile_tree.size();
    // workspace layout: the sections copied from the host, then the ones the
    // kernels write; each 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const double ident[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    const size_t o_aln = 0, o_tree = up(o_aln + sizeof(AlnDev) * B), o_ops = up(o_tree + sizeof(TreeDev) * B),
                 o_etree = up(o_ops + sizeof(Op) * ops.size()), o_ttree = up(o_etree + sizeof(int32_t) * NE),
                 o_len = up(o_ttree + sizeof(int32_t) * tiles), o_ident = up(o_len + sizeof(double) * NE),
                 in_bytes = o_ident + sizeof(ident), o_pm = up(in_bytes),
                 o_part = up(o_pm + sizeof(double) * pm_off), o_lnl = up(o_part + sizeof(double) * 3 * tiles),
                 total = o_lnl + sizeof(double) * B;
    if (total > pt::kNoAllocBytes)
        return fail(PT_ENOMEM, "batch needs " + std::to_string(total) + " bytes of the " +
                                   std::to_string(pt::kNoAllocBytes) + "-byte no-allocation workspace");
    std::vector<uint8_t> img(in_bytes);
    std::memcpy(img.data() + o_aln, ad.data(), sizeof(AlnDev) * B);
    std::memcpy(img.data() + o_tree, td.data(), sizeof(TreeDev) * B);
    std::memcpy(img.data() + o_ops, ops.data(), sizeof(Op) * ops.size());
    std::memcpy(img.data() + o_etree, edge_tree.data(), sizeof(int32_t) * NE);
    std::memcpy(img.data() + o_ttree, tile_tree.data(), sizeof(int32_t) * tiles);
    std::memcpy(img.data() + o_len, brlen, sizeof(double) * NE);
    std::memcpy(img.data() + o_ident, ident, sizeof(ident));
    char *ws = reinterpret_cast<char *>(ctx->noalloc);
    hipStream_t s = ctx->stream;
    PT_HIP(hipSetDevice(ctx->device));
    PT_HIP(hipMemcpyAsync(ws, img.data(), in_bytes, hipMemcpyHostToDevice, s));
    pt::BatchArgs a{};
    a.trees = reinterpret_cast<const TreeDev *>(ws + o_tree);
    a.alns = reinterpret_cast<const AlnDev *>(ws + o_aln);
    a.ops = reinterpret_cast<const Op *>(ws + o_ops);
    a.edge_tree = reinterpret_cast<const int32_t *>(ws + o_etree);
    a.tile_tree = reinterpret_cast<const int32_t *>(ws + o_ttree);
    a.pmat = reinterpret_cast<double *>(ws + o_pm);
    a.part = reinterpret_cast<double *>(ws + o_part);
    a.n_trees = B;
    a.n_tiles = tiles;
    a.n_edges = NE;
    a.part_cols = 1;
    a.kp = kp;
    a.reg_depth = depth;
    a.ident = reinterpret_cast<const double *>(ws + o_ident);
    double *d_lnl = reinterpret_cast<double *>(ws + o_lnl);
    hipError_t e;
    if ((e = pt::launch_pmat(a, reinterpret_cast<const double *>(ws + o_len), s)) != hipSuccess ||
        (e = pt::launch_loglik_reg(kp, a, lds, s)) != hipSuccess ||
        (e = pt::launch_reduce(false, a, d_lnl, nullptr, nullptr, s)) != hipSuccess)
        return fail(PT_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    std::vector<double> out(B);
    PT_HIP(hipMemcpyAsync(out.data(), d_lnl, sizeof(double) * B, hipMemcpyDeviceToHost, s));
    PT_HIP(hipStreamSynchronize(s));
    std::copy(out.begin(), out.end(), lnl_out);
    return PT_OK;
}

pt_status pt_plan_create(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns, const pt_trees *trees,
                         const uint8_t *opt_mask, int32_t precision, int32_t kinds, pt_plan **out) {
    if (!out) return fail(PT_EINVAL, "out is NULL");
    return plan_build(ctx, alns, n_alns, trees, opt_mask, precision, kinds, out);
}

void pt_plan_destroy(pt_plan *plan) { free_plan(plan); }

pt_status pt_plan_set_graphs(pt_plan *plan, int32_t enable) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    plan->graphs = enable != 0;
    return PT_OK;
}

pt_status pt_plan_loglik(pt_plan *plan, const double *d_brlen, double *d_lnl, void *stream) {
    if (!plan || !(plan->kinds & PT_PLAN_LOGLIK)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_LOGLIK");
    if (plan->n_trees && (!d_brlen || !d_lnl)) return fail(PT_EINVAL, "NULL device pointer");
    return run(plan, PT_PLAN_LOGLIK, d_brlen, nullptr, nullptr, d_lnl, nullptr, nullptr, nullptr, nullptr,
               (hipStream_t)stream);
}

pt_status pt_plan_optimize(pt_plan *plan, double *d_brlen_inout, const pt_opt *opt, double *d_lnl, int32_t *d_passes,
                           int32_t *d_status, void *stream) {
    if (!plan || !(plan->kinds & PT_PLAN_OPTIMIZE)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_OPTIMIZE");
    if (plan->n_trees && (!d_brlen_inout || !d_lnl)) return fail(PT_EINVAL, "NULL device pointer");
    pt_opt o;
    if (opt) o = *opt; else pt_opt_default(plan->precision, &o);
    pt_status st = check_opt(o);
    if (st) return st;
    pt::OptParams p = to_params(o);
    return run(plan, PT_PLAN_OPTIMIZE, nullptr, d_brlen_inout, &p, d_lnl, d_passes, d_status, nullptr, nullptr,
               (hipStream_t)stream);
}

pt_status pt_plan_grad(pt_plan *plan, const double *d_brlen, double *d_lnl, double *d_grad, double *d_hess,
                       void *stream) {
    if (!plan || !(plan->kinds & PT_PLAN_GRAD)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_GRAD");
    if (plan->n_trees && (!d_brlen || !d_lnl || !d_grad)) return fail(PT_EINVAL, "NULL device pointer");
    return run(plan, PT_PLAN_GRAD, d_brlen, nullptr, nullptr, d_lnl, nullptr, nullptr, d_grad, d_hess,
               (hipStream_t)stream);
}

pt_status pt_plan_autotune(pt_plan *plan, const double *d_brlen, const pt_opt *opt, int32_t *block, int32_t *items) {
    if (!plan || !(plan->kinds & PT_PLAN_OPTIMIZE)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_OPTIMIZE");
    if (plan->n_trees == 0) return PT_OK;
    if (!d_brlen) return fail(PT_EINVAL, "d_brlen is NULL");
    pt_opt o;
    if (opt) o = *opt; else pt_opt_default(plan->precision, &o);
    pt_status st = check_opt(o);
    if (st) return st;
    pt::OptParams p = to_params(o);
    PT_HIP(hipSetDevice(plan->ctx->device));
    hipStream_t s = plan->ctx->stream;
    double *d_lnl = nullptr;
    if ((st = dev_alloc(plan, &d_lnl, sizeof(double) * plan->n_trees))) return st;
    int best_b = plan->opt_block, best_g = plan->opt_groups;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    PT_HIP(hipEventCreate(&e0));
    PT_HIP(hipEventCreate(&e1));
    const size_t nb = sizeof(double) * plan->n_edges;
    for (const auto &shape : std::vector<std::pair<int, int>>{{256, 1}, {512, 1}, {256, 2}, {512, 2}, {256, 3},
                                                            {512, 3}, {256, 4}, {512, 4}, {256, 5}, {512, 5},
                                                            {256, 6}, {512, 6}, {256, 8}, {512, 8}}) {
        const int bs = shape.first, groups = shape.second;
        if (configure_shape(plan, bs, groups) != PT_OK) continue;
        float trial = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            PT_HIP(hipMemcpyAsync(plan->d_scratch, d_brlen, nb, hipMemcpyDeviceToDevice, s));
            PT_HIP(hipEventRecord(e0, s));
            st = enqueue(plan, PT_PLAN_OPTIMIZE, nullptr, plan->d_scratch, &p, d_lnl, nullptr, nullptr, nullptr,
                         nullptr, s);
            if (st) return st;
            PT_HIP(hipEventRecord(e1, s));
            PT_HIP(hipEventSynchronize(e1));
            float ms = 0;
            PT_HIP(hipEventElapsedTime(&ms, e0, e1));
            trial = std::min(trial, ms);
        }
        if (trial < best_ms) {
            best_ms = trial;
            best_b = bs;
            best_g = groups;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((st = configure_shape(plan, best_b, best_g))) return st;
    for (auto &kv : plan->execs) (void)hipGraphExecDestroy(kv.second);
    plan->execs.clear();
    plan->ctx->tuned[std::make_tuple(plan->precision, plan->kp, plan->max_P)] = {best_b, best_g};
    if (block) *block = plan->opt_block;
    if (items) *items = plan->opt_items;
    return PT_OK;
}

pt_status pt_plan_set_launch(pt_plan *plan, int32_t block, int32_t groups) {
    if (!plan || !(plan->kinds & PT_PLAN_OPTIMIZE)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_OPTIMIZE");
    if (plan->n_trees == 0) return PT_OK;
    const int ob = plan->opt_block, og = plan->opt_groups;
    pt_status st = configure_shape(plan, block, groups);
    if (st) {
        const std::string why = pt_last_error();
        if (configure_shape(plan, ob, og) != PT_OK) return fail(PT_EINTERNAL, "could not restore the launch shape");
        return fail(st, why);
    }
    for (auto &kv : plan->execs) (void)hipGraphExecDestroy(kv.second);
    plan->execs.clear();
    return PT_OK;
}

pt_status pt_ctx_set_group_wait(pt_ctx *ctx, int64_t cycles) {
    if (!ctx) return fail(PT_EINVAL, "ctx is NULL");
    ctx->group_wait = cycles > 0 ? (long long)cycles : 0;
    return PT_OK;
}

pt_status pt_plan_set_tile_patterns(pt_plan *plan, int32_t patterns) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    return set_tile_pats(plan, patterns);
}

pt_status pt_plan_tile_patterns(const pt_plan *plan, int32_t *patterns) {
    if (!plan || !patterns) return fail(PT_EINVAL, "NULL argument");
    *patterns = plan->tile_pats;
    return PT_OK;
}

pt_status pt_plan_autotune_tiles(pt_plan *plan, const double *d_brlen, int32_t *patterns_out) {
    if (!plan || !(plan->kinds & (PT_PLAN_LOGLIK | PT_PLAN_GRAD)))
        return fail(PT_EINVAL, "plan was not created with PT_PLAN_LOGLIK or PT_PLAN_GRAD");
    if (plan->n_trees == 0) {
        if (patterns_out) *patterns_out = plan->tile_pats;
        return PT_OK;
    }
    if (!d_brlen) return fail(PT_EINVAL, "d_brlen is NULL");
    PT_HIP(hipSetDevice(plan->ctx->device));
    hipStream_t s = plan->ctx->stream;
    // time what the tiles run: the gradient when the plan has one, else the
    // stored likelihood pass
    const int kind = (plan->kinds & PT_PLAN_GRAD) ? PT_PLAN_GRAD : PT_PLAN_LOGLIK;
    const int ll_prev = plan->ll_stored;
    if (kind == PT_PLAN_LOGLIK) plan->ll_stored = 1;
    double *d_l = nullptr, *d_g = nullptr;
    pt_status st = dev_alloc(plan, &d_l, sizeof(double) * plan->n_trees);
    if (!st && kind == PT_PLAN_GRAD) st = dev_alloc(plan, &d_g, sizeof(double) * std::max<int64_t>(1, plan->n_edges));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = plan->tile_pats;
    float best_ms = 1e30f;
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(PT_EDEVICE, "hipEventCreate failed");
    for (int pats : {256, 128, 64}) {
        if (st) break;
        if ((st = set_tile_pats(plan, pats))) break;
        float trial = 1e30f;
        for (int rep = 0; rep < 3 && !st; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) { st = fail(PT_EDEVICE, "hipEventRecord failed"); break; }
            st = enqueue(plan, kind, d_brlen, nullptr, nullptr, d_l, nullptr, nullptr, d_g, nullptr, s);
            if (st) break;
            float ms = 0;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(PT_EDEVICE, "event timing failed");
                break;
            }
            if (rep > 0) trial = std::min(trial, ms);  // the first run warms up
        }
        if (!st && trial < best_ms) {
            best_ms = trial;
            best = pats;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    plan->ll_stored = ll_prev;
    if (st) return st;
    if ((st = set_tile_pats(plan, best))) return st;
    plan->ctx->tuned_tiles[std::make_tuple(plan->precision, plan->kp, plan->max_P, plan->max_E)] = best;
    if (patterns_out) *patterns_out = best;
    return PT_OK;
}

pt_status pt_plan_set_loglik_path(pt_plan *plan, int32_t path) {
    if (!plan || !(plan->kinds & PT_PLAN_LOGLIK)) return fail(PT_EINVAL, "plan was not created with PT_PLAN_LOGLIK");
    if (path != PT_LOGLIK_REGISTERS && path != PT_LOGLIK_STORED) return fail(PT_EINVAL, "unknown lnL path");
    if (path == PT_LOGLIK_REGISTERS && plan->n_trees > 0 && !plan->reg_ok)
        return fail(PT_EUNSUPPORTED, "a tree of this plan exceeds the register-resident pass (stack or tip tile)");
    if (path == PT_LOGLIK_STORED && plan->n_trees > 0 && !plan->stored_ok)
        return fail(PT_EUNSUPPORTED, "a tree of this plan exceeds the LDS of the stored pass");
    plan->ll_stored = path == PT_LOGLIK_STORED;
    for (auto &kv : plan->execs) (void)hipGraphExecDestroy(kv.second);
    plan->execs.clear();
    return PT_OK;
}

pt_status pt_plan_launch_shape(const pt_plan *plan, int32_t *block, int32_t *items, int32_t *groups) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    if (block) *block = plan->opt_block;
    if (items) *items = plan->opt_items;
    if (groups) *groups = plan->opt_groups;
    return PT_OK;
}

namespace {

// Brent's minimiser of a function of one variable on [a, b] (R. P. Brent,
// "Algorithms for Minimization without Derivatives", 1973, chapter 5):
// golden-section steps, replaced by a parabola through the three best points
// when its minimum lies well inside the bracket and the step is shrinking.
// Reverse communication -- point() is the abscissa to evaluate next and
// tell() takes its value -- so that the minimisations of many trees advance
// in lockstep, one batched likelihood launch per step.
struct BrentMin {
    double a = 0, b = 0, x = 0, w = 0, v = 0, fx = 0, fw = 0, fv = 0, d = 0, e = 0, u = 0, tol = 0;
    bool started = false, done = false;

    void init(double lo, double hi, double x0, double tol_) {
        a = lo;
        b = hi;
        x = w = v = u = std::min(std::max(x0, lo), hi);
        d = e = 0.0;
        tol = tol_;
        started = done = false;
    }
    double point() const { return u; }
    void tell(double fu) {
        if (!started) {
            fx = fw = fv = fu;
            started = true;
        } else if (fu <= fx) {
            if (u >= x) a = x; else b = x;
            v = w; fv = fw;
            w = x; fw = fx;
            x = u; fx = fu;
        } else {
            if (u < x) a = u; else b = u;
            if (fu <= fw || w == x) {
                v = w; fv = fw;
                w = u; fw = fu;
            } else if (fu <= fv || v == x || v == w) {
                v = u; fv = fu;
            }
        }
        step();
    }

  private:
    void step() {
        const double golden = 0.5 * (3.0 - std::sqrt(5.0));
        const double xm = 0.5 * (a + b);
        const double tol1 = 1.5e-8 * std::fabs(x) + tol / 3.0, tol2 = 2.0 * tol1;
        if (std::fabs(x - xm) <= tol2 - 0.5 * (b - a)) {
            done = true;
            u = x;
            return;
        }
        bool parabola = false;
        if (std::fabs(e) > tol1) {
            double r = (x - w) * (fx - fv), q = (x - v) * (fx - fw), p = (x - v) * q - (x - w) * r;
            q = 2.0 * (q - r);
            if (q > 0.0) p = -p;
            q = std::fabs(q);
            const double e_prev = e;
            e = d;
            if (std::fabs(p) < std::fabs(0.5 * q * e_prev) && p > q * (a - x) && p < q * (b - x)) {
                d = p / q;
                parabola = true;
                const double t = x + d;
                if (t - a < tol2 || b - t < tol2) d = std::copysign(tol1, xm - x);
            }
        }
        if (!parabola) {
            e = x >= xm ? a - x : b - x;
            d = golden * e;
        }
        u = x + (std::fabs(d) >= tol1 ? d : std::copysign(tol1, d));
    }
};

pt_status set_alpha(pt_plan *pl, const double *alpha, hipStream_t s) {
    std::string err;
    for (int b = 0; b < pl->n_trees; ++b) {
        AlnDev d = pl->alns_base_h[b];
        if (alpha && d.K > 1) {
            pt_status st = pt::gamma_category_rates(alpha[b], d.K, d.rate, err);
            if (st) return fail(st, "tree " + std::to_string(b) + ": " + err);
            for (int k = d.K; k < pt::kMaxCats; ++k) d.rate[k] = 0.0;
        }
        pl->alns_h[b] = d;
    }
    if (pl->n_trees == 0) return PT_OK;
    PT_HIP(hipSetDevice(pl->ctx->device));
    PT_HIP(hipMemcpyAsync(pl->d_alns, pl->alns_h.data(), sizeof(AlnDev) * pl->n_trees, hipMemcpyHostToDevice, s));
    PT_HIP(hipStreamSynchronize(s));
    return PT_OK;
}

}  // namespace

pt_status pt_plan_set_alpha(pt_plan *plan, const double *alpha, void *stream) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    if (alpha)
        for (int b = 0; b < plan->n_trees; ++b)
            if (!(alpha[b] > 0.0) || !std::isfinite(alpha[b]))
                return fail(PT_EINVAL, "alpha[" + std::to_string(b) + "] must be finite and > 0");
    return set_alpha(plan, alpha, (hipStream_t)stream);
}

pt_status pt_plan_optimize_alpha(pt_plan *plan, double *d_brlen_inout, const pt_opt *opt, double *alpha_inout,
                                 double alpha_min, double alpha_max, double tol_alpha, int32_t max_rounds,
                                 double *lnl_out, int32_t *rounds_out, void *stream) {
    if (!plan || (plan->kinds & (PT_PLAN_OPTIMIZE | PT_PLAN_LOGLIK)) != (PT_PLAN_OPTIMIZE | PT_PLAN_LOGLIK))
        return fail(PT_EINVAL, "plan was not created with PT_PLAN_OPTIMIZE | PT_PLAN_LOGLIK");
    const int B = plan->n_trees;
    if (B && (!d_brlen_inout || !alpha_inout || !lnl_out)) return fail(PT_EINVAL, "NULL argument");
    if (!(alpha_min > 0.0) || !(alpha_max > alpha_min) || !std::isfinite(alpha_max))
        return fail(PT_EINVAL, "need 0 < alpha_min < alpha_max < inf");
    if (!(tol_alpha > 0.0) || max_rounds < 1) return fail(PT_EINVAL, "need tol_alpha > 0 and max_rounds >= 1");
    for (int b = 0; b < B; ++b)
        if (!(alpha_inout[b] >= alpha_min && alpha_inout[b] <= alpha_max))
            return fail(PT_EINVAL, "alpha[" + std::to_string(b) + "] outside [alpha_min, alpha_max]");
    pt_opt o;
    if (opt) o = *opt; else pt_opt_default(plan->precision, &o);
    pt_status st = check_opt(o);
    if (st) return st;
    if (B == 0) {
        if (rounds_out) *rounds_out = 0;
        return PT_OK;
    }
    const pt::OptParams p = to_params(o);
    hipStream_t s = (hipStream_t)stream;
    if (!plan->d_alpha_lnl && (st = dev_alloc(plan, &plan->d_alpha_lnl, sizeof(double) * B))) return st;
    std::vector<double> alpha(alpha_inout, alpha_inout + B), trial(B), f(B), best(B, -INFINITY), cur(B);
    std::vector<char> active(B, 1);  // trees whose shape still moves
    std::vector<BrentMin> br(B);
    const double lo = std::log(alpha_min), hi = std::log(alpha_max);
    int rounds = 0;
    for (;;) {
        // lengths at the current shapes; their lnL (the optimiser's, from
        // FP64 partials in either precision) judges convergence
        if ((st = set_alpha(plan, alpha.data(), s))) return st;
        if ((st = run(plan, PT_PLAN_OPTIMIZE, nullptr, d_brlen_inout, &p, plan->d_alpha_lnl, nullptr, nullptr,
                      nullptr, nullptr, s)))
            return st;
        PT_HIP(hipMemcpyAsync(cur.data(), plan->d_alpha_lnl, sizeof(double) * B, hipMemcpyDeviceToHost, s));
        PT_HIP(hipStreamSynchronize(s));
        // a tree whose last round gained less than tol_lnl keeps its shape
        bool any_active = false;
        for (int b = 0; b < B; ++b) {
            if (rounds > 0 && cur[b] - best[b] < o.tol_lnl) active[b] = 0;
            any_active = any_active || active[b];
        }
        best = cur;
        if (!any_active || rounds == max_rounds) break;
        ++rounds;
        // shapes at those lengths: Brent on log alpha, the active trees in lockstep
        for (int b = 0; b < B; ++b) {
            br[b].init(lo, hi, std::log(alpha[b]), tol_alpha);
            br[b].done = !active[b];
        }
        for (int it = 0; it < 200; ++it) {
            bool any = false;
            for (int b = 0; b < B; ++b) {
                any = any || !br[b].done;
                trial[b] = std::exp(br[b].done ? br[b].x : br[b].point());
            }
            if (!any) break;
            if ((st = set_alpha(plan, trial.data(), s))) return st;
            if ((st = run(plan, PT_PLAN_LOGLIK, d_brlen_inout, nullptr, nullptr, plan->d_alpha_lnl, nullptr, nullptr,
                          nullptr, nullptr, s)))
                return st;
            PT_HIP(hipMemcpyAsync(f.data(), plan->d_alpha_lnl, sizeof(double) * B, hipMemcpyDeviceToHost, s));
            PT_HIP(hipStreamSynchronize(s));
            for (int b = 0; b < B; ++b)
                if (!br[b].done) br[b].tell(-f[b]);
        }
        for (int b = 0; b < B; ++b) alpha[b] = std::exp(br[b].x);
    }
    std::copy(best.begin(), best.end(), lnl_out);
    std::copy(alpha.begin(), alpha.end(), alpha_inout);
    if (rounds_out) *rounds_out = rounds;
    return PT_OK;
}

pt_status pt_plan_traffic(const pt_plan *plan, int32_t kind, const int32_t *passes, double *bytes_out) {
    if (!plan || !bytes_out) return fail(PT_EINVAL, "NULL argument");
    if (!(plan->kinds & kind) || (kind != PT_PLAN_LOGLIK && kind != PT_PLAN_GRAD && kind != PT_PLAN_OPTIMIZE))
        return fail(PT_EINVAL, "kind not in this plan");
    const std::vector<TreeDev> &tv = kind == PT_PLAN_LOGLIK ? plan->tll_h : kind == PT_PLAN_GRAD ? plan->tgr_h : plan->top_h;
    const double b = (double)store_bytes(plan->precision);
    double total = 0.0;
    if (kind == PT_PLAN_LOGLIK && plan->reg_ok && !plan->ll_stored) {
        // register-resident pass: every tip code and weight once per pattern
        for (int t = 0; t < plan->n_trees; ++t) {
            const AlnDev &a = plan->alns_h[tv[t].aln];
            total += (double)a.P * (a.n_taxa + 8);
        }
        *bytes_out = total;
        return PT_OK;
    }
    for (int t = 0; t < plan->n_trees; ++t) {
        const AlnDev &a = plan->alns_h[tv[t].aln];
        const double slot = (double)a.P * a.K * 4 * b + (double)a.P * 2, tip = (double)a.P;
        auto side = [&](int ref) { return ref < 0 ? tip : slot; };
        auto prog = [&](int o0, int no) {
            double s2 = 0.0;
            for (int o = 0; o < no; ++o) {
                const Op &op = plan->ops_h[o0 + o];
                if (op.code == pt::OP_UPDATE) s2 += side(op.a) + side(op.b) + slot;
                else s2 += side(op.a) + side(op.b) + 8.0 * a.P;
            }
            return s2;
        };
        double bt = prog(tv[t].op_first, tv[t].n_first);
        if (kind == PT_PLAN_OPTIMIZE) {
            int ps = passes ? passes[t] : 1;
            if (ps > 1) bt += (ps - 1) * prog(tv[t].op_steady, tv[t].n_steady);
        }
        total += bt;
    }
    *bytes_out = total;
    return PT_OK;
}

pt_status pt_plan_set_profile(pt_plan *plan, void *d_counters) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    plan->d_prof = reinterpret_cast<long long *>(d_counters);
    for (auto &kv : plan->execs) (void)hipGraphExecDestroy(kv.second);
    plan->execs.clear();
    return PT_OK;
}

pt_status pt_plan_info(const pt_plan *plan, int32_t *n_trees, int64_t *n_edges, int64_t *device_bytes) {
    if (!plan) return fail(PT_EINVAL, "plan is NULL");
    if (n_trees) *n_trees = plan->n_trees;
    if (n_edges) *n_edges = plan->n_edges;
    if (device_bytes) *device_bytes = plan->device_bytes;
    return PT_OK;
}

pt_status pt_model_info(const pt_model *model, double *cat_rates, double *U, double *Uinv, double *lam) {
    if (!model) return fail(PT_EINVAL, "model is NULL");
    AlnDev d{};
    std::string err;
    pt_status st = pt::build_model(*model, d, err);
    if (st) return fail(st, err);
    if (cat_rates) std::copy(d.rate, d.rate + d.K, cat_rates);
    if (U) std::copy(d.U, d.U + 16, U);
    if (Uinv) std::copy(d.Uinv, d.Uinv + 16, Uinv);
    if (lam) std::copy(d.lam, d.lam + 4, lam);
    return PT_OK;
}

pt_status pt_tree_check(int32_t n_taxa, const int32_t *edges) {
    if (!edges) return fail(PT_EINVAL, "edges is NULL");
    pt::Tree t;
    std::string err;
    pt_status st = pt::build_tree(n_taxa, edges, t, err);
    return st ? fail(st, err) : PT_OK;
}

pt_status pt_nni_neighbors(int32_t n, const int32_t *edges, const double *brlen, int32_t *out_edges, double *out_brlen,
                           int32_t *out_touched) {
    if (!edges || !out_edges) return fail(PT_EINVAL, "NULL argument");
    std::string err;
    pt_status st = pt::nni_neighbors(n, edges, brlen, out_edges, out_brlen, out_touched, err);
    return st ? fail(st, err) : PT_OK;
}

pt_status pt_topology_key(int32_t n, const int32_t *edges, uint64_t *out) {
    if (!edges || !out) return fail(PT_EINVAL, "NULL argument");
    std::string err;
    pt_status st = pt::topology_key(n, edges, out, err);
    return st ? fail(st, err) : PT_OK;
}

pt_status pt_topology_keys(int32_t n, int32_t count, const int32_t *edges, uint64_t *out) {
    if (count < 0 || (count > 0 && (!edges || !out))) return fail(PT_EINVAL, "bad arguments");
    const size_t E = n >= 2 ? (size_t)(2 * n - 3) : 0, W = (size_t)(n + 63) / 64;
    std::string err;
    for (int32_t i = 0; i < count; ++i) {
        pt_status st = pt::topology_key(n, edges + i * E * 2, out + i * (size_t)(n > 3 ? n - 3 : 0) * W, err);
        if (st) return fail(st, "tree " + std::to_string(i) + ": " + err);
    }
    return PT_OK;
}

pt_status pt_radius_masks(int32_t n, int32_t count, const int32_t *edges, const int32_t *centres, int32_t radius,
                          uint8_t *out) {
    if (count < 0 || (count > 0 && (!edges || !centres || !out))) return fail(PT_EINVAL, "bad arguments");
    const size_t E = n >= 2 ? (size_t)(n == 2 ? 1 : 2 * n - 3) : 0;
    std::string err;
    for (int32_t i = 0; i < count; ++i) {
        pt_status st = pt::radius_mask(n, edges + i * E * 2, centres[i], radius, out + i * E, err);
        if (st) return fail(st, "tree " + std::to_string(i) + ": " + err);
    }
    return PT_OK;
}

pt_status pt_split_frequencies(int32_t n, int32_t count, const uint64_t *keys, const double *lnl, int32_t cap,
                               int32_t *n_splits, uint64_t *splits, double *freq) {
    if (!keys || !lnl || !n_splits || (cap > 0 && (!splits || !freq)) || cap < 0)
        return fail(PT_EINVAL, "bad arguments");
    std::string err;
    pt_status st = pt::split_frequencies(n, count, keys, lnl, cap, n_splits, splits, freq, err);
    return st ? fail(st, err) : PT_OK;
}

pt_status pt_majority_consensus(int32_t n, int32_t n_splits, const uint64_t *splits, const double *freq, char *out,
                                int32_t cap, int32_t *len_out) {
    if (n_splits < 0 || (n_splits > 0 && (!splits || !freq)) || !out || !len_out || cap < 1)
        return fail(PT_EINVAL, "bad arguments");
    std::string err;
    pt_status st = pt::majority_consensus(n, n_splits, splits, freq, out, cap, len_out, err);
    return st ? fail(st, err) : PT_OK;
}

pt_status pt_nni_features(int32_t n, const int32_t *edges, const double *brlen, float *out) {
    if (!edges || !brlen || !out) return fail(PT_EINVAL, "NULL argument");
    std::string err;
    pt_status st = pt::nni_features(n, edges, brlen, out, err);
    return st ? fail(st, err) : PT_OK;
}

}  // extern "C"

struct pt_mlp {
    pt_ctx *ctx = nullptr;
    int ni = 0, nh = 0, no = 0, np = 0;
    int64_t step = 0;
    float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
    int cap = 0;
    float *d_h = nullptr, *d_y = nullptr, *d_dy = nullptr, *d_dz = nullptr;
    double *d_rl = nullptr, *d_part = nullptr;  // d_part: row-tile sums of the weight gradient
};

namespace {

void mlp_free_scratch(pt_mlp *m) {
    for (void *p : {(void *)m->d_h, (void *)m->d_y, (void *)m->d_dy, (void *)m->d_dz, (void *)m->d_rl,
                    (void *)m->d_part})
        if (p) (void)hipFree(p);
    m->d_h = m->d_y = m->d_dy = m->d_dz = nullptr;
    m->d_rl = m->d_part = nullptr;
    m->cap = 0;
}

pt_status mlp_scratch(pt_mlp *m, int rows) {
    if (rows <= m->cap) return PT_OK;
    mlp_free_scratch(m);
    const size_t r = (size_t)rows;
    PT_HIP(hipMalloc(&m->d_h, sizeof(float) * r * m->nh));
    PT_HIP(hipMalloc(&m->d_dz, sizeof(float) * r * m->nh));
    PT_HIP(hipMalloc(&m->d_y, sizeof(float) * r * m->no));
    PT_HIP(hipMalloc(&m->d_dy, sizeof(float) * r * m->no));
    PT_HIP(hipMalloc(&m->d_rl, sizeof(double) * r));
    const size_t part = pt::mlp_wgrad_part_doubles(rows, m->ni, m->nh, m->no);
    if (part) PT_HIP(hipMalloc(&m->d_part, sizeof(double) * part));
    m->cap = rows;
    return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_mlp_create(pt_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params,
                        pt_mlp **out) {
    if (!ctx || !params || !out) return fail(PT_EINVAL, "NULL argument");
    if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_in > 4096 || n_hidden > 4096 || n_out > 4096)
        return fail(PT_EINVAL, "layer sizes must be in 1..4096");
    std::unique_ptr<pt_mlp> m(new pt_mlp);
    m->ctx = ctx;
    m->ni = n_in;
    m->nh = n_hidden;
    m->no = n_out;
    m->np = n_in * n_hidden + n_hidden + n_hidden * n_out + n_out;
    for (int i = 0; i < m->np; ++i)
        if (!std::isfinite(params[i])) return fail(PT_EINVAL, "parameters must be finite");
    PT_HIP(hipSetDevice(ctx->device));
    const size_t b = sizeof(float) * m->np;
    PT_HIP(hipMalloc(&m->d_p, b));
    PT_HIP(hipMalloc(&m->d_m, b));
    PT_HIP(hipMalloc(&m->d_v, b));
    PT_HIP(hipMalloc(&m->d_g, b));
    PT_HIP(hipMemcpy(m->d_p, params, b, hipMemcpyHostToDevice));
    PT_HIP(hipMemset(m->d_m, 0, b));
    PT_HIP(hipMemset(m->d_v, 0, b));
    *out = m.release();
    return PT_OK;
}

void pt_mlp_destroy(pt_mlp *mlp) {
    if (!mlp) return;
    mlp_free_scratch(mlp);
    for (void *p : {(void *)mlp->d_p, (void *)mlp->d_m, (void *)mlp->d_v, (void *)mlp->d_g})
        if (p) (void)hipFree(p);
    delete mlp;
}

int64_t pt_mlp_param_count(const pt_mlp *mlp) { return mlp ? mlp->np : 0; }

pt_status pt_mlp_get_params(pt_mlp *mlp, float *params_out) {
    if (!mlp || !params_out) return fail(PT_EINVAL, "NULL argument");
    PT_HIP(hipMemcpy(params_out, mlp->d_p, sizeof(float) * mlp->np, hipMemcpyDeviceToHost));
    return PT_OK;
}

pt_status pt_mlp_set_params(pt_mlp *mlp, const float *params) {
    if (!mlp || !params) return fail(PT_EINVAL, "NULL argument");
    PT_HIP(hipMemcpy(mlp->d_p, params, sizeof(float) * mlp->np, hipMemcpyHostToDevice));
    return PT_OK;
}

pt_status pt_mlp_forward(pt_mlp *mlp, const float *d_x, int32_t rows, float *d_y, void *stream) {
    if (!mlp || rows < 0 || (rows > 0 && (!d_x || !d_y))) return fail(PT_EINVAL, "bad arguments");
    pt_status st = mlp_scratch(mlp, rows);
    if (st) return st;
    PT_HIP(pt::mlp_forward(d_x, mlp->d_p, rows, mlp->ni, mlp->nh, mlp->no, mlp->d_h, d_y, (hipStream_t)stream));
    return PT_OK;
}

pt_status pt_mlp_warm_start(pt_mlp *mlp, const float *d_x, int32_t rows, const int32_t *d_pos, const double *d_base,
                            double shift, double t_min, double t_max, double *d_brlen, void *stream) {
    if (!mlp || rows < 0 || (rows > 0 && (!d_x || !d_pos || !d_base || !d_brlen)))
        return fail(PT_EINVAL, "bad arguments");
    if (!(t_min > 0.0) || !(t_max > t_min)) return fail(PT_EINVAL, "need 0 < t_min < t_max");
    if (!(shift > 0.0) || !std::isfinite(shift)) return fail(PT_EINVAL, "need shift > 0");
    pt_status st = mlp_scratch(mlp, rows);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    PT_HIP(pt::mlp_forward(d_x, mlp->d_p, rows, mlp->ni, mlp->nh, mlp->no, mlp->d_h, mlp->d_y, s));
    PT_HIP(pt::mlp_warm_apply(mlp->d_y, d_pos, d_base, rows, mlp->no, shift, t_min, t_max, d_brlen, s));
    return PT_OK;
}

pt_status pt_mlp_gradient(pt_mlp *mlp, const float *d_x, const float *d_target, int32_t rows, float *d_grad,
                          double *d_loss, void *stream) {
    if (!mlp || rows < 1 || !d_x || !d_target || !d_grad) return fail(PT_EINVAL, "bad arguments");
    pt_status st = mlp_scratch(mlp, rows);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    PT_HIP(pt::mlp_forward(d_x, mlp->d_p, rows, mlp->ni, mlp->nh, mlp->no, mlp->d_h, mlp->d_y, s));
    PT_HIP(pt::mlp_loss_grad(mlp->d_y, d_target, rows, mlp->no, mlp->d_dy, mlp->d_rl, d_loss, s));
    PT_HIP(pt::mlp_backward(d_x, mlp->d_p, mlp->d_h, mlp->d_dy, rows, mlp->ni, mlp->nh, mlp->no, mlp->d_dz, d_grad,
                            mlp->d_part, s));
    return PT_OK;
}

pt_status pt_mlp_train_step(pt_mlp *mlp, const float *d_x, const float *d_target, int32_t rows, const pt_adam *opt,
                            double *d_loss, void *stream) {
    if (!opt || !(opt->lr > 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
        !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !(opt->eps > 0.0f))
        return fail(PT_EINVAL, "bad Adam settings");
    pt_status st = pt_mlp_gradient(mlp, d_x, d_target, rows, mlp ? mlp->d_g : nullptr, d_loss, stream);
    if (st) return st;
    mlp->step += 1;
    const float c1 = 1.0f - std::pow(opt->beta1, (float)mlp->step);
    const float c2 = 1.0f - std::pow(opt->beta2, (float)mlp->step);
    PT_HIP(pt::mlp_adam(mlp->d_p, mlp->d_g, mlp->d_m, mlp->d_v, mlp->np, opt->lr, opt->beta1, opt->beta2, opt->eps,
                        c1, c2, (hipStream_t)stream));
    return PT_OK;
}

}  // extern "C"
