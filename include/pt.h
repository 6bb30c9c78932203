/*
 * pt.h -- C ABI of the MI355X tree-likelihood library.
 *
 * The library evaluates and maximises the log-likelihood of many unrooted
 * binary trees ("topologies") over nucleotide alignments under GTR + discrete
 * Gamma rate variation.  It is the numerical hot path of a systematic search
 * of the high-likelihood set of topologies: a visited topology has its branch
 * lengths optimised to maximise the likelihood, and the neighbours proposed by
 * nearest-neighbour interchange (NNI) are scored by full or partial branch
 * optimisation (Whidden et al., Methods, "Methods Overview" and "Phylogenetic
 * Topographer", the enumerated visit steps and the radius option).
 *
 * Conventions used by every call:
 *   - Status codes only; nothing throws across this boundary.  On error the
 *     outputs are left untouched and pt_last_error() describes the failure.
 *     Every argument is validated on the host before any device work.
 *   - States A,C,G,T.  A tip code is a 4-bit mask, bit j set when state j is
 *     possible (one-hot for a resolved base, 0xF for a gap or N).
 *   - A tree on n taxa is an edge list int32[2n-3][2] of node ids: leaves are
 *     0..n-1 (alignment rows), internal nodes n..2n-3 of degree 3.  Edge order
 *     and orientation are free.  n = 2 is the single edge (0,1).  Branch
 *     lengths, gradients and masks are indexed like the edges.
 *   - Host pointers are owned by the caller and only read (or written, for
 *     outputs) during the call; host-pointer calls are synchronous.  Device
 *     pointers (the pt_plan_* calls) must stay valid until the work enqueued
 *     on the given stream has finished.
 *   - precision PT_FP64: partials stored and combined in FP64.
 *     precision PT_FP32: partials stored in FP32 with per-pattern power-of-two
 *     scaling; transition matrices, arithmetic and every sum over patterns in
 *     FP64.
 */
#ifndef PT_H
#define PT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pt_status;
#define PT_OK 0
#define PT_EINVAL (-1)        /* an argument failed validation */
#define PT_ENOMEM (-2)        /* host or device allocation failed, or the arena cap */
#define PT_EDEVICE (-3)       /* a HIP runtime call failed */
#define PT_EUNSUPPORTED (-4)  /* valid input beyond the library's limits */
#define PT_EINTERNAL (-5)

#define PT_FP64 0
#define PT_FP32 1

/* Message of the last failing call on this thread ("" when none). */
const char *pt_last_error(void);

/* ----------------------------------------------------------------- context */

/* A context owns one device's stream, memory and tuning table.  Limits:
 * device index as seen by HIP.  The environment variable PT_ARENA_CAP_BYTES
 * (decimal) caps the device bytes one batch may use; host-pointer batch calls
 * split a batch that exceeds it into smaller batches with identical results.
 * Device memory of destroyed plans stays with the context for later plans
 * (a new plan takes a kept block of one to two times the size it needs), up
 * to PT_POOL_CAP_BYTES (decimal, default 64 GiB); a failing allocation first
 * returns the kept blocks to the device.  pt_ctx_destroy frees them; a plan
 * that outlives its context may still be destroyed (its memory is then freed
 * when the last such plan goes), but no other call may use it. */
typedef struct pt_ctx pt_ctx;
pt_status pt_ctx_create(int32_t device, pt_ctx **out);
void pt_ctx_destroy(pt_ctx *ctx);
/* Shader clocks after which a cross-block wait of the optimisation kernel
 * (trees split over several blocks, pt_plan_set_launch) gives up and marks
 * its tree status 2, for launches made from now on with this context;
 * cycles <= 0 restores the default, 2^27 (about 50 ms).  A small limit lets
 * a caller test its handling of status 2; every wait stays bounded. */
pt_status pt_ctx_set_group_wait(pt_ctx *ctx, int64_t cycles);

/* ------------------------------------------------------------------- model */

/* GTR + discrete Gamma (the paper's runs use JC69 + Gamma and it supports
 * GTR; Methods, "Phylogenetic Topographer").  Q_ij = rates_ij * freqs_j for
 * i != j, normalised to one expected substitution per unit branch length.
 * n_cats equal-weight categories, each rate the mean of Gamma(alpha, alpha)
 * over its quantile interval; n_cats = 1 means no rate variation. */
typedef struct {
    double rates[6];   /* exchangeabilities AC,AG,AT,CG,CT,GT; > 0, any scale */
    double freqs[4];   /* A,C,G,T; > 0 and summing to 1 within 1e-9 */
    double alpha;      /* Gamma shape > 0; ignored when n_cats == 1 */
    int32_t n_cats;    /* 1..8 */
} pt_model;

/* An alignment as site patterns: tips uint8[n_taxa][n_patterns] tip codes
 * (row-major), weights double[n_patterns] (> 0, the pattern counts).  Copied
 * to the device; the caller's arrays may be freed on return.  2 <= n_taxa,
 * 1 <= n_patterns. */
typedef struct pt_aln pt_aln;
pt_status pt_aln_create(pt_ctx *ctx, int32_t n_taxa, int32_t n_patterns,
                        const uint8_t *tips, const double *weights,
                        const pt_model *model, pt_aln **out);
void pt_aln_destroy(pt_aln *aln);

/* A batch of trees.  Tree b uses alignment alns[aln_index[b]], has n_b taxa
 * (that alignment's row count) and its 2n_b-3 edges are
 * edges[2*edge_offset[b] .. 2*edge_offset[b+1]).  Flat per-edge arrays
 * (lengths, masks, gradients) use the same offsets. */
typedef struct {
    int32_t n_trees;
    const int32_t *aln_index;    /* [n_trees] */
    const int64_t *edge_offset;  /* [n_trees + 1], edge_offset[0] = 0 */
    const int32_t *edges;        /* [edge_offset[n_trees]][2] */
} pt_trees;

/* Branch-length optimisation settings.  Per edge: safeguarded Newton on
 * t in [t_min, t_max], at most max_newton derivative evaluations, stopping
 * when a step would move t by at most tol_newton * max(t, 1e-6) (not taken),
 * or after taking a Newton step of at most max(sqrt(tol_newton), 0.03) *
 * max(t, 1e-6) (quadratic convergence; the next pass revisits the edge, and
 * the per-tree rule below bounds the final accuracy).  From a tree's second
 * pass on, an edge whose Newton step exceeds tol_t relative moves 1.2 times
 * that step, kept in [t_min, t_max] (nonlinear successive over-relaxation:
 * the same maximum in fewer passes; a converged tree's last pass has no step
 * above tol_t, so its lengths are plain Newton results).
 * Per tree: passes over the masked edges until a pass raises the objective
 * by less than tol_lnl and changes no length by more than tol_t relative, or
 * max_passes; a change that starts or ends at t_min or t_max counts only
 * when its gain by the quadratic model at the step's start (first and
 * second derivative) is at least tol_lnl / (2n - 3), or the model is not
 * concave there (with FP32 partials a length whose optimum is t_min would
 * otherwise keep moving on and off the bound by noise-level amounts that
 * change nothing).  With FP32 partials that exemption applies to every
 * change, and a pass's rise is the sum over its steps of the quadratic
 * model's value d1 dt + d2 dt^2 / 2 at each step's start (FP32 partials
 * resolve lnL only to about 1e-4, above tol_lnl, while the model sums are
 * free of that rounding noise).
 * The objective is lnL (prior_rate = 0, maximum likelihood) or, with
 * prior_rate > 0, lnL plus the log density of independent Exponential
 * (prior_rate) priors on every length, sum_e (log prior_rate - prior_rate
 * t_e): MAP lengths (Methods, "Phylogenetic Topographer": the optional
 * exponential branch-length prior; the paper's runs use rate 10).  The
 * optimiser's lnl output is then that objective. */
typedef struct {
    double t_min, t_max;
    double tol_lnl, tol_t, tol_newton;
    int32_t max_passes, max_newton;
    double prior_rate; /* >= 0, finite */
} pt_opt;

/* Defaults for a precision: t_min 1e-8, t_max 100, max_passes 200,
 * max_newton 32, prior_rate 0; FP64 tol_lnl 1e-8, tol_t 1e-5, tol_newton 1e-9; FP32
 * tol_lnl 1e-5, tol_t 1e-3, tol_newton 1e-6 (the reported lnL is
 * evaluated from FP64 partials at the final lengths). */
void pt_opt_default(int32_t precision, pt_opt *out);

/* --------------------------------------------------- host-pointer batches */

/* lnL of every tree at the given lengths (brlen[total edges], >= 0). */
pt_status pt_batch_loglik(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns,
                          const pt_trees *trees, const double *brlen,
                          int32_t precision, double *lnl_out /* [n_trees] */);

/* Maximise lnL over the branch lengths of every tree, starting from
 * brlen_inout and writing the optimised lengths back.  opt_mask[total edges]
 * (NULL = all) selects the edges that move (partial optimisation, the
 * paper's radius option).  opt NULL = pt_opt_default(precision).
 * passes_out / status_out may be NULL; status 0 = the stopping rule was met,
 * 1 = max_passes reached first (not an error).  When the trees of a chunk
 * are split over several blocks (pt_plan_set_launch) and a cross-block wait
 * times out (other work holding compute units; status 2 in the plan calls),
 * the chunk is optimised again from its starting lengths with one block per
 * tree, and those results are returned. */
pt_status pt_batch_optimize_branches(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns,
                                     const pt_trees *trees, double *brlen_inout,
                                     const uint8_t *opt_mask, const pt_opt *opt,
                                     int32_t precision, double *lnl_out,
                                     int32_t *passes_out, int32_t *status_out);

/* lnL and d lnL / d t_e for every edge of every tree (reverse-mode: one
 * post-order and one pre-order sweep of partials).  hess_diag_out (NULL ok)
 * receives d2 lnL / d t_e^2. */
pt_status pt_batch_branch_grad(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns,
                               const pt_trees *trees, const double *brlen,
                               int32_t precision, double *lnl_out,
                               double *grad_out, double *hess_diag_out);

/* pt_batch_loglik for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * same arguments, validation and results, computed by the register-resident
 * pass (FP64, see pt_plan_set_loglik_path) with no hipMalloc, hipFree or
 * other allocating call.  Descriptors, programs, lengths, transition
 * matrices and per-tile sums go to a fixed 64 MiB workspace per device,
 * held by the library until the process ends (about 900 trees of 64 taxa
 * with four categories); PT_ENOMEM, naming the bytes needed, for a batch
 * that does not fit, PT_EUNSUPPORTED for a tree beyond the register pass.
 * Host-pointer call, synchronous on the context's stream.  Every call on a
 * device shares its workspace: calls that overlap on one device (other
 * threads, other contexts of the device) race and must be serialised by
 * the caller. */
pt_status pt_batch_loglik_noalloc(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns,
                                  const pt_trees *trees, const double *brlen,
                                  int32_t precision, double *lnl_out /* [n_trees] */);

/* ------------------------------------------------------ device-side plans */

/* A plan compiles a batch once (validation, rooting, the per-tree program of
 * partial updates and edge steps, device descriptors, partial buffers) so it
 * can be run many times on device-resident lengths.  kinds is a bitwise OR
 * of PT_PLAN_*.  opt_mask as in pt_batch_optimize_branches (fixed per plan).
 * Plan calls enqueue on `stream` (a hipStream_t; NULL = the null stream)
 * and return without waiting.  With graphs enabled (pt_plan_set_graphs), each
 * distinct argument set on a non-NULL stream is captured once into a HIP
 * graph and replayed.  Every layout of a plan uses the category count of the
 * widest alignment its trees use (padded to 1, 2, 4 or 8), so a plan mixing
 * category counts can exceed the per-tree LDS limit (PT_EUNSUPPORTED); the
 * host-pointer batch calls split batches by category count themselves. */
#define PT_PLAN_LOGLIK 1
#define PT_PLAN_OPTIMIZE 2
#define PT_PLAN_GRAD 4
typedef struct pt_plan pt_plan;
pt_status pt_plan_create(pt_ctx *ctx, pt_aln *const *alns, int32_t n_alns,
                         const pt_trees *trees, const uint8_t *opt_mask,
                         int32_t precision, int32_t kinds, pt_plan **out);
/* Waits for the device to finish, then gives the plan's device memory back
 * to its context's kept blocks (see pt_ctx_create); valid also after the
 * context was destroyed. */
void pt_plan_destroy(pt_plan *plan);
pt_status pt_plan_set_graphs(pt_plan *plan, int32_t enable);

/* d_brlen: device double[total edges]; d_lnl: device double[n_trees]. */
pt_status pt_plan_loglik(pt_plan *plan, const double *d_brlen, double *d_lnl, void *stream);
/* d_passes, d_status: device int32[n_trees] or NULL; status as in
 * pt_batch_optimize_branches, plus 2 = a cross-block wait timed out (the
 * tree's lnL is then NaN; see pt_plan_set_launch). */
pt_status pt_plan_optimize(pt_plan *plan, double *d_brlen_inout, const pt_opt *opt,
                           double *d_lnl, int32_t *d_passes, int32_t *d_status,
                           void *stream);
/* d_grad: device double[total edges]; d_hess NULL ok. */
pt_status pt_plan_grad(pt_plan *plan, const double *d_brlen, double *d_lnl,
                       double *d_grad, double *d_hess, void *stream);

/* Patterns per tile of the stored post-order pass and the gradient (64, 128
 * or 256 = one block of that many threads, one pattern each; 256 by
 * default): more, smaller tiles give a small batch more blocks to spread
 * over the device, larger ones fewer passes over each tree's matrices.
 * Re-tiling synchronises the device and drops the plan's captured graphs;
 * results are the same up to the order of the per-tile sums.  EINVAL for
 * another count.  pt_plan_autotune_tiles times the plan's gradient (or, with
 * no gradient, its stored likelihood pass) at each count, from the lengths
 * d_brlen, keeps the fastest for the plan and for later plans of the same
 * precision, padded categories and largest pattern and edge counts in this
 * context, and writes it to *patterns_out (NULL ok). */
pt_status pt_plan_set_tile_patterns(pt_plan *plan, int32_t patterns);
pt_status pt_plan_tile_patterns(const pt_plan *plan, int32_t *patterns);
pt_status pt_plan_autotune_tiles(pt_plan *plan, const double *d_brlen, int32_t *patterns_out);

/* Which pass computes lnL on a PT_PLAN_LOGLIK plan.
 * PT_LOGLIK_REGISTERS (the default whenever every tree fits it): Felsenstein
 * pruning with no partial stored in device memory -- each pattern and
 * category keeps its partials in FP64, an accumulator in registers and a
 * stack of at most 8 slots in LDS, filled in an order that keeps it shallow
 * (enough for any tree of fewer than 512 taxa), and per pattern only the tip
 * codes and the weight are read; the result is FP64 in either precision.
 * A block needs 32 bytes per thread per stack slot plus the tile's tip codes
 * (n bytes per pattern) within the device's LDS per block.
 * PT_LOGLIK_STORED: the post-order pass that starts an optimisation or a
 * gradient, storing every partial in the plan's precision (with FP32
 * partials its lnL carries their rounding, about 1e-4 at a few thousand
 * sites).  PT_EUNSUPPORTED for PT_LOGLIK_REGISTERS when a tree does not fit;
 * such a plan uses the stored pass.  Gradient calls with FP32 partials
 * report the register-resident lnL when the plan's trees fit it. */
#define PT_LOGLIK_REGISTERS 0
#define PT_LOGLIK_STORED 1
pt_status pt_plan_set_loglik_path(pt_plan *plan, int32_t path);

/* Time the optimisation kernel's launch shapes on this plan (lengths are
 * restored after every trial) and keep the fastest for the plan and for
 * every later plan of the same shape class in this context.  Shapes are 256
 * or 512 threads per block, with 1 to 8 blocks per tree (see
 * pt_plan_set_launch).  Writes the chosen threads per block and items per
 * thread to *block, *items (NULL ok). */
pt_status pt_plan_autotune(pt_plan *plan, const double *d_brlen, const pt_opt *opt,
                           int32_t *block, int32_t *items);

/* Set the optimisation kernel's launch shape: `block` threads per block
 * (256 or 512) and `groups` blocks per tree (1..8).  With groups = 1 a block
 * takes one tree at a time from a work queue.  With groups > 1 each tree's
 * patterns are split into `groups` contiguous shares, one per block, and
 * every Newton and lnL reduction is summed across the tree's blocks, which
 * wait for one another (bounded in time; a wait that runs out gives the
 * tree status 2 and lnL NaN).  This is for batches too small to fill the
 * device, and the waits need every block resident at once: it is refused
 * (PT_EUNSUPPORTED, shape unchanged) unless n_trees * groups blocks fit
 * on the device at the kernel's occupancy, and it assumes no other kernel
 * holds the compute units meanwhile.  Also refused: shapes whose kernel
 * would spill registers or whose pattern share is too large.  A new plan
 * uses the shape its context's autotuner last chose for plans of its kind,
 * else, when it has at most half as many trees as the device has compute
 * units, 256 threads and up to 4 blocks per tree, else one block per tree. */
pt_status pt_plan_set_launch(pt_plan *plan, int32_t block, int32_t groups);
/* The optimisation kernel's current shape (any pointer may be NULL). */
pt_status pt_plan_launch_shape(const pt_plan *plan, int32_t *block, int32_t *items, int32_t *groups);

/* Per-tree Gamma shapes (the paper's optional model optimisation, Methods,
 * "Phylogenetic Topographer": in its simplified case, the shape of the
 * Gamma rate distribution is optimised for each visited topology).
 * alpha: host double[n_trees], each finite and > 0, or NULL to return every
 * tree to its alignment's own shape.  Every later call on this plan uses
 * tree b's K discrete-Gamma category means at alpha[b] (Yang 1994, the same
 * discretisation as pt_aln_create); trees with one category are unchanged.
 * The per-tree model descriptors are copied on `stream`, and the call
 * returns after the copy (not to be captured into a graph). */
pt_status pt_plan_set_alpha(pt_plan *plan, const double *alpha, void *stream);

/* Joint optimisation of every tree's branch lengths and Gamma shape: the
 * lengths are optimised at fixed shapes (pt_plan_optimize with opt), then,
 * in each round, the shape of every active tree at fixed lengths by Brent's
 * one-dimensional minimiser on log alpha over [alpha_min, alpha_max] (Brent
 * 1973; the trees in lockstep, one batched pt_plan_loglik per step, each
 * minimisation ending when its bracket is below tol_alpha in log alpha)
 * followed by all lengths again.  A tree whose lnL, after a round's length
 * optimisation, rose by less than opt->tol_lnl keeps its shape from then
 * on; the call ends when no tree is active or after max_rounds rounds,
 * always on a length optimisation.  The plan needs
 * PT_PLAN_OPTIMIZE | PT_PLAN_LOGLIK.  d_brlen_inout: device double[total
 * edges]; alpha_inout: host double[n_trees], starting shapes inside the
 * bounds, overwritten with the optimised ones (the plan keeps them, see
 * pt_plan_set_alpha); lnl_out: host double[n_trees], lnL at the returned
 * shapes and lengths (the optimiser's objective); rounds_out: host, NULL
 * ok, the number of shape updates.
 * Synchronises `stream` after every step.  EINVAL for bad bounds, a start
 * outside them, tol_alpha <= 0 or max_rounds < 1. */
pt_status pt_plan_optimize_alpha(pt_plan *plan, double *d_brlen_inout, const pt_opt *opt, double *alpha_inout,
                                 double alpha_min, double alpha_max, double tol_alpha, int32_t max_rounds,
                                 double *lnl_out, int32_t *rounds_out, void *stream);

/* Algorithmic device-memory bytes one run of `kind` moves: every partial,
 * scaler, tip code and weight its programs read or write once per use
 * (Newton iterations and transition matrices add none).  For
 * PT_PLAN_OPTIMIZE, passes[n_trees] (host; NULL = 1) gives the passes each
 * tree ran.  Used to express kernel throughput against the memory
 * bandwidth roofline. */
pt_status pt_plan_traffic(const pt_plan *plan, int32_t kind, const int32_t *passes,
                          double *bytes_out);

/* Phase profile of the optimisation kernel: with d_counters (device
 * int64[n_trees][8]) set, every later pt_plan_optimize writes per tree:
 * passes, edge steps, Newton iterations, partial updates, then shader-clock
 * cycles spent in updates, in building eigenbasis tables, in Newton
 * iterations, and in total.  NULL turns it off.  Costs a few clock reads
 * per step; meant for tuning, not for timed runs. */
pt_status pt_plan_set_profile(pt_plan *plan, void *d_counters);

/* Number of trees, total edges and device bytes held by the plan. */
pt_status pt_plan_info(const pt_plan *plan, int32_t *n_trees, int64_t *n_edges,
                       int64_t *device_bytes);

/* ----------------------------------------------------- host-only utilities */

/* Validates a model exactly as pt_aln_create does and returns what the
 * kernels use: cat_rates[n_cats] (category rates, mean 1), and the
 * eigen-decomposition P(t) = U diag(exp(lam t)) Uinv (U, Uinv row-major 4x4,
 * lam[4]).  Any output may be NULL.  No device is touched. */
pt_status pt_model_info(const pt_model *model, double *cat_rates, double *U, double *Uinv,
                        double *lam);

/* Validates an edge list (node ids in range, leaves of degree 1, internal
 * nodes of degree 3, connected) without touching a device. */
pt_status pt_tree_check(int32_t n_taxa, const int32_t *edges);

/* ------------------------------------------------------ host-only topology */

/* The 2(n-3) NNI neighbours (Methods, "Phylogenetic Topographer": the search
 * visits every NNI neighbour of a queued topology).  For internal edge (u,v)
 * taken in edge order, with u's other edges a < b and v's other edges c < d
 * by edge index, neighbour 2i swaps the subtrees on b and c and neighbour
 * 2i+1 swaps b and d.  Lengths stay with their edges.  Outputs:
 * out_edges int32[2(n-3)][2n-3][2], out_brlen double[2(n-3)][2n-3] (brlen
 * may be NULL, then out_brlen is not written), out_touched
 * int32[2(n-3)][5] (central edge, then b, the swapped partner, and the two
 * remaining edges at u and v; NULL ok).  n >= 4. */
pt_status pt_nni_neighbors(int32_t n, const int32_t *edges, const double *brlen,
                           int32_t *out_edges, double *out_brlen, int32_t *out_touched);

/* Canonical topology key: the n-3 non-trivial splits, each the leaf bitmask
 * of the side without taxon 0 in W = (n+63)/64 little-endian uint64 words,
 * sorted ascending (as W-word numbers, most significant word last).
 * out: uint64[n-3][W].  Equal keys <=> equal unrooted topologies.  n >= 4. */
pt_status pt_topology_key(int32_t n, const int32_t *edges, uint64_t *out);
/* The keys of `count` trees on n taxa at once: edges int32[count][2n-3][2],
 * out uint64[count][n-3][W].  On error nothing is guaranteed about out. */
pt_status pt_topology_keys(int32_t n, int32_t count, const int32_t *edges, uint64_t *out);

/* Radius-limited optimisation masks (Methods, "Phylogenetic Topographer":
 * proposals may optimise the lengths within radius r of the new edge).  For
 * tree i, centres[i] is the new edge and u its first endpoint that is an
 * internal node.  The centre edge has depth 0; walking away from the centre
 * edge through u, each edge is one deeper than the edge it is reached from.
 * out[i][e] = 1 for the edges of depth <= radius, else 0: radius 0 is the
 * centre edge alone, radius 1 adds u's two other edges, and radius -1 marks
 * every edge.  edges int32[count][2n-3][2], centres int32[count], out
 * uint8[count][2n-3] (the opt_mask layout).  EINVAL for an invalid tree, a
 * centre out of range or radius < -1; out is then undefined. */
pt_status pt_radius_masks(int32_t n, int32_t count, const int32_t *edges, const int32_t *centres,
                          int32_t radius, uint8_t *out);

/* ---------------------------------------------- high-likelihood set summary */

/* Split frequencies of a high-likelihood set (Results, "Split Frequency
 * Comparison": each topology is weighted by its maximised likelihood,
 * normalised over the set, and a split's frequency is the summed weight of
 * the topologies that contain it):
 *   freq(s) = sum_{i : s in key_i} exp(lnl_i - lmax) / sum_i exp(lnl_i - lmax).
 * keys uint64[count][n-3][W] as written by pt_topology_keys, lnl[count]
 * finite.  Writes the *n_splits distinct splits, uint64[*n_splits][W], and
 * their frequencies, by decreasing frequency (ties: the order of the splits
 * as numbers).  cap is the capacity of splits / freq in splits; count *
 * (n-3) always suffices.  EINVAL (with *n_splits set to the number needed)
 * when cap is too small; EINVAL for count < 1, n < 4, a non-finite lnl or a
 * key holding taxon 0 or a taxon >= n.  Host only. */
pt_status pt_split_frequencies(int32_t n, int32_t count, const uint64_t *keys, const double *lnl, int32_t cap,
                               int32_t *n_splits, uint64_t *splits, double *freq);

/* Majority-rule consensus (Results, "Split Frequency Comparison"): the
 * splits of frequency above 1/2, which are pairwise compatible, as a Newick
 * string rooted at taxon 0.  Leaves are taxon indices; each clade carries its
 * frequency as its label ("%.6f"); children appear in order of their
 * smallest taxon, taxon 0 first at the root.  A star tree when no split
 * passes.  splits / freq as pt_split_frequencies writes them (any order).
 * out char[cap] receives the NUL-terminated string; *len_out is its size
 * with the NUL.  EINVAL when cap is too small (len_out still set), or for a
 * trivial split, one holding taxon 0, a frequency outside [0, 1], or
 * incompatible or repeated splits above 1/2.  Host only. */
pt_status pt_majority_consensus(int32_t n, int32_t n_splits, const uint64_t *splits, const double *freq, char *out,
                                int32_t cap, int32_t *len_out);

/* -------------------------------------------- warm-start network (learned) */

/* Features of every NNI move of a tree whose lengths have been optimised,
 * in pt_nni_neighbors order, PT_NNI_FEATURES floats each: log t of the five
 * edges the move touches (central, b, its swap partner, the remaining edge
 * at u, the remaining edge at v; t floored at 1e-6), log leaf count and
 * log(clade length + 1e-3) of the four subtrees hanging off the last four,
 * and log of the total tree length.  out: float[2(n-3)][PT_NNI_FEATURES].
 * n >= 4.  Host only. */
#define PT_NNI_FEATURES 14
pt_status pt_nni_features(int32_t n, const int32_t *edges, const double *brlen, float *out);

/* A two-layer perceptron y = tanh(x W1 + b1) W2 + b2 in FP32, evaluated and
 * trained (mean squared error, Adam) by the library's own kernels.  It maps
 * the features of an NNI move to the log-ratio of the five touched edges'
 * optimised lengths to the parent's lengths, to warm-start the neighbour's
 * branch optimisation (the search always judges a topology by its fully
 * optimised lnL, so the network only changes where Newton starts).
 * Parameters are packed W1[n_in][n_hidden], b1[n_hidden], W2[n_hidden][n_out],
 * b2[n_out]; `params` (host) gives their initial values.  Device pointers in
 * the calls below are row-major float arrays; work is enqueued on `stream`
 * (NULL = null stream).  A call with more rows than any before grows the
 * network's scratch buffers (an allocation). */
typedef struct pt_mlp pt_mlp;
typedef struct {
    float lr, beta1, beta2, eps;
} pt_adam;
pt_status pt_mlp_create(pt_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params,
                        pt_mlp **out);
void pt_mlp_destroy(pt_mlp *mlp);
/* Number of packed parameters. */
int64_t pt_mlp_param_count(const pt_mlp *mlp);
pt_status pt_mlp_get_params(pt_mlp *mlp, float *params_out);
pt_status pt_mlp_set_params(pt_mlp *mlp, const float *params);
/* d_y[rows][n_out] = network(d_x[rows][n_in]). */
pt_status pt_mlp_forward(pt_mlp *mlp, const float *d_x, int32_t rows, float *d_y, void *stream);
/* Gradient of the mean over rows and outputs of (y - target)^2 with respect
 * to the packed parameters (d_grad, device float[param_count]); d_loss
 * (device double, NULL ok) receives the sum of squared errors. */
pt_status pt_mlp_gradient(pt_mlp *mlp, const float *d_x, const float *d_target, int32_t rows, float *d_grad,
                          double *d_loss, void *stream);
/* Warm start of NNI neighbours: y = network(d_x) as above, then for every
 * row r and output o with d_pos[r][o] >= 0,
 *   d_brlen[d_pos[r][o]] = clamp((max(d_base[r][o], 0) + shift) * exp(y[r][o]) - shift, t_min, t_max),
 * i.e. the outputs are log-ratios of shifted lengths of a neighbour and its
 * parent (shift > 0 keeps lengths near zero from dominating).  d_pos: device
 * int32[rows][n_out], indices into d_brlen (distinct and in range: the
 * caller's responsibility); d_base: device double[rows][n_out]. */
pt_status pt_mlp_warm_start(pt_mlp *mlp, const float *d_x, int32_t rows, const int32_t *d_pos, const double *d_base,
                            double shift, double t_min, double t_max, double *d_brlen, void *stream);
/* One Adam step on that loss. */
pt_status pt_mlp_train_step(pt_mlp *mlp, const float *d_x, const float *d_target, int32_t rows,
                            const pt_adam *opt, double *d_loss, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PT_H */
