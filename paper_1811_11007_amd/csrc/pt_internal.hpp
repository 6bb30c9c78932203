// pt_internal.hpp -- host-side internals of the library.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "pt.h"
#include "pt_device.hpp"

namespace pt {

// ----------------------------------------------------------------- model
pt_status build_model(const pt_model &m, AlnDev &d, std::string &err);
pt_status gamma_category_rates(double alpha, int K, double *out, std::string &err);

// ------------------------------------------------------------------ trees
struct Tree {
    int n = 0, n_nodes = 0, n_edges = 0;
    std::vector<int32_t> ends;   // [E][2]
    std::vector<int> nbr;        // [n_nodes][3]
    std::vector<int> nedge;      // [n_nodes][3]
    std::vector<int> deg;        // [n_nodes]
    int n_slots() const { return n >= 3 ? 3 * (n - 2) : 0; }
};

// Validates an edge list: node ids in range, leaves of degree 1, internal
// nodes of degree 3, connected.
pt_status build_tree(int n, const int32_t *edges, Tree &t, std::string &err);

// Programs (sequences of Op) executed by the kernels, one per tree.
// lnL across one edge: the n-2 updates that make both sides valid, then EVAL.
void compile_loglik(const Tree &t, std::vector<Op> &ops);
// The same with the n-2 slots it uses renumbered 0..n-3, so the program fits
// in two thirds of a tree's partial buffer at twice the element size (the
// FP64 evaluation that ends an FP32 optimisation reuses the FP32 buffer).
void compile_loglik_dense(const Tree &t, std::vector<Op> &ops);
// lnL as a register program (OP_RUPDATE / OP_RPUSH / OP_REVAL, rooted on
// edge 0); returns the stack slots it needs.
int compile_loglik_reg(const Tree &t, std::vector<Op> &ops);
// Every directional partial once, then EVAL on every edge (column = edge).
void compile_grad(const Tree &t, std::vector<Op> &ops);
// Smoothing passes over the masked edges in depth-first edge order: before
// each edge step, exactly the partial updates whose inputs changed.  `first`
// starts from no valid partial; `steady` is every later pass.
void compile_optimize(const Tree &t, const uint8_t *mask, std::vector<Op> &first,
                      std::vector<Op> &steady);

// --------------------------------------------------------------- topology
pt_status nni_neighbors(int n, const int32_t *edges, const double *brlen, int32_t *out_edges,
                        double *out_brlen, int32_t *out_touched, std::string &err);
pt_status topology_key(int n, const int32_t *edges, uint64_t *out, std::string &err);
pt_status nni_features(int n, const int32_t *edges, const double *brlen, float *out, std::string &err);
pt_status radius_mask(int n, const int32_t *edges, int centre, int r, uint8_t *out, std::string &err);

// ------------------------------------------------------------ HLS summaries
pt_status split_frequencies(int n, int count, const uint64_t *keys, const double *lnl, int cap, int32_t *n_out,
                            uint64_t *splits, double *freq, std::string &err);
pt_status majority_consensus(int n, int count, const uint64_t *splits, const double *freq, char *out, int cap,
                             int32_t *len_out, std::string &err);

}  // namespace pt
