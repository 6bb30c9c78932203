// hls.cpp -- summaries of a high-likelihood set (host only).
//
// Split frequencies weight each topology of the set by its maximised
// likelihood, normalised over the set, and give every split the summed weight
// of the topologies that contain it (Results, "Split Frequency Comparison").
// The majority-rule consensus keeps the splits of frequency above 1/2.
//
// A split is the leaf bitmask of the side without taxon 0 (W = (n+63)/64
// little-endian words, as in topology keys), which makes it a clade of the
// tree rooted at leaf 0: two splits are compatible exactly when their
// clades are disjoint or nested.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>

#include "pt_internal.hpp"

namespace pt {

namespace {

// Most significant word last, as in topology keys.
bool split_less(const uint64_t *a, const uint64_t *b, int W) {
    for (int w = W - 1; w >= 0; --w)
        if (a[w] != b[w]) return a[w] < b[w];
    return false;
}

int split_bits(const uint64_t *a, int W) {
    int c = 0;
    for (int w = 0; w < W; ++w) c += __builtin_popcountll(a[w]);
    return c;
}

}  // namespace

pt_status split_frequencies(int n, int count, const uint64_t *keys, const double *lnl, int cap, int32_t *n_out,
                            uint64_t *splits, double *freq, std::string &err) {
    if (n < 4) { err = "split frequencies need n >= 4"; return PT_EINVAL; }
    if (count < 1) { err = "need at least one topology"; return PT_EINVAL; }
    const int W = (n + 63) / 64, S = n - 3;
    double lmax = -INFINITY;
    for (int i = 0; i < count; ++i) {
        if (!std::isfinite(lnl[i])) { err = "lnl[" + std::to_string(i) + "] is not finite"; return PT_EINVAL; }
        lmax = std::max(lmax, lnl[i]);
    }
    // every occurrence (topology i, split j), sorted by split then topology,
    // so that each split's weights are summed in topology order
    std::vector<int64_t> occ((size_t)count * S);
    for (size_t x = 0; x < occ.size(); ++x) occ[x] = (int64_t)x;
    const uint64_t last_mask = (n % 64) ? (1ull << (n % 64)) - 1 : ~0ull;
    for (size_t x = 0; x < occ.size(); ++x) {
        const uint64_t *s = keys + x * W;
        if ((s[0] & 1ull) || (s[W - 1] & ~last_mask)) {
            err = "key of topology " + std::to_string(x / S) + " holds taxon 0 or a taxon >= n";
            return PT_EINVAL;
        }
    }
    std::stable_sort(occ.begin(), occ.end(),
                     [&](int64_t a, int64_t b) { return split_less(keys + a * W, keys + b * W, W); });
    std::vector<double> wt(count);
    double z = 0.0;
    for (int i = 0; i < count; ++i) {
        wt[i] = std::exp(lnl[i] - lmax);
        z += wt[i];
    }
    std::vector<int64_t> first;  // occurrence index of each distinct split
    std::vector<double> acc;
    for (size_t x = 0; x < occ.size(); ++x) {
        const uint64_t *s = keys + occ[x] * W;
        if (first.empty() || split_less(keys + first.back() * W, s, W)) {
            first.push_back(occ[x]);
            acc.push_back(0.0);
        }
        acc.back() += wt[occ[x] / S];
    }
    const int m = (int)first.size();
    *n_out = m;
    if (m > cap) {
        err = "capacity " + std::to_string(cap) + " is below the " + std::to_string(m) + " distinct splits";
        return PT_EINVAL;
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return acc[a] > acc[b]; });
    for (int r = 0; r < m; ++r) {
        std::memcpy(splits + (size_t)r * W, keys + first[idx[r]] * W, sizeof(uint64_t) * W);
        freq[r] = acc[idx[r]] / z;
    }
    return PT_OK;
}

pt_status majority_consensus(int n, int count, const uint64_t *splits, const double *freq, char *out, int cap,
                             int32_t *len_out, std::string &err) {
    if (n < 2) { err = "need n >= 2"; return PT_EINVAL; }
    const int W = (n + 63) / 64;
    const uint64_t last_mask = (n % 64) ? (1ull << (n % 64)) - 1 : ~0ull;
    std::vector<int> sel;
    for (int i = 0; i < count; ++i) {
        if (!(freq[i] >= 0.0 && freq[i] <= 1.0 + 1e-9)) { err = "freq out of [0, 1]"; return PT_EINVAL; }
        const uint64_t *s = splits + (size_t)i * W;
        const int b = split_bits(s, W);
        if ((s[0] & 1ull) || (s[W - 1] & ~last_mask) || b < 2 || b > n - 2) {
            err = "split " + std::to_string(i) + " is not a non-trivial split without taxon 0";
            return PT_EINVAL;
        }
        if (freq[i] > 0.5) sel.push_back(i);
    }
    // larger clades first; parents are the smallest enclosing clade
    std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) {
        return split_bits(splits + (size_t)a * W, W) > split_bits(splits + (size_t)b * W, W);
    });
    const int m = (int)sel.size();
    auto inside = [&](int a, int b) {  // clade a within clade b
        const uint64_t *x = splits + (size_t)sel[a] * W, *y = splits + (size_t)sel[b] * W;
        for (int w = 0; w < W; ++w)
            if (x[w] & ~y[w]) return false;
        return true;
    };
    std::vector<int> parent(m, -1);
    for (int a = 0; a < m; ++a) {
        for (int b = a - 1; b >= 0; --b) {  // smallest enclosing clade is the latest larger one
            const uint64_t *x = splits + (size_t)sel[a] * W, *y = splits + (size_t)sel[b] * W;
            bool disjoint = true;
            for (int w = 0; w < W; ++w) disjoint = disjoint && !(x[w] & y[w]);
            if (disjoint) continue;
            if (!inside(a, b) || std::memcmp(x, y, sizeof(uint64_t) * W) == 0) {
                err = "splits above 1/2 are incompatible or repeated";
                return PT_EINVAL;
            }
            if (parent[a] < 0) parent[a] = b;
        }
    }
    // leaf parents: the smallest clade holding the leaf, the first found
    // from the small end (-1: the root)
    std::vector<int> leaf_parent(n, -1);
    for (int leaf = 1; leaf < n; ++leaf)
        for (int a = m - 1; a >= 0; --a)
            if ((splits[(size_t)sel[a] * W + leaf / 64] >> (leaf % 64)) & 1ull) {
                leaf_parent[leaf] = a;
                break;
            }
    // children in order of their smallest leaf
    std::vector<int> min_leaf(m, n);
    for (int leaf = n - 1; leaf >= 1; --leaf)
        for (int a = leaf_parent[leaf]; a >= 0; a = parent[a]) min_leaf[a] = std::min(min_leaf[a], leaf);
    std::vector<std::vector<std::pair<int, int>>> kids(m + 1);  // (min leaf, node: >= 0 clade, < 0 leaf ~x)
    for (int leaf = 1; leaf < n; ++leaf) kids[leaf_parent[leaf] + 1].push_back({leaf, ~leaf});
    for (int a = 0; a < m; ++a) kids[parent[a] + 1].push_back({min_leaf[a], a});
    for (auto &k : kids) std::sort(k.begin(), k.end());
    std::string s = "(0";
    std::function<void(int)> emit = [&](int a) {
        s += "(";
        bool firstk = true;
        for (const auto &k : kids[a + 1]) {
            if (!firstk) s += ",";
            firstk = false;
            if (k.second < 0) s += std::to_string(~k.second);
            else emit(k.second);
        }
        char lab[32];
        std::snprintf(lab, sizeof lab, ")%.6f", freq[sel[a]]);
        s += lab;
    };
    for (const auto &k : kids[0]) {
        s += ",";
        if (k.second < 0) s += std::to_string(~k.second);
        else emit(k.second);
    }
    s += ");";
    *len_out = (int32_t)s.size() + 1;
    if ((int)s.size() + 1 > cap) {
        err = "output capacity " + std::to_string(cap) + " is below " + std::to_string(s.size() + 1) + " bytes";
        return PT_EINVAL;
    }
    std::memcpy(out, s.c_str(), s.size() + 1);
    return PT_OK;
}

}  // namespace pt
