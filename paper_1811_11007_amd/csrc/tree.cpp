// tree.cpp -- tree validation, per-tree kernel programs and host topology ops.
//
// Directional partials.  For internal node v and its neighbour u, slot
// (v, u) holds the partial likelihood of v's side of edge (v, u), at v:
// the product over v's two other neighbours c of P(t_vc) times the partial of
// c's side.  With every slot valid, lnL and the derivatives across any edge
// (u, v) follow from slots (u, v) and (v, u) alone (re-rooting on an edge,
// the pulley principle), which is what the edge steps of coordinate-wise
// branch optimisation need.  The compiler simulates which slots a length
// change invalidates and emits exactly the updates each step needs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "pt_internal.hpp"

namespace pt {

pt_status build_tree(int n, const int32_t *edges, Tree &t, std::string &err) {
    if (n < 2) { err = "a tree needs at least 2 taxa"; return PT_EINVAL; }
    t.n = n;
    t.n_nodes = n == 2 ? 2 : 2 * n - 2;
    t.n_edges = n == 2 ? 1 : 2 * n - 3;
    t.ends.assign(edges, edges + 2 * t.n_edges);
    t.nbr.assign(3 * t.n_nodes, -1);
    t.nedge.assign(3 * t.n_nodes, -1);
    t.deg.assign(t.n_nodes, 0);
    for (int e = 0; e < t.n_edges; ++e) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= t.n_nodes || b >= t.n_nodes) {
            err = "edge " + std::to_string(e) + ": node id out of range";
            return PT_EINVAL;
        }
        if (a == b) { err = "edge " + std::to_string(e) + " is a self-loop"; return PT_EINVAL; }
        if (t.deg[a] >= 3 || t.deg[b] >= 3) {
            err = "node of degree > 3 at edge " + std::to_string(e);
            return PT_EINVAL;
        }
        t.nbr[3 * a + t.deg[a]] = b; t.nedge[3 * a + t.deg[a]++] = e;
        t.nbr[3 * b + t.deg[b]] = a; t.nedge[3 * b + t.deg[b]++] = e;
    }
    for (int v = 0; v < t.n_nodes; ++v) {
        int want = v < n ? 1 : 3;
        if (t.deg[v] != want) {
            err = "node " + std::to_string(v) + " has degree " + std::to_string(t.deg[v]) +
                  ", expected " + std::to_string(want);
            return PT_EINVAL;
        }
    }
    std::vector<char> seen(t.n_nodes, 0);
    std::vector<int> stack{0};
    seen[0] = 1;
    int count = 0;
    while (!stack.empty()) {
        int v = stack.back();
        stack.pop_back();
        ++count;
        for (int j = 0; j < t.deg[v]; ++j)
            if (!seen[t.nbr[3 * v + j]]) { seen[t.nbr[3 * v + j]] = 1; stack.push_back(t.nbr[3 * v + j]); }
    }
    if (count != t.n_nodes) { err = "edge list is not connected (contains a cycle)"; return PT_EINVAL; }
    return PT_OK;
}

namespace {

// Slot bookkeeping shared by the three compilers.
struct Slots {
    const Tree &t;
    std::vector<uint8_t> valid;
    std::vector<std::vector<uint64_t>> deps;  // per slot: bitset of edges inside
    int words;
    std::vector<Op> *out = nullptr;
    int updates = 0;

    explicit Slots(const Tree &tree) : t(tree), valid(tree.n_slots(), 0) {
        words = (t.n_edges + 63) / 64;
        deps.assign(t.n_slots(), std::vector<uint64_t>(words, 0));
        std::vector<uint8_t> done(t.n_slots(), 0);
        std::function<void(int)> fill = [&](int s) {
            if (done[s]) return;
            int v = s / 3 + t.n, j = s % 3;
            for (int q = 0; q < 3; ++q) {
                if (q == j) continue;
                int c = t.nbr[3 * v + q], e = t.nedge[3 * v + q];
                deps[s][e / 64] |= 1ull << (e % 64);
                int r = ref(c, v);
                if (r >= 0) {
                    fill(r);
                    for (int w = 0; w < words; ++w) deps[s][w] |= deps[r][w];
                }
            }
            done[s] = 1;
        };
        for (int s = 0; s < t.n_slots(); ++s) fill(s);
    }
    // side of node v facing neighbour u: tip -(v+1) or slot index
    int ref(int v, int u) const {
        if (v < t.n) return -(v + 1);
        for (int j = 0; j < 3; ++j)
            if (t.nbr[3 * v + j] == u) return (v - t.n) * 3 + j;
        return INT32_MIN;
    }
    void ensure(int r) {
        if (r < 0 || valid[r]) return;
        int v = r / 3 + t.n, j = r % 3;
        int q0 = -1, q1 = -1;
        for (int q = 0; q < 3; ++q) {
            if (q == j) continue;
            (q0 < 0 ? q0 : q1) = q;
        }
        int c0 = t.nbr[3 * v + q0], c1 = t.nbr[3 * v + q1];
        int ra = ref(c0, v), rb = ref(c1, v);
        ensure(ra);
        ensure(rb);
        Op op{};
        op.code = OP_UPDATE;
        op.dst = r;
        op.a = ra; op.ea = t.nedge[3 * v + q0];
        op.b = rb; op.eb = t.nedge[3 * v + q1];
        out->push_back(op);
        ++updates;
        valid[r] = 1;
    }
    void touch(int e) {
        for (int s = 0; s < t.n_slots(); ++s)
            if (deps[s][e / 64] >> (e % 64) & 1) valid[s] = 0;
    }
};

Op edge_op(int code, int e, int a, int b, int col) {
    Op op{};
    op.code = code;
    op.dst = e;
    op.a = a;
    op.b = b;
    op.ea = col;
    return op;
}

}  // namespace

void compile_loglik(const Tree &t, std::vector<Op> &ops) {
    Slots s(t);
    s.out = &ops;
    int u = t.ends[0], v = t.ends[1];
    int ra = s.ref(u, v), rb = s.ref(v, u);
    s.ensure(ra);
    s.ensure(rb);
    ops.push_back(edge_op(OP_EVAL, 0, ra, rb, 0));
}

void compile_loglik_dense(const Tree &t, std::vector<Op> &ops) {
    std::vector<Op> p;
    compile_loglik(t, p);
    std::vector<int> id(t.n_slots(), -1);
    int next = 0;
    auto map = [&](int r) { return r < 0 ? r : id[r]; };
    for (Op op : p) {
        if (op.code == OP_UPDATE) {
            op.a = map(op.a);
            op.b = map(op.b);
            id[op.dst] = next++;
            op.dst = id[op.dst];
        } else {
            op.a = map(op.a);
            op.b = map(op.b);
        }
        ops.push_back(op);
    }
}

// Register program of the lnL: Felsenstein's post-order pass rooted on edge
// 0, written for a machine whose only partials are an accumulator and a
// small stack.  Of an internal node's two child subtrees, the one needing
// more stack is evaluated first (Sethi and Ullman 1970), so a tree of n taxa
// needs at most floor(log2 n) - 1 stack slots.  Side references: >= 0 a
// leaf's tip, REF_ACC the accumulator, <= REF_STACK0 stack slot
// REF_STACK0 - ref.  Every OP_RUPDATE and OP_REVAL has one of three side
// forms, (tip, tip), (accumulator, tip) or (stack slot, accumulator), which
// the kernel relies on.
int compile_loglik_reg(const Tree &t, std::vector<Op> &ops) {
    const int n = t.n;
    auto child_pair = [&](int v, int parent, int c[2], int e[2]) {
        int k = 0;
        for (int j = 0; j < 3; ++j)
            if (t.nbr[3 * v + j] != parent) { c[k] = t.nbr[3 * v + j]; e[k] = t.nedge[3 * v + j]; ++k; }
    };
    std::function<int(int, int)> need = [&](int v, int parent) -> int {
        if (v < n) return 0;
        int c[2], e[2];
        child_pair(v, parent, c, e);
        const int a = need(c[0], v), b = need(c[1], v);
        return a == b ? a + 1 : std::max(a, b);
    };
    int depth = 0;
    auto emit_op = [&](int code, int dst, int a, int ea, int b, int eb) {
        Op op{};
        op.code = code;
        op.dst = dst;
        op.a = a;
        op.ea = ea;
        op.b = b;
        op.eb = eb;
        ops.push_back(op);
    };
    // Leaves the partial of v's side (seen from parent) in the accumulator,
    // using stack slots from sp up.
    std::function<void(int, int, int)> emit = [&](int v, int parent, int sp) {
        int c[2], e[2];
        child_pair(v, parent, c, e);
        if (need(c[1], v) > need(c[0], v)) { std::swap(c[0], c[1]); std::swap(e[0], e[1]); }
        if (c[0] < n) {  // two tips
            emit_op(OP_RUPDATE, 0, c[0], e[0], c[1], e[1]);
        } else if (c[1] < n) {
            emit(c[0], v, sp);
            emit_op(OP_RUPDATE, 0, REF_ACC, e[0], c[1], e[1]);
        } else {
            emit(c[0], v, sp);
            emit_op(OP_RPUSH, sp, 0, 0, 0, 0);
            depth = std::max(depth, sp + 1);
            emit(c[1], v, sp + 1);
            emit_op(OP_RUPDATE, 0, REF_STACK0 - sp, e[0], REF_ACC, e[1]);
        }
    };
    int u = t.ends[0], v = t.ends[1];
    if (need(v, u) > need(u, v)) std::swap(u, v);  // u's side first
    if (u < n) {  // two tips (n = 2)
        emit_op(OP_REVAL, 0, u, -1, v, 0);
    } else if (v < n) {
        emit(u, v, 0);
        emit_op(OP_REVAL, 0, REF_ACC, -1, v, 0);
    } else {
        emit(u, v, 0);
        emit_op(OP_RPUSH, 0, 0, 0, 0, 0);
        depth = std::max(depth, 1);
        emit(v, u, 1);
        emit_op(OP_REVAL, 0, REF_STACK0, -1, REF_ACC, 0);
    }
    return depth;
}

void compile_grad(const Tree &t, std::vector<Op> &ops) {
    Slots s(t);
    s.out = &ops;
    for (int e = 0; e < t.n_edges; ++e) {
        int u = t.ends[2 * e], v = t.ends[2 * e + 1];
        int ra = s.ref(u, v), rb = s.ref(v, u);
        s.ensure(ra);
        s.ensure(rb);
        ops.push_back(edge_op(OP_EVAL, e, ra, rb, e));
    }
}

void compile_optimize(const Tree &t, const uint8_t *mask, std::vector<Op> &first,
                      std::vector<Op> &steady) {
    // depth-first edge order from the edge of leaf 0
    std::vector<int> order;
    std::function<void(int, int)> visit = [&](int x, int y) {
        for (int j = 0; j < t.deg[y]; ++j) {
            int z = t.nbr[3 * y + j];
            if (z == x) continue;
            order.push_back(t.nedge[3 * y + j]);
            visit(y, z);
        }
    };
    order.push_back(t.nedge[0]);
    visit(0, t.nbr[0]);
    if (t.n == 2) order.assign(1, 0);

    Slots s(t);
    auto pass = [&](std::vector<Op> &ops) {
        s.out = &ops;
        for (int e : order) {
            if (mask && !mask[e]) continue;
            int u = t.ends[2 * e], v = t.ends[2 * e + 1];
            int ra = s.ref(u, v), rb = s.ref(v, u);
            s.ensure(ra);
            s.ensure(rb);
            ops.push_back(edge_op(OP_NEWTON, e, ra, rb, 0));
            s.touch(e);
        }
        // the last edge step of a pass also reports the tree's lnL
        if (!ops.empty()) ops.back().ea = 1;
    };
    pass(first);
    // The validity pattern after a pass is the same for every pass that
    // starts from it; iterate until the emitted program repeats.
    std::vector<Op> prev;
    pass(steady);
    for (int guard = 0; guard < 8; ++guard) {
        std::vector<Op> again;
        pass(again);
        if (again.size() == steady.size() &&
            std::memcmp(again.data(), steady.data(), again.size() * sizeof(Op)) == 0)
            break;
        steady.swap(again);
    }
}

// ------------------------------------------------------------- topology

pt_status nni_neighbors(int n, const int32_t *edges, const double *brlen, int32_t *out_edges,
                        double *out_brlen, int32_t *out_touched, std::string &err) {
    if (n < 4) { err = "NNI needs n >= 4"; return PT_EINVAL; }
    Tree t;
    pt_status st = build_tree(n, edges, t, err);
    if (st) return st;
    const int E = t.n_edges;
    int k = 0;
    for (int e = 0; e < E; ++e) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < n || v < n) continue;
        int eu[2], ev[2], iu = 0, iv = 0;
        for (int j = 0; j < 3; ++j) {
            if (t.nedge[3 * u + j] != e) eu[iu++] = t.nedge[3 * u + j];
            if (t.nedge[3 * v + j] != e) ev[iv++] = t.nedge[3 * v + j];
        }
        std::sort(eu, eu + 2);
        std::sort(ev, ev + 2);
        for (int w = 0; w < 2; ++w, ++k) {
            int32_t *o = out_edges + (size_t)k * 2 * E;
            std::memcpy(o, edges, sizeof(int32_t) * 2 * E);
            int eb = eu[1], ec = ev[w];
            for (int x = 0; x < 2; ++x) {
                if (o[2 * eb + x] == u) o[2 * eb + x] = v;
                if (o[2 * ec + x] == v) o[2 * ec + x] = u;
            }
            if (out_brlen && brlen) std::memcpy(out_brlen + (size_t)k * E, brlen, sizeof(double) * E);
            if (out_touched) {
                int32_t *tt = out_touched + (size_t)k * 5;
                tt[0] = e; tt[1] = eb; tt[2] = ec; tt[3] = eu[0]; tt[4] = ev[1 - w];
            }
        }
    }
    return PT_OK;
}

// Radius-limited optimisation mask (Methods, "Phylogenetic Topographer",
// the radius option): the centre edge has depth 0; from the selected
// endpoint u of the centre edge (its first endpoint that is an internal
// node), each further edge reached through u is one deeper than the edge it
// is reached from.  Edges of depth <= r are marked; r = -1 marks all.  The
// walk never crosses the centre edge, so r = 1 gives the centre edge and
// u's two other edges.
pt_status radius_mask(int n, const int32_t *edges, int centre, int r, uint8_t *out, std::string &err) {
    Tree t;
    pt_status st = build_tree(n, edges, t, err);
    if (st) return st;
    const int E = t.n_edges;
    if (centre < 0 || centre >= E) { err = "centre edge out of range"; return PT_EINVAL; }
    if (r < -1) { err = "radius must be >= -1"; return PT_EINVAL; }
    if (r == -1) {
        std::fill(out, out + E, (uint8_t)1);
        return PT_OK;
    }
    std::fill(out, out + E, (uint8_t)0);
    out[centre] = 1;
    int u = edges[2 * centre];
    if (u < n) u = edges[2 * centre + 1];
    if (u < n || r == 0) return PT_OK;
    // frontier of (node, edge it was entered by, depth of that edge)
    struct Item { int node, via, depth; };
    std::vector<Item> todo{{u, centre, 0}};
    while (!todo.empty()) {
        const Item it = todo.back();
        todo.pop_back();
        if (it.node < n || it.depth == r) continue;
        for (int j = 0; j < 3; ++j) {
            const int f = t.nedge[3 * it.node + j];
            if (f == it.via) continue;
            out[f] = 1;
            todo.push_back({t.nbr[3 * it.node + j], f, it.depth + 1});
        }
    }
    return PT_OK;
}

namespace {

// Leaf count and total edge length of the subtree hanging from `node` away
// from `from`.
void clade(const Tree &t, const double *brlen, int node, int from, int &leaves, double &len) {
    if (node < t.n) {
        leaves += 1;
        return;
    }
    for (int j = 0; j < 3; ++j) {
        const int c = t.nbr[3 * node + j];
        if (c == from) continue;
        len += brlen[t.nedge[3 * node + j]];
        clade(t, brlen, c, node, leaves, len);
    }
}

}  // namespace

pt_status nni_features(int n, const int32_t *edges, const double *brlen, float *out, std::string &err) {
    if (n < 4) { err = "NNI needs n >= 4"; return PT_EINVAL; }
    Tree t;
    pt_status st = build_tree(n, edges, t, err);
    if (st) return st;
    const int E = t.n_edges;
    std::vector<int32_t> ne((size_t)2 * (n - 3) * 2 * E);
    std::vector<int32_t> touched((size_t)2 * (n - 3) * 5);
    st = nni_neighbors(n, edges, nullptr, ne.data(), nullptr, touched.data(), err);
    if (st) return st;
    double total = 0.0;
    for (int e = 0; e < E; ++e) total += brlen[e];
    auto lt = [](double x) { return (float)std::log(std::max(x, 1e-6)); };
    for (int k = 0; k < 2 * (n - 3); ++k) {
        const int32_t *tt = touched.data() + (size_t)k * 5;
        float *f = out + (size_t)k * 14;
        const int ce = tt[0];
        const int u = edges[2 * ce], v = edges[2 * ce + 1];
        for (int q = 0; q < 5; ++q) f[q] = lt(brlen[tt[q]]);
        for (int q = 1; q < 5; ++q) {
            // the end of edge tt[q] away from the central edge
            const int x0 = edges[2 * tt[q]], x1 = edges[2 * tt[q] + 1];
            const int near = (x0 == u || x0 == v) ? x0 : x1;
            const int far = near == x0 ? x1 : x0;
            int leaves = 0;
            double len = 0.0;
            clade(t, brlen, far, near, leaves, len);
            f[4 + q] = (float)std::log((double)leaves);
            f[8 + q] = (float)std::log(len + 1e-3);
        }
        f[13] = (float)std::log(total);
    }
    return PT_OK;
}

pt_status topology_key(int n, const int32_t *edges, uint64_t *out, std::string &err) {
    if (n < 4) { err = "topology keys need n >= 4"; return PT_EINVAL; }
    Tree t;
    pt_status st = build_tree(n, edges, t, err);
    if (st) return st;
    const int W = (n + 63) / 64;
    // iterative depth-first order from leaf 0, then leaf sets bottom-up
    // (flat arrays: one allocation each)
    std::vector<uint64_t> below((size_t)t.n_nodes * W, 0);
    std::vector<int> parent(t.n_nodes, -1), order, stack;
    order.reserve(t.n_nodes);
    stack.reserve(t.n_nodes);
    stack.push_back(0);
    parent[0] = 0;
    while (!stack.empty()) {
        int v = stack.back();
        stack.pop_back();
        order.push_back(v);
        for (int j = 0; j < t.deg[v]; ++j) {
            int c = t.nbr[3 * v + j];
            if (parent[c] < 0 && c != 0) { parent[c] = v; stack.push_back(c); }
        }
    }
    std::vector<uint64_t> splits;
    splits.reserve((size_t)(n - 3) * W);
    for (int i = (int)order.size() - 1; i >= 1; --i) {
        const int v = order[i];
        uint64_t *bv = below.data() + (size_t)v * W;
        if (v < n) bv[v / 64] |= 1ull << (v % 64);
        int cnt = 0;
        for (int w = 0; w < W; ++w) cnt += __builtin_popcountll(bv[w]);
        if (cnt >= 2 && cnt <= n - 2) splits.insert(splits.end(), bv, bv + W);
        uint64_t *bp = below.data() + (size_t)parent[v] * W;
        for (int w = 0; w < W; ++w) bp[w] |= bv[w];
    }
    if ((int)(splits.size() / W) != n - 3) { err = "internal error: split count"; return PT_EINTERNAL; }
    if (W == 1) {
        std::sort(splits.begin(), splits.end());
        std::copy(splits.begin(), splits.end(), out);
        return PT_OK;
    }
    std::vector<int> idx(n - 3);
    for (int i = 0; i < n - 3; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) {
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t a = splits[(size_t)x * W + w], b = splits[(size_t)y * W + w];
            if (a != b) return a < b;
        }
        return false;
    });
    for (int i = 0; i < n - 3; ++i)
        for (int w = 0; w < W; ++w) out[(size_t)i * W + w] = splits[(size_t)idx[i] * W + w];
    return PT_OK;
}

}  // namespace pt
