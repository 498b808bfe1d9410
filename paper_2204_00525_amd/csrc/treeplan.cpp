// Join-tree selection (the experiments section, "Effect of join trees": the
// method is fastest on the join tree whose intermediate results are
// smallest, which for key/foreign-key schemas keeps the large fact table away
// from the root so its join attributes are aggregated away early).
//
// The candidates are every join tree of the relations (a spanning tree over
// pairs of relations, in which the relations holding any one attribute stay
// connected: the running intersection property) with every choice of root.
// Each is scored by the work of the register-tile QR that dominates this
// library's forward pass, the sum over the blocks of R0 of rows x columns^2:
//   relation i contributes (m_i - G_i) n_i^2          (tails of heads_and_tails)
//                        + (G_i - P_i) nsub_i^2      (tails of project_away, non-root)
//   the root contributes G_root n^2                  (its joined heads)
// with m_i the rows, G_i the distinct values of all its join attributes, P_i
// the distinct values of the attributes it shares with its parent, n_i its
// columns, nsub_i the columns of its subtree and n the total.  Only P_i and
// nsub_i depend on the tree.  The distinct counts are exact (open addressing
// over the key tuples); dangling tuples are not removed first, so the score
// is an estimate for databases that are not fully reduced.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

namespace figaro {
extern thread_local std::string g_thread_error;
}  // namespace figaro

using namespace figaro;

namespace {

constexpr int kMaxTreeRelations = 12;
constexpr int64_t kMaxTrees = 1 << 20;

figaro_status fail(figaro_status st, const std::string &msg) {
    g_thread_error = msg;
    return st;
}

uint64_t mix64(uint64_t x) {   // splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

struct Schema {
    int r = 0;
    std::vector<int64_t> m;
    std::vector<int32_t> ncols;
    std::vector<std::vector<int32_t>> attrs;             // per relation, as given
    std::vector<std::vector<std::vector<int64_t>>> keys; // per relation [k][m]
    std::map<std::pair<int, std::vector<int32_t>>, int64_t> distinct_memo;

    int key_pos(int i, int32_t a) const {
        for (size_t q = 0; q < attrs[i].size(); ++q)
            if (attrs[i][q] == a) return (int)q;
        return -1;
    }
    std::vector<int32_t> shared(int i, int j) const {
        std::vector<int32_t> out;
        for (int32_t a : attrs[i])
            if (key_pos(j, a) >= 0) out.push_back(a);
        std::sort(out.begin(), out.end());
        return out;
    }
    // distinct value tuples of the attributes `as` of relation i
    int64_t distinct(int i, const std::vector<int32_t> &as) {
        auto key = std::make_pair(i, as);
        auto it = distinct_memo.find(key);
        if (it != distinct_memo.end()) return it->second;
        const int64_t rows = m[i];
        int64_t count = 0;
        if (rows > 0 && as.empty()) {
            count = 1;
        } else if (rows > 0) {
            std::vector<const int64_t *> cols;
            for (int32_t a : as) cols.push_back(keys[i][key_pos(i, a)].data());
            size_t cap = 16;
            while (cap < 2 * (size_t)rows) cap <<= 1;
            std::vector<int64_t> slot(cap, -1);
            for (int64_t t = 0; t < rows; ++t) {
                uint64_t h = 0x9e3779b97f4a7c15ull;
                for (const int64_t *c : cols) h = mix64(h ^ mix64((uint64_t)c[t]));
                size_t s = (size_t)h & (cap - 1);
                for (;;) {
                    const int64_t u = slot[s];
                    if (u < 0) {
                        slot[s] = t;
                        ++count;
                        break;
                    }
                    bool eq = true;
                    for (const int64_t *c : cols)
                        if (c[u] != c[t]) {
                            eq = false;
                            break;
                        }
                    if (eq) break;
                    s = (s + 1) & (cap - 1);
                }
            }
        }
        distinct_memo.emplace(key, count);
        return count;
    }
};

figaro_status load_schema(Schema &S, int32_t r, const figaro_relation_desc *rels, int32_t keys_on_host,
                          hipStream_t stream) {
    if (r < 1 || r > kMaxTreeRelations || !rels)
        return fail(FIGARO_EINVAL, "relation count must be between 1 and 12");
    S.r = r;
    S.m.resize(r);
    S.ncols.resize(r);
    S.attrs.resize(r);
    S.keys.resize(r);
    for (int i = 0; i < r; ++i) {
        const auto &d = rels[i];
        if (d.rows < 0 || d.num_cols < 1 || d.num_keys < 0 || d.num_keys > 32)
            return fail(FIGARO_EINVAL, "relation " + std::to_string(i) + ": bad size");
        if (d.num_keys > 0 && (!d.key_attr || (!d.key_cols && d.rows > 0) || (d.key_dtype != 4 && d.key_dtype != 8)))
            return fail(FIGARO_EINVAL, "relation " + std::to_string(i) + ": bad key arguments");
        S.m[i] = d.rows;
        S.ncols[i] = d.num_cols;
        S.attrs[i].assign(d.key_attr, d.key_attr + d.num_keys);
        std::vector<int32_t> sorted = S.attrs[i];
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(FIGARO_EINVAL, "relation " + std::to_string(i) + ": repeated attribute");
        const size_t elem = (size_t)d.key_dtype, total = (size_t)d.num_keys * (size_t)d.rows;
        std::vector<char> raw(total * elem);
        if (total > 0) {
            if (keys_on_host) {
                std::memcpy(raw.data(), d.key_cols, raw.size());
            } else if (hipMemcpyAsync(raw.data(), d.key_cols, raw.size(), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                       hipStreamSynchronize(stream) != hipSuccess) {
                return fail(FIGARO_EHIP, "copying the keys of relation " + std::to_string(i) + " failed");
            }
        }
        S.keys[i].assign(d.num_keys, std::vector<int64_t>((size_t)d.rows));
        for (int q = 0; q < d.num_keys; ++q)
            for (int64_t t = 0; t < d.rows; ++t) {
                const size_t at = (size_t)q * (size_t)d.rows + (size_t)t;
                S.keys[i][q][t] = elem == 4 ? (int64_t)reinterpret_cast<const int32_t *>(raw.data())[at]
                                            : reinterpret_cast<const int64_t *>(raw.data())[at];
            }
    }
    return FIGARO_OK;
}

// Edges of a spanning tree (pairs i < j) -> whether every attribute's
// relations form a connected part of it, and every key attribute is shared
// with a tree neighbour.
bool running_intersection(const Schema &S, const std::vector<std::pair<int, int>> &edges) {
    std::map<int32_t, int> holders;
    for (int i = 0; i < S.r; ++i)
        for (int32_t a : S.attrs[i]) holders[a]++;
    std::map<int32_t, int> inner;
    for (auto [i, j] : edges)
        for (int32_t a : S.shared(i, j)) inner[a]++;
    for (auto [a, h] : holders) {
        if (h < 2) return false;     // a key attribute nobody else has
        if (inner[a] != h - 1) return false;
    }
    return true;
}

// Parents of the tree rooted at `root`, and the score.
double score(Schema &S, const std::vector<std::pair<int, int>> &edges, int root, std::vector<int32_t> &parent) {
    const int r = S.r;
    std::vector<std::vector<int>> adj(r);
    for (auto [i, j] : edges) {
        adj[i].push_back(j);
        adj[j].push_back(i);
    }
    parent.assign(r, -2);
    parent[root] = -1;
    std::vector<int> order{root};
    for (size_t q = 0; q < order.size(); ++q)
        for (int v : adj[order[q]])
            if (parent[v] == -2) {
                parent[v] = order[q];
                order.push_back(v);
            }
    std::vector<double> nsub(r, 0.0);
    for (int q = r - 1; q >= 0; --q) {
        const int v = order[q];
        nsub[v] += S.ncols[v];
        if (parent[v] >= 0) nsub[parent[v]] += nsub[v];
    }
    double cost = 0.0;
    for (int i = 0; i < r; ++i) {
        std::vector<int32_t> all = S.attrs[i];
        std::sort(all.begin(), all.end());
        const double G = (double)S.distinct(i, all);
        const double ni = S.ncols[i];
        cost += ((double)S.m[i] - G) * ni * ni;
        if (parent[i] >= 0) {
            const double P = (double)S.distinct(i, S.shared(i, parent[i]));
            cost += (G - P) * nsub[i] * nsub[i];
        } else {
            cost += G * nsub[i] * nsub[i];
        }
    }
    return cost;
}

// Every spanning tree of the graph on `candidate` edges (edge subsets of size
// r - 1 without a cycle), in a fixed order.
void spanning_trees(int r, const std::vector<std::pair<int, int>> &cand, size_t at,
                    std::vector<std::pair<int, int>> &cur, std::vector<int> &comp,
                    std::vector<std::vector<std::pair<int, int>>> &out) {
    if ((int)cur.size() == r - 1) {
        out.push_back(cur);
        return;
    }
    if ((int64_t)out.size() >= kMaxTrees) return;
    if (cand.size() - at < (size_t)(r - 1) - cur.size()) return;
    for (size_t e = at; e < cand.size(); ++e) {
        const int a = comp[cand[e].first], b = comp[cand[e].second];
        if (a == b) continue;
        std::vector<int> saved = comp;
        for (int &c : comp)
            if (c == b) c = a;
        cur.push_back(cand[e]);
        spanning_trees(r, cand, e + 1, cur, comp, out);
        cur.pop_back();
        comp = saved;
        if ((int64_t)out.size() >= kMaxTrees) return;
    }
}

}  // namespace

extern "C" {

figaro_status figaro_join_tree_cost(int32_t r, const figaro_relation_desc *rels, int32_t keys_on_host,
                                    double *cost_out, hipStream_t stream) {
    Schema S;
    figaro_status st = load_schema(S, r, rels, keys_on_host, stream);
    if (st != FIGARO_OK) return st;
    if (!cost_out) return fail(FIGARO_EINVAL, "cost_out is NULL");
    std::vector<std::pair<int, int>> edges;
    int root = -1;
    for (int i = 0; i < r; ++i) {
        const int p = rels[i].parent;
        if (p == -1) {
            if (root >= 0) return fail(FIGARO_ENOTTREE, "more than one root");
            root = i;
        } else if (p < 0 || p >= r || p == i) {
            return fail(FIGARO_ENOTTREE, "parent out of range");
        } else {
            edges.push_back({std::min(i, p), std::max(i, p)});
        }
    }
    if (root < 0) return fail(FIGARO_ENOTTREE, "no root");
    std::vector<int> comp(r);
    std::iota(comp.begin(), comp.end(), 0);
    for (auto [i, j] : edges) {
        const int a = comp[i], b = comp[j];
        if (a == b) return fail(FIGARO_ENOTTREE, "parent links contain a cycle");
        for (int &c : comp)
            if (c == b) c = a;
    }
    if (!running_intersection(S, edges))
        return fail(FIGARO_ENOTTREE, "the tree violates the running intersection property or leaves a key unshared");
    std::vector<int32_t> parent;
    *cost_out = score(S, edges, root, parent);
    return FIGARO_OK;
}

figaro_status figaro_choose_join_tree(int32_t r, const figaro_relation_desc *rels, int32_t keys_on_host,
                                      int32_t *parents_out, double *cost_out, hipStream_t stream) {
    Schema S;
    figaro_status st = load_schema(S, r, rels, keys_on_host, stream);
    if (st != FIGARO_OK) return st;
    if (!parents_out) return fail(FIGARO_EINVAL, "parents_out is NULL");
    // candidate edges: relations that share attributes; when those leave the
    // relations disconnected, every pair (the missing links are Cartesian
    // products, allowed between relations that share nothing)
    std::vector<std::pair<int, int>> cand, all;
    for (int i = 0; i < r; ++i)
        for (int j = i + 1; j < r; ++j) {
            all.push_back({i, j});
            if (!S.shared(i, j).empty()) cand.push_back({i, j});
        }
    std::vector<std::vector<std::pair<int, int>>> trees;
    std::vector<std::pair<int, int>> cur;
    std::vector<int> comp(r);
    std::iota(comp.begin(), comp.end(), 0);
    spanning_trees(r, cand, 0, cur, comp, trees);
    if (trees.empty() && r > 1) {
        std::iota(comp.begin(), comp.end(), 0);
        spanning_trees(r, all, 0, cur, comp, trees);
    }
    if (r == 1) trees.push_back({});
    double best = 0.0;
    std::vector<int32_t> best_parent;
    for (const auto &t : trees) {
        if (!running_intersection(S, t)) continue;
        for (int root = 0; root < r; ++root) {
            std::vector<int32_t> parent;
            const double c = score(S, t, root, parent);
            if (best_parent.empty() || c < best) {
                best = c;
                best_parent = parent;
            }
        }
    }
    if (best_parent.empty()) return fail(FIGARO_ENOTTREE, "no join tree exists (the join is cyclic)");
    std::copy(best_parent.begin(), best_parent.end(), parents_out);
    if (cost_out) *cost_out = best;
    return FIGARO_OK;
}

}  // extern "C"
