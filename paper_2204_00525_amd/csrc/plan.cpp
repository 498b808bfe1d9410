// Plan construction: everything that depends on the keys only.
//
//  * validation of the join tree (single root, connected, running
//    intersection, every key attribute shared with a neighbour);
//  * semi-join reduction of dangling tuples (the paper assumes a fully
//    reduced database; a bottom-up then top-down pass of semi-joins over the
//    join tree produces one);
//  * the sort order both of the paper's algorithms assume: each relation
//    sorted on the attributes it shares with its parent, then on its other
//    key attributes (ties by row index);
//  * the count queries of Fig. 4 by Algorithm 2 (bottom-up pass computing
//    rows_per_key, Theta_down and Phi_down, top-down pass computing
//    full_join_size, Phi_up and Phi_circ), exactly, in 64-bit integers;
//  * the scale factors of Algorithm 3, and the tables of the segmented
//    head/tail kernels (pieces, chunks, tail coefficients);
//  * the device workspace.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

using u128 = unsigned __int128;

namespace figaro {

thread_local std::string g_thread_error;

figaro_status set_error(figaro_plan_s *p, figaro_status st, const std::string &msg) {
    if (p) p->last_error = msg;
    g_thread_error = msg;
    return st;
}

namespace {

constexpr int64_t kExactLimit = int64_t(1) << 53;   // counts must stay below 2^53

struct Packer {
    // packs the dense ids of a list of attributes (high bits first)
    std::vector<int32_t> attrs;   // global attribute ids, in packing order
    std::vector<int> shift;
    int bits = 0;
};

struct Builder {
    figaro_plan_s *p;
    int32_t r;
    std::vector<std::vector<int64_t>> keys;     // per relation [k][m] raw keys
    std::vector<std::vector<int32_t>> ids;      // per relation [k][m] dense ids
    std::vector<int> attr_bits;                 // per attribute id (dense index)
    std::vector<int32_t> attr_list;             // distinct attribute ids
    std::vector<std::vector<char>> alive;

    int attr_index(int32_t a) const {
        auto it = std::lower_bound(attr_list.begin(), attr_list.end(), a);
        return int(it - attr_list.begin());
    }
    int key_pos(int i, int32_t a) const {
        const auto &at = p->rel[i].attrs;
        for (size_t q = 0; q < at.size(); ++q)
            if (at[q] == a) return int(q);
        return -1;
    }
    std::vector<int32_t> shared(int i, int j) const {
        std::vector<int32_t> out;
        for (int32_t a : p->rel[i].attrs)
            if (key_pos(j, a) >= 0) out.push_back(a);
        std::sort(out.begin(), out.end());
        return out;
    }
    Packer make_packer(const std::vector<int32_t> &attrs) const {
        Packer pk;
        pk.attrs = attrs;
        int total = 0;
        for (int32_t a : attrs) total += attr_bits[attr_index(a)];
        pk.bits = total;
        int s = total;
        for (int32_t a : attrs) {
            s -= attr_bits[attr_index(a)];
            pk.shift.push_back(s);
        }
        return pk;
    }
    u128 pack(int i, int64_t row, const Packer &pk) const {
        u128 v = 0;
        for (size_t q = 0; q < pk.attrs.size(); ++q) {
            int kp = key_pos(i, pk.attrs[q]);
            v |= (u128)(uint32_t)ids[i][(size_t)kp * p->rel[i].m_in + row] << pk.shift[q];
        }
        return v;
    }
    // packed keys of every row of relation i
    std::vector<u128> pack_all(int i, const Packer &pk) const {
        const int64_t m = p->rel[i].m_in;
        std::vector<u128> v(m, 0);
        for (size_t q = 0; q < pk.attrs.size(); ++q) {
            const int32_t *col = ids[i].data() + (size_t)key_pos(i, pk.attrs[q]) * m;
            const int sh = pk.shift[q];
            for (int64_t t = 0; t < m; ++t) v[t] |= (u128)(uint32_t)col[t] << sh;
        }
        return v;
    }
};

// Sorts 128-bit words whose set bits all lie below `bits`: least significant
// digit first radix sort, 16-bit digits (stable passes, so equal digits keep
// their order).
void radix_sort_u128(std::vector<u128> &v, int bits) {
    if (v.size() < 2) return;
    std::vector<u128> tmp(v.size());
    std::vector<int64_t> count(1 << 16);
    for (int shift = 0; shift < bits; shift += 16) {
        std::fill(count.begin(), count.end(), 0);
        for (u128 x : v) ++count[(size_t)(x >> shift) & 0xffff];
        int64_t sum = 0;
        for (auto &c : count) {
            const int64_t t = c;
            c = sum;
            sum += t;
        }
        for (u128 x : v) tmp[count[(size_t)(x >> shift) & 0xffff]++] = x;
        v.swap(tmp);
    }
}

// Position of packed keys in a sorted list of distinct keys: a direct table
// when the keys have few bits, else binary search.
struct KeyIndex {
    static constexpr int kDirectBits = 26;
    bool direct = false;
    std::vector<int32_t> table;         // direct: key -> position, -1 absent
    const std::vector<u128> *sorted = nullptr;
    KeyIndex(const std::vector<u128> &keys, int bits) : sorted(&keys) {
        if (bits <= kDirectBits) {
            direct = true;
            table.assign((size_t)1 << bits, -1);
            for (size_t q = 0; q < keys.size(); ++q) table[(size_t)keys[q]] = (int32_t)q;
        }
    }
    int64_t find(u128 k) const {
        if (direct) return table[(size_t)k];
        auto it = std::lower_bound(sorted->begin(), sorted->end(), k);
        return (it == sorted->end() || *it != k) ? -1 : (int64_t)(it - sorted->begin());
    }
};

void postorder(const figaro_plan_s *p, int v, std::vector<int32_t> &out) {
    for (int c : p->rel[v].children) postorder(p, c, out);
    out.push_back(v);
}

}  // namespace

// Build the levels `first`, first + 1, ... of one segmented head/tail task
// from the state of level `first`:
//   goff : [ngroups+1] item offsets of the groups over this level's items
//   cnt  : per-item counts (empty with unit = every item counts 1, level 0)
//   phi  : per-group tail scale
//   tile : items per chunk of the first level (the task's tile shape)
// The upper levels are small and latency-bound: they take the shape with two
// waves per SIMD (variant 2) and its smaller chunks, which doubles the waves
// in flight (ncols <= 32; wider tasks keep the task's shape).
figaro_status build_task_levels(figaro_plan_s *p, Task &T, int first, int64_t items, std::vector<int64_t> goff,
                                std::vector<int64_t> cnt, bool unit, const std::vector<double> &phi, int tile) {
    const int up_variant = (T.ncols <= 32) ? 2 : T.variant;
    const int tile_up = std::min(tile, tile_items_for(T.ncols, up_variant));
    const int64_t ngroups = (int64_t)goff.size() - 1;
    int64_t nitems = items;
    for (int level = first; level < 64; ++level) {
        Level L;
        L.items = nitems;
        L.unit = unit;
        L.variant = level == 0 ? T.variant : up_variant;
        // chunks
        std::vector<int64_t> cs;
        cs.push_back(0);
        if (level == 0) {
            for (int64_t s = tile; s < nitems; s += tile) cs.push_back(s);
            cs.push_back(nitems);
        } else {
            int64_t cur = 0;       // items in the current chunk
            for (int64_t g = 0; g < ngroups; ++g) {
                int64_t gs = goff[g], ge = goff[g + 1], sz = ge - gs;
                if (sz > tile_up) {
                    if (cur > 0) { cs.push_back(gs); cur = 0; }
                    for (int64_t s = gs + tile_up; s < ge; s += tile_up) cs.push_back(s);
                    cs.push_back(ge);
                    cur = 0;
                } else {
                    if (cur + sz > tile_up) { cs.push_back(gs); cur = 0; }
                    cur += sz;
                }
            }
            if (cs.back() != nitems) cs.push_back(nitems);
        }
        L.nchunks = (int64_t)cs.size() - 1;
        // pieces: chunk x group intersections
        std::vector<int32_t> pid(nitems);
        std::vector<int32_t> cpiece(L.nchunks + 1);
        std::vector<int64_t> pstart;
        std::vector<int64_t> pgroup;
        std::vector<int64_t> pcount;
        int64_t g = 0;
        for (int64_t c = 0; c < L.nchunks; ++c) {
            int64_t a = cs[c], b = cs[c + 1];
            int64_t t = a;
            cpiece[c] = (int32_t)pstart.size();
            while (t < b) {
                while (goff[g + 1] <= t) ++g;
                int64_t e = std::min(b, goff[g + 1]);
                int64_t idx = (int64_t)pstart.size();
                pstart.push_back(t);
                pgroup.push_back(g);
                int64_t sum = 0;
                for (int64_t q = t; q < e; ++q) {
                    pid[q] = (int32_t)idx;
                    sum += unit ? 1 : cnt[q];
                }
                pcount.push_back(sum);
                t = e;
            }
        }
        L.npieces = (int64_t)pstart.size();
        if (L.npieces >= (int64_t(1) << 31) - 2)
            return set_error(p, FIGARO_EUNSUPPORTED, "too many pieces in one head/tail level");
        cpiece[L.nchunks] = (int32_t)L.npieces;
        pstart.push_back(nitems);
        hipError_t e;
        if ((e = dev_upload(p, &L.d_pid, pid)) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        if ((e = dev_upload(p, &L.d_piece_start, pstart)) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        if ((e = dev_upload(p, &L.d_chunk_start, cs)) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        if ((e = dev_upload(p, &L.d_chunk_piece0, cpiece)) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        if (unit) {
            std::vector<double> pp(L.npieces + 1, 0.0);   // one entry of padding for 16-byte copies
            for (int64_t q = 0; q < L.npieces; ++q) pp[q] = phi[pgroup[q]];
            if (dev_upload(p, &L.d_phi_piece, pp) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        } else {
            std::vector<double> al(nitems), be(nitems);
            for (int64_t q = 0; q < L.npieces; ++q) {
                int64_t W = 0;
                double ph = phi[pgroup[q]];
                for (int64_t t = pstart[q]; t < pstart[q + 1]; ++t) {
                    int64_t c = cnt[t];
                    if (W == 0) {
                        al[t] = 0.0;
                        be[t] = 0.0;
                    } else {
                        double sW = std::sqrt((double)W), sc = std::sqrt((double)c),
                               sWi = std::sqrt((double)(W + c));
                        al[t] = ph * sW / (sc * sWi);
                        be[t] = ph * sc / (sW * sWi);
                    }
                    W += c;
                }
            }
            if (dev_upload(p, &L.d_alpha, al) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            if (dev_upload(p, &L.d_beta, be) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        }
        if (dev_alloc(p, (void **)&L.d_pieces, sizeof(double) * (size_t)T.ncols * (size_t)L.npieces) != hipSuccess ||
            dev_alloc(p, (void **)&L.d_gpieces, sizeof(double) * (size_t)T.ncols * (size_t)L.npieces) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        L.waves = (int32_t)std::min<int64_t>(L.nchunks, p->waves_cap);
        if (L.waves < 1) L.waves = 1;
        T.levels.push_back(L);
        if (L.npieces == ngroups) return FIGARO_OK;
        // next level: items are the pieces
        std::vector<int64_t> ngoff(ngroups + 1, 0);
        for (int64_t q = 0; q < L.npieces; ++q) ngoff[pgroup[q] + 1]++;
        for (int64_t q = 0; q < ngroups; ++q) ngoff[q + 1] += ngoff[q];
        goff = ngoff;
        cnt = pcount;
        nitems = L.npieces;
        unit = false;
    }
    return set_error(p, FIGARO_EUNSUPPORTED, "head/tail levels do not converge");
}

namespace {

figaro_status build_task(figaro_plan_s *p, Task &T, int64_t items, const std::vector<int64_t> &group_off,
                         const std::vector<int64_t> &counts, const std::vector<double> &phi, int tile) {
    return build_task_levels(p, T, 0, items, group_off, counts, counts.empty(), phi, tile);
}

}  // namespace

figaro_status join_chunks(figaro_plan_s *p, RelPlan &R, size_t c, const std::vector<int64_t> &off) {
    const int64_t Pc = (int64_t)off.size() - 1;
    int64_t longest = 0;
    for (int64_t q = 0; q < Pc; ++q) longest = std::max(longest, off[q + 1] - off[q]);
    if (longest <= kJoinChunk) {
        R.join_nchunks.push_back(0);
        R.d_chunk_off.push_back(nullptr);
        R.d_chunk_q.push_back(nullptr);
        R.d_join_part.push_back(nullptr);
        return FIGARO_OK;
    }
    std::vector<int64_t> coff(Pc + 1, 0);
    for (int64_t q = 0; q < Pc; ++q) coff[q + 1] = coff[q] + (off[q + 1] - off[q] + kJoinChunk - 1) / kJoinChunk;
    std::vector<int32_t> cq(coff[Pc]);
    for (int64_t q = 0; q < Pc; ++q)
        for (int64_t k = coff[q]; k < coff[q + 1]; ++k) cq[k] = (int32_t)q;
    int64_t *dco = nullptr;
    int32_t *dcq = nullptr;
    double *part = nullptr;
    const int64_t cols = p->rel[R.children[c]].nsub;
    if (dev_upload(p, &dco, coff) != hipSuccess || dev_upload(p, &dcq, cq) != hipSuccess ||
        dev_alloc(p, (void **)&part, sizeof(double) * (size_t)coff[Pc] * (size_t)cols) != hipSuccess)
        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    R.join_nchunks.push_back(coff[Pc]);
    R.d_chunk_off.push_back(dco);
    R.d_chunk_q.push_back(dcq);
    R.d_join_part.push_back(part);
    return FIGARO_OK;
}

figaro_status finish_task(figaro_plan_s *p, Task &T, int32_t n_total) {
    std::vector<int32_t> inv(n_total, -1);
    for (size_t q = 0; q < T.cols.size(); ++q) inv[T.cols[q]] = (int32_t)q;
    if (dev_upload(p, &T.d_colmap, T.cols) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    if (dev_upload(p, &T.d_inv_colmap, inv) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    return FIGARO_OK;
}

namespace {

// Phase timing of plan construction, printed to stderr when the environment
// variable FIGARO_PLAN_TIMING is set.
struct PhaseTimer {
    bool on = std::getenv("FIGARO_PLAN_TIMING") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char *phase) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[figaro plan] %-28s %9.3f s\n", phase, std::chrono::duration<double>(now - t).count());
        t = now;
    }
};

figaro_status build(figaro_plan_s *p, int32_t r, const figaro_relation_desc *rels,
                    const figaro_plan_options *opts, hipStream_t stream) {
    PhaseTimer timer;
    Builder B;
    B.p = p;
    B.r = r;
    p->r = r;
    p->rel.resize(r);
    p->tile_items = opts ? opts->tile_items : 0;
    p->waves_cap = (opts && opts->waves_per_task > 0) ? opts->waves_per_task : 1024;
    const bool keys_on_host = opts && opts->keys_on_host;
    p->analyze_only = opts && opts->analyze_only;
    p->variant = opts ? opts->variant : 0;
    p->separate_join = opts && opts->separate_join;
    if (p->variant < 0 || p->variant >= num_variants())
        return set_error(p, FIGARO_EINVAL, "variant out of range");
    if (p->tile_items < 0) return set_error(p, FIGARO_EINVAL, "tile_items must be >= 0");
    // ---- argument checks
    int roots = 0;
    for (int i = 0; i < r; ++i) {
        const auto &d = rels[i];
        auto &R = p->rel[i];
        if (d.rows < 0) return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": rows < 0");
        if (d.num_keys < 0 || d.num_keys > 32)
            return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": num_keys out of range");
        if (d.num_keys > 0 && (d.key_attr == nullptr || (d.key_cols == nullptr && d.rows > 0)))
            return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": null key pointer");
        if (d.num_keys > 0 && d.key_dtype != 4 && d.key_dtype != 8)
            return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": key_dtype must be 4 or 8");
        if (d.num_cols < 1) return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": num_cols < 1");
        if (d.parent < -1 || d.parent >= r || d.parent == i)
            return set_error(p, FIGARO_ENOTTREE, "relation " + std::to_string(i) + ": parent out of range");
        if (d.parent == -1) { ++roots; p->root = i; }
        R.m_in = d.rows;
        R.nkeys = d.num_keys;
        R.attrs.assign(d.key_attr, d.key_attr + d.num_keys);
        R.ncols = d.num_cols;
        R.parent = d.parent;
        for (int a = 0; a < d.num_keys; ++a)
            for (int b = a + 1; b < d.num_keys; ++b)
                if (R.attrs[a] == R.attrs[b])
                    return set_error(p, FIGARO_EINVAL, "relation " + std::to_string(i) + ": repeated key attribute");
    }
    if (roots != 1) return set_error(p, FIGARO_ENOTTREE, "the join tree must have exactly one root");
    for (int i = 0; i < r; ++i)
        if (p->rel[i].parent >= 0) p->rel[p->rel[i].parent].children.push_back(i);
    {
        // connected from the root (each node has one parent, so reachability of all nodes == tree)
        std::vector<char> seen(r, 0);
        std::vector<int> st{p->root};
        int cnt = 0;
        while (!st.empty()) {
            int v = st.back();
            st.pop_back();
            if (seen[v]) return set_error(p, FIGARO_ENOTTREE, "cycle in parent links");
            seen[v] = 1;
            ++cnt;
            for (int c : p->rel[v].children) st.push_back(c);
        }
        if (cnt != r) return set_error(p, FIGARO_ENOTTREE, "parent links do not form one tree");
    }
    postorder(p, p->root, p->post);
    // running intersection and shared keys
    {
        std::vector<int32_t> all;
        for (int i = 0; i < r; ++i) all.insert(all.end(), p->rel[i].attrs.begin(), p->rel[i].attrs.end());
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        B.attr_list = all;
        for (int32_t a : all) {
            int nodes = 0, edges = 0;
            for (int i = 0; i < r; ++i) {
                if (B.key_pos(i, a) < 0) continue;
                ++nodes;
                int pp = p->rel[i].parent;
                if (pp >= 0 && B.key_pos(pp, a) >= 0) ++edges;
            }
            if (edges != nodes - 1)
                return set_error(p, FIGARO_ENOTTREE,
                                 "attribute " + std::to_string(a) + " violates the running intersection property");
        }
        for (int i = 0; i < r; ++i)
            for (int32_t a : p->rel[i].attrs) {
                bool ok = p->rel[i].parent >= 0 && B.key_pos(p->rel[i].parent, a) >= 0;
                for (int c : p->rel[i].children) ok = ok || B.key_pos(c, a) >= 0;
                if (!ok)
                    return set_error(p, FIGARO_EUNSHARED_KEY, "relation " + std::to_string(i) + ": key attribute " +
                                                                  std::to_string(a) + " is shared with no neighbour");
            }
    }
    // columns
    int32_t n = 0;
    for (int i = 0; i < r; ++i) {
        p->rel[i].col0 = n;
        n += p->rel[i].ncols;
    }
    p->n = n;
    if (n > kMaxWideCols) return set_error(p, FIGARO_EUNSUPPORTED, "more than 16384 data columns in total");
    p->wide = n > kMaxCols;
    // keys on the device: segmentation, counts and the tasks' first levels
    // there (the host path below stays for host keys and analysis-only plans)
    if (!keys_on_host && !p->analyze_only && !(opts && opts->host_plan)) {
        p->device_plan = true;
        figaro_status st = build_keys_on_device(p, rels, stream);
        if (st != FIGARO_OK) return st;
        timer.mark("plan on the device");
        return finish_plan(p);
    }
    // ---- keys to the host
    B.keys.resize(r);
    for (int i = 0; i < r; ++i) {
        const auto &d = rels[i];
        size_t cnt = (size_t)d.num_keys * (size_t)d.rows;
        B.keys[i].resize(cnt);
        if (cnt == 0) continue;
        if (keys_on_host) {
            if (d.key_dtype == 8) {
                std::memcpy(B.keys[i].data(), d.key_cols, cnt * 8);
            } else {
                const int32_t *src = (const int32_t *)d.key_cols;
                for (size_t q = 0; q < cnt; ++q) B.keys[i][q] = src[q];
            }
        } else if (d.key_dtype == 8) {
            if (hipMemcpyAsync(B.keys[i].data(), d.key_cols, cnt * 8, hipMemcpyDeviceToHost, stream) != hipSuccess)
                return set_error(p, FIGARO_EHIP, "copying key columns to the host failed");
        } else {
            std::vector<int32_t> tmp(cnt);
            if (hipMemcpyAsync(tmp.data(), d.key_cols, cnt * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return set_error(p, FIGARO_EHIP, "copying key columns to the host failed");
            for (size_t q = 0; q < cnt; ++q) B.keys[i][q] = tmp[q];
        }
    }
    if (!keys_on_host && hipStreamSynchronize(stream) != hipSuccess)
        return set_error(p, FIGARO_EHIP, "hipStreamSynchronize failed");
    timer.mark("keys to the host");
    // ---- dictionary-encode every attribute
    B.attr_bits.assign(B.attr_list.size(), 1);
    B.ids.resize(r);
    for (int i = 0; i < r; ++i) B.ids[i].resize(B.keys[i].size());
    for (size_t ai = 0; ai < B.attr_list.size(); ++ai) {
        int32_t a = B.attr_list[ai];
        std::vector<int64_t> vals;
        for (int i = 0; i < r; ++i) {
            int kp = B.key_pos(i, a);
            if (kp < 0) continue;
            const int64_t *col = B.keys[i].data() + (size_t)kp * p->rel[i].m_in;
            vals.insert(vals.end(), col, col + p->rel[i].m_in);
        }
        // dense ids in increasing key order: a presence table over the key
        // range when it is small, else sort and binary search
        int64_t lo = 0, hi = -1;
        if (!vals.empty()) {
            const auto mm = std::minmax_element(vals.begin(), vals.end());
            lo = *mm.first;
            hi = *mm.second;
        }
        const bool table = !vals.empty() && (uint64_t)(hi - lo) < (uint64_t)(8 * vals.size() + (1 << 20));
        std::vector<int32_t> rank;
        size_t distinct;
        if (table) {
            rank.assign((size_t)(hi - lo) + 1, 0);
            for (int64_t v : vals) rank[(size_t)(v - lo)] = 1;
            int32_t next = 0;
            for (auto &x : rank) x = x ? next++ : -1;
            distinct = (size_t)next;
        } else {
            std::sort(vals.begin(), vals.end());
            vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
            distinct = vals.size();
        }
        int bits = 1;
        while ((int64_t(1) << bits) < (int64_t)distinct) ++bits;
        B.attr_bits[ai] = bits;
        for (int i = 0; i < r; ++i) {
            int kp = B.key_pos(i, a);
            if (kp < 0) continue;
            const int64_t *col = B.keys[i].data() + (size_t)kp * p->rel[i].m_in;
            int32_t *out = B.ids[i].data() + (size_t)kp * p->rel[i].m_in;
            if (table)
                for (int64_t t = 0; t < p->rel[i].m_in; ++t) out[t] = rank[(size_t)(col[t] - lo)];
            else
                for (int64_t t = 0; t < p->rel[i].m_in; ++t)
                    out[t] = (int32_t)(std::lower_bound(vals.begin(), vals.end(), col[t]) - vals.begin());
        }
    }
    for (int i = 0; i < r; ++i) {
        Packer pk = B.make_packer(p->rel[i].attrs);
        if (pk.bits > 127)
            return set_error(p, FIGARO_EUNSUPPORTED, "composite key of relation " + std::to_string(i) +
                                                         " needs more than 127 bits");
    }
    timer.mark("dictionary encoding");
    // ---- semi-join reduction (bottom-up, then top-down)
    B.alive.resize(r);
    for (int i = 0; i < r; ++i) B.alive[i].assign(p->rel[i].m_in, 1);
    auto semijoin = [&](int keep_side, int probe_side) {
        // keep rows of keep_side whose projection on the shared attributes
        // occurs among the alive rows of probe_side
        std::vector<int32_t> sh = B.shared(keep_side, probe_side);
        Packer pk = B.make_packer(sh);
        const std::vector<u128> pk_probe = B.pack_all(probe_side, pk);
        const std::vector<u128> pk_keep = B.pack_all(keep_side, pk);
        if (pk.bits <= KeyIndex::kDirectBits) {
            // presence table over the packed keys
            std::vector<char> present((size_t)1 << pk.bits, 0);
            for (int64_t t = 0; t < p->rel[probe_side].m_in; ++t)
                if (B.alive[probe_side][t]) present[(size_t)pk_probe[t]] = 1;
            for (int64_t t = 0; t < p->rel[keep_side].m_in; ++t)
                if (B.alive[keep_side][t] && !present[(size_t)pk_keep[t]]) B.alive[keep_side][t] = 0;
            return;
        }
        std::vector<u128> set;
        set.reserve(p->rel[probe_side].m_in);
        for (int64_t t = 0; t < p->rel[probe_side].m_in; ++t)
            if (B.alive[probe_side][t]) set.push_back(pk_probe[t]);
        radix_sort_u128(set, pk.bits);
        set.erase(std::unique(set.begin(), set.end()), set.end());
        const KeyIndex index(set, pk.bits);
        for (int64_t t = 0; t < p->rel[keep_side].m_in; ++t)
            if (B.alive[keep_side][t] && index.find(pk_keep[t]) < 0) B.alive[keep_side][t] = 0;
    };
    for (int v : p->post)
        if (p->rel[v].parent >= 0) semijoin(p->rel[v].parent, v);
    for (auto it = p->post.rbegin(); it != p->post.rend(); ++it)
        if (p->rel[*it].parent >= 0) semijoin(*it, p->rel[*it].parent);
    for (int i = 0; i < r; ++i) {
        int64_t m = 0;
        for (int64_t t = 0; t < p->rel[i].m_in; ++t) m += B.alive[i][t];
        p->rel[i].m = m;
        if (m == 0) return set_error(p, FIGARO_EEMPTY_JOIN, "the join is empty");
    }
    timer.mark("semi-join reduction");
    // ---- sort, segment, parent groups
    std::vector<Packer> xp_pack(r), full_pack(r);
    std::vector<std::vector<u128>> pgroup_keys(r);
    std::vector<std::vector<u128>> seg_keys(r);     // full packed key of each segment (xp high)
    for (int i = 0; i < r; ++i) {
        auto &R = p->rel[i];
        std::vector<int32_t> xp = R.parent >= 0 ? B.shared(i, R.parent) : std::vector<int32_t>{};
        std::vector<int32_t> rest;
        for (int32_t a : R.attrs)
            if (std::find(xp.begin(), xp.end(), a) == xp.end()) rest.push_back(a);
        std::sort(rest.begin(), rest.end());
        xp_pack[i] = B.make_packer(xp);
        std::vector<int32_t> order = xp;
        order.insert(order.end(), rest.begin(), rest.end());
        full_pack[i] = B.make_packer(order);
        const int rest_bits = full_pack[i].bits - xp_pack[i].bits;
        std::vector<std::pair<u128, int64_t>> kv;
        kv.reserve(R.m);
        {
            const std::vector<u128> packed = B.pack_all(i, full_pack[i]);
            int row_bits = 1;
            while ((int64_t(1) << row_bits) < R.m_in) ++row_bits;
            if (full_pack[i].bits + row_bits <= 128) {
                // (key, row) in one 128-bit word: one comparison per step
                std::vector<u128> w;
                w.reserve(R.m);
                for (int64_t t = 0; t < R.m_in; ++t)
                    if (B.alive[i][t]) w.push_back((packed[t] << row_bits) | (u128)t);
                radix_sort_u128(w, full_pack[i].bits + row_bits);
                const u128 row_mask = ((u128)1 << row_bits) - 1;
                for (u128 x : w) kv.emplace_back(x >> row_bits, (int64_t)(x & row_mask));
            } else {
                for (int64_t t = 0; t < R.m_in; ++t)
                    if (B.alive[i][t]) kv.emplace_back(packed[t], t);
                std::sort(kv.begin(), kv.end());
            }
        }
        R.perm.resize(R.m_in);
        for (int64_t q = 0; q < R.m; ++q) R.perm[q] = kv[q].second;
        int64_t q = R.m;
        for (int64_t t = 0; t < R.m_in; ++t)
            if (!B.alive[i][t]) R.perm[q++] = t;
        R.seg_off.clear();
        for (int64_t t = 0; t < R.m; ++t)
            if (t == 0 || kv[t].first != kv[t - 1].first) {
                R.seg_off.push_back(t);
                seg_keys[i].push_back(kv[t].first);
            }
        R.seg_off.push_back(R.m);
        R.G = (int64_t)R.seg_off.size() - 1;
        R.par_off.clear();
        if (R.parent >= 0) {
            for (int64_t g = 0; g < R.G; ++g) {
                u128 hi = rest_bits >= 128 ? (u128)0 : (seg_keys[i][g] >> rest_bits);
                if (g == 0 || hi != pgroup_keys[i].back()) {
                    R.par_off.push_back(g);
                    pgroup_keys[i].push_back(hi);
                }
            }
            R.par_off.push_back(R.G);
            R.P = (int64_t)R.par_off.size() - 1;
        } else {
            R.P = 0;
        }
        R.singleton = (R.G == R.m);
        if (!p->analyze_only && dev_upload(p, &R.d_perm, R.perm) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    }
    timer.mark("sort and segments");
    // ---- child index of every key group
    std::vector<std::vector<std::vector<int32_t>>> cidx(r);
    for (int i = 0; i < r; ++i) {
        auto &R = p->rel[i];
        for (int c : R.children) {
            std::vector<int32_t> idx(R.G);
            const KeyIndex index(pgroup_keys[c], xp_pack[c].bits);
            const std::vector<u128> packed = B.pack_all(i, xp_pack[c]);
            for (int64_t g = 0; g < R.G; ++g) {
                const int64_t q = index.find(packed[R.perm[R.seg_off[g]]]);
                if (q < 0) return set_error(p, FIGARO_EINVAL, "internal: unmatched key after reduction");
                idx[g] = (int32_t)q;
            }
            cidx[i].push_back(idx);
        }
    }
    timer.mark("child indices");
    // ---- count queries, Algorithm 2
    auto check = [&](u128 v) { return v < (u128)kExactLimit; };
    for (int v : p->post) {   // pass 1: bottom-up
        auto &R = p->rel[v];
        R.rpk.resize(R.G);
        R.theta.resize(R.G);
        for (int64_t g = 0; g < R.G; ++g) {
            R.rpk[g] = R.seg_off[g + 1] - R.seg_off[g];
            u128 th = (u128)R.rpk[g];
            for (size_t c = 0; c < R.children.size(); ++c) {
                th *= (u128)p->rel[R.children[c]].phi_down[cidx[v][c][g]];
                if (!check(th)) return set_error(p, FIGARO_EOVERFLOW, "a count query reaches 2^53");
            }
            R.theta[g] = (int64_t)th;
        }
        if (R.parent >= 0) {
            R.phi_down.assign(R.P, 0);
            for (int64_t q = 0; q < R.P; ++q) {
                u128 s = 0;
                for (int64_t g = R.par_off[q]; g < R.par_off[q + 1]; ++g) s += (u128)R.theta[g];
                if (!check(s)) return set_error(p, FIGARO_EOVERFLOW, "a count query reaches 2^53");
                R.phi_down[q] = (int64_t)s;
            }
        }
    }
    {
        u128 total = 0;
        for (int64_t t : p->rel[p->root].theta) total += (u128)t;
        if (!check(total)) return set_error(p, FIGARO_EOVERFLOW, "the join size reaches 2^53");
        p->join_rows = (double)(int64_t)total;
    }
    for (auto it = p->post.rbegin(); it != p->post.rend(); ++it) {   // pass 2: top-down
        int v = *it;
        auto &R = p->rel[v];
        R.fjs.resize(R.G);
        R.phi_circ.resize(R.G);
        std::vector<std::vector<u128>> acc(R.children.size());
        for (size_t c = 0; c < R.children.size(); ++c) acc[c].assign(p->rel[R.children[c]].P, 0);
        int64_t q = 0;
        for (int64_t g = 0; g < R.G; ++g) {
            u128 up = 1;
            if (R.parent >= 0) {
                while (R.par_off[q + 1] <= g) ++q;
                up = (u128)R.phi_up[q];
            }
            u128 f = up * (u128)R.theta[g];
            if (!check(f)) return set_error(p, FIGARO_EOVERFLOW, "a count query reaches 2^53");
            R.fjs[g] = (int64_t)f;
            for (size_t c = 0; c < R.children.size(); ++c) acc[c][cidx[v][c][g]] += f;
            R.phi_circ[g] = (int64_t)(f / (u128)R.rpk[g]);
        }
        for (size_t c = 0; c < R.children.size(); ++c) {
            auto &C = p->rel[R.children[c]];
            C.phi_up.resize(C.P);
            for (int64_t k = 0; k < C.P; ++k) {
                if (acc[c][k] % (u128)C.phi_down[k] != 0)
                    return set_error(p, FIGARO_EINVAL, "internal: inexact division in the count queries");
                C.phi_up[k] = (int64_t)(acc[c][k] / (u128)C.phi_down[k]);
            }
        }
    }
    if (p->analyze_only) return FIGARO_OK;
    timer.mark("count queries");
    // ---- subtree columns, scale factors, head/tail tasks
    std::vector<std::vector<int32_t>> subtree_cols(r);
    for (int v : p->post) {
        auto &R = p->rel[v];
        std::vector<int32_t> cols;
        for (int c = 0; c < R.ncols; ++c) cols.push_back(R.col0 + c);
        for (int c : R.children) cols.insert(cols.end(), subtree_cols[c].begin(), subtree_cols[c].end());
        std::sort(cols.begin(), cols.end());
        subtree_cols[v] = cols;
        R.sub_cols = cols;
        R.nsub = (int32_t)cols.size();
        R.own_pos = (int32_t)(std::lower_bound(cols.begin(), cols.end(), R.col0) - cols.begin());
    }
    for (int v : p->post) {
        auto &R = p->rel[v];
        R.a2.variant = p->variant;
        const int tile_a2 = p->tile_items > 0 ? std::min(p->tile_items, tile_items_for(R.ncols, p->variant))
                                              : tile_items_for(R.ncols, p->variant);
        // heads_and_tails of S_v
        if (!R.singleton) {
            R.a2.active = true;
            R.a2.ncols = R.ncols;
            R.a2.block_id = 3 * v + 0;
            for (int c = 0; c < R.ncols; ++c) R.a2.cols.push_back(R.col0 + c);
            std::vector<double> phi(R.G);
            for (int64_t g = 0; g < R.G; ++g) phi[g] = std::sqrt((double)R.phi_circ[g]);
            figaro_status st = build_task(p, R.a2, R.m, R.seg_off, {}, phi, tile_a2);
            if (st != FIGARO_OK) return st;
            if ((st = finish_task(p, R.a2, n)) != FIGARO_OK) return st;
        }
        if (!R.children.empty()) {
            R.col_src.assign(R.nsub, -1);
            R.col_idx.assign(R.nsub, 0);
            for (int c = 0; c < R.ncols; ++c) {
                R.col_src[R.own_pos + c] = -1;
                R.col_idx[R.own_pos + c] = (int16_t)c;
            }
            std::vector<double> own(R.G);
            std::vector<std::vector<double>> mult(R.children.size(), std::vector<double>(R.G));
            for (int64_t g = 0; g < R.G; ++g) {
                u128 prod = 1;
                for (size_t c = 0; c < R.children.size(); ++c)
                    prod *= (u128)p->rel[R.children[c]].phi_down[cidx[v][c][g]];
                own[g] = (double)(int64_t)prod;
                for (size_t c = 0; c < R.children.size(); ++c) {
                    u128 m = (u128)R.rpk[g];
                    for (size_t c2 = 0; c2 < R.children.size(); ++c2)
                        if (c2 != c) m *= (u128)p->rel[R.children[c2]].phi_down[cidx[v][c2][g]];
                    mult[c][g] = (double)(int64_t)m;
                }
            }
            if (dev_upload(p, &R.d_own_mult, own) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            for (size_t c = 0; c < R.children.size(); ++c) {
                int32_t *di;
                double *dm;
                int32_t *dp;
                if (dev_upload(p, &di, cidx[v][c]) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                if (dev_upload(p, &dm, mult[c]) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                std::vector<int32_t> pos;
                for (int32_t col : subtree_cols[R.children[c]])
                    pos.push_back((int32_t)(std::lower_bound(R.sub_cols.begin(), R.sub_cols.end(), col) -
                                            R.sub_cols.begin()));
                if (dev_upload(p, &dp, pos) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                for (size_t q = 0; q < pos.size(); ++q) {
                    R.col_src[pos[q]] = (int16_t)c;
                    R.col_idx[pos[q]] = (int16_t)q;
                }
                R.d_cidx.push_back(di);
                R.d_mult.push_back(dm);
                R.d_colpos.push_back(dp);
            }
            if (R.children.size() > (size_t)kMaxChildren)
                return set_error(p, FIGARO_EUNSUPPORTED, "more than 16 children of one relation");
            // the forward pass reads the joined heads of a relation that
            // projects its join attributes away in place (first head/tail
            // level) when it has at most kFuseMaxChildren children; the
            // backward pass, which reads them twice, stores them
            if (dev_upload(p, &R.d_col_src, R.col_src) != hipSuccess ||
                dev_upload(p, &R.d_col_idx, R.col_idx) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            // (the in-place view carries its column codes by value: at most
            // kMaxCols subtree columns)
            R.fuse_join = R.parent >= 0 && R.P < R.G && R.children.size() <= (size_t)kFuseMaxChildren &&
                          R.nsub <= kMaxCols && !p->separate_join;
            if (R.fuse_join)
                for (int ch : R.children) {
                    double *rm;
                    const auto &C = p->rel[ch];
                    if (dev_alloc(p, (void **)&rm, sizeof(double) * (size_t)C.P * (size_t)C.nsub) != hipSuccess)
                        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                    R.d_sigma_rm.push_back(rm);
                }
            R.ld_s = (R.G + 15) / 16 * 16;
            if (dev_alloc(p, (void **)&R.d_s, sizeof(double) * (size_t)R.nsub * (size_t)R.ld_s) != hipSuccess ||
                dev_alloc(p, (void **)&R.d_gs, sizeof(double) * (size_t)R.nsub * (size_t)R.G) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            // inverse of the child index: parent key groups grouped by child group
            for (size_t c = 0; c < R.children.size(); ++c) {
                const int64_t Pc = p->rel[R.children[c]].P;
                std::vector<int64_t> off(Pc + 1, 0);
                for (int64_t g = 0; g < R.G; ++g) off[cidx[v][c][g] + 1]++;
                for (int64_t q = 0; q < Pc; ++q) off[q + 1] += off[q];
                std::vector<int32_t> idx(R.G);
                std::vector<int64_t> pos(off.begin(), off.end() - 1);
                for (int64_t g = 0; g < R.G; ++g) idx[pos[cidx[v][c][g]]++] = (int32_t)g;
                int64_t *doff;
                int32_t *didx;
                if (dev_upload(p, &doff, off) != hipSuccess || dev_upload(p, &didx, idx) != hipSuccess)
                    return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                R.d_inv_off.push_back(doff);
                R.d_inv_idx.push_back(didx);
                if (figaro_status st = join_chunks(p, R, c, off); st != FIGARO_OK) return st;
            }
            if (R.parent >= 0 && R.P < R.G) {
                R.a4.active = true;
                R.a4.ncols = R.nsub;
                R.a4.block_id = 3 * v + 1;
                R.a4.cols = R.sub_cols;
                std::vector<double> phi(R.P);
                for (int64_t q = 0; q < R.P; ++q) phi[q] = std::sqrt((double)R.phi_up[q]);
                R.a4.variant = p->variant;
                const int tile_a4 = p->tile_items > 0 ? std::min(p->tile_items, tile_items_for(R.nsub, p->variant))
                                                      : tile_items_for(R.nsub, p->variant);
                figaro_status st = build_task(p, R.a4, R.G, R.par_off, R.theta, phi, tile_a4);
                if (st != FIGARO_OK) return st;
                if ((st = finish_task(p, R.a4, n)) != FIGARO_OK) return st;
            }
        }
        if (R.parent < 0) {
            std::vector<double> isc(R.G);
            for (int64_t g = 0; g < R.G; ++g) isc[g] = 1.0 / std::sqrt((double)R.theta[g]);
            if (dev_upload(p, &R.d_inv_sqrt_c, isc) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        }
    }
    timer.mark("tasks and uploads");
    return finish_plan(p);
}

}  // namespace

figaro_status finish_plan(figaro_plan_s *p) {
    const int32_t n = p->n;
    // the arrays the join-row enumeration reads: a host-built plan copies its
    // offsets and counts over (a device-built plan has them there)
    if (!p->device_plan) {
        for (auto &R : p->rel) {
            if (dev_upload(p, &R.d_seg_off, R.seg_off) != hipSuccess || dev_upload(p, &R.d_theta, R.theta) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            if (R.parent >= 0 && (dev_upload(p, &R.d_par_off, R.par_off) != hipSuccess ||
                                  dev_upload(p, &R.d_phi_down, R.phi_down) != hipSuccess))
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        }
    }
    if (figaro_status st = enumeration_arrays(p, 0); st != FIGARO_OK) return st;
    // ---- stack rows (fused R's of every launch, then the root rows) and R0 rows
    // Wide plans keep the stack's first n rows for the R's of their wide
    // heads_and_tails tasks, whose tails go to regions of their own.
    int64_t srow = p->wide ? n : 0, r0row = 0;
    std::vector<Task *> regions;
    int64_t region_doubles = 0;
    for (int v : p->post) {
        auto &R = p->rel[v];
        for (Task *T : {&R.a2, &R.a4}) {
            if (!T->active) continue;
            const bool region = p->wide && T == &R.a2 && T->ncols > kFusedMaxCols;
            int64_t rrow = 0;
            for (auto &L : T->levels) {
                if (region) {
                    L.stack_row0 = rrow;
                    rrow += L.items;
                } else {
                    L.stack_row0 = srow;
                    // the first level folds its tails into one R per
                    // workgroup; the upper levels hold few rows and append
                    // their tails as is, and so do all levels of a wide task
                    if (&L == &T->levels[0] && T->ncols <= kFusedMaxCols)
                        srow += (int64_t)((L.waves + waves_per_block() - 1) / waves_per_block()) * T->ncols;
                    else
                        srow += L.items;
                }
                L.r0_row0 = r0row;
                r0row += L.items;
            }
            if (region) {
                T->region_ld = std::max<int64_t>(rrow, 1);
                region_doubles += T->region_ld * T->ncols;
                regions.push_back(T);
            }
        }
        if (R.parent < 0) {
            R.root_row0 = srow;
            srow += R.G;
            R.r0_root_row0 = r0row;
            r0row += R.G;
        }
    }
    p->stack_rows = srow;
    p->r0_rows = r0row;
    // device column tables of the wide tasks (their chunks share a launch)
    for (auto &R : p->rel)
        for (Task *T : {&R.a2, &R.a4}) {
            if (!T->active || T->ncols <= kFusedMaxCols) continue;
            std::vector<uint16_t> c16(T->cols.begin(), T->cols.end());
            if (dev_upload(p, &T->d_cols16, c16) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        }
    if (p->wide) {
        // workspaces: the final QR's, then one per region (their panels
        // share launches, so each keeps its reflectors apart)
        const int64_t final_rows = wide_qr_panel_rows(srow, n, true);
        int64_t ws_doubles = wide_qr_workspace_doubles(final_rows, n);
        for (Task *T : regions)
            ws_doubles += wide_qr_workspace_doubles(wide_qr_panel_rows(T->region_ld, T->ncols, false), T->ncols);
        p->stack_ld[0] = std::max<int64_t>(srow, 1);
        double *ws = nullptr, *reg = nullptr;
        if (dev_alloc(p, (void **)&p->d_stack[0], sizeof(double) * (size_t)n * (size_t)p->stack_ld[0]) !=
                hipSuccess ||
            dev_alloc(p, (void **)&reg, sizeof(double) * (size_t)region_doubles) != hipSuccess ||
            dev_alloc(p, (void **)&ws, sizeof(double) * (size_t)ws_doubles) != hipSuccess ||
            dev_alloc(p, (void **)&p->d_status, sizeof(int32_t) * 4) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        std::string err;
        if (figaro_status st = wide_qr_init(p->wqr, ws, final_rows, n, nullptr, err); st != FIGARO_OK)
            return set_error(p, st, err);
        ws += wide_qr_workspace_doubles(final_rows, n);
        p->region_qr.resize(regions.size());
        for (size_t q = 0; q < regions.size(); ++q) {
            Task *T = regions[q];
            T->d_region = reg;
            reg += T->region_ld * T->ncols;
            const int64_t rows = wide_qr_panel_rows(T->region_ld, T->ncols, false);
            if (figaro_status st = wide_qr_init(p->region_qr[q], ws, rows, T->ncols, p->wqr.blas, err);
                st != FIGARO_OK)
                return set_error(p, st, err);
            ws += wide_qr_workspace_doubles(rows, T->ncols);
        }
        return FIGARO_OK;
    }
    // dense TSQR levels over the stack: a workgroup folds tiles_per_wave
    // steps of wpb tiles (wpb waves on separate tiles; one shared tile for
    // n > 16) into one R of n rows, so each level divides the rows by
    // at least 4
    const int64_t dt = dense_tile_rows_for(n, p->variant);
    const int64_t wpb = dense_waves_per_block(n);
    const int64_t step_rows = wpb * dt;
    const bool wide = n > kFusedMaxCols;
    // n <= 16: one tile per wave at every level (each level costs the
    // latency of two tile steps, data then merge), and a last level of at
    // most one tile per wave; a last level of one tile needs no merge at all.
    // Shared tiles (n > 16): the same, one shared step per level, as long
    // as a tile holds at least 2.7 R's worth of rows (512-row tiles up to 64
    // columns, 256-row tiles up to 96); with 256-row tiles of more than 96
    // columns two steps per level, so that a level still quarters the rows.
    // (A level of t steps shrinks the rows t*tile/n-fold; the chain of
    // dependent tile steps is shortest where t / log(t*tile/n) is least.)
    const int64_t mid_tpw = (wide && n > 96) ? 2 : 1, final_tiles = mid_tpw;
    int64_t rows = srow;
    int64_t maxnext = 0;
    while (true) {
        DenseLevel D;
        D.rows = rows;
        if (rows <= final_tiles * step_rows) {
            D.waves = 1;
            D.tiles_per_wave = std::max<int64_t>(1, (rows + step_rows - 1) / step_rows);
            p->dense.push_back(D);
            break;
        }
        D.tiles_per_wave = mid_tpw;
        D.waves = (int32_t)((rows + mid_tpw * step_rows - 1) / (mid_tpw * step_rows));
        p->dense.push_back(D);
        rows = (int64_t)D.waves * n;
        maxnext = std::max(maxnext, rows);
    }
    if (dev_alloc(p, (void **)&p->d_K, sizeof(double) * (size_t)n * (size_t)n) != hipSuccess ||
        dev_alloc(p, (void **)&p->d_W, sizeof(double) * (size_t)n * (size_t)n) != hipSuccess ||
        dev_alloc(p, (void **)&p->d_status, sizeof(int32_t) * 4) != hipSuccess)
        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    p->stack_ld[0] = std::max<int64_t>(srow, 1);
    p->stack_ld[1] = std::max<int64_t>(maxnext, 1);
    if (dev_alloc(p, (void **)&p->d_stack[0], sizeof(double) * (size_t)n * (size_t)p->stack_ld[0]) != hipSuccess ||
        dev_alloc(p, (void **)&p->d_stack[1], sizeof(double) * (size_t)n * (size_t)p->stack_ld[1]) != hipSuccess)
        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    return FIGARO_OK;
}

}  // namespace figaro

using namespace figaro;

extern "C" {

figaro_status figaro_plan_create(figaro_plan_t *out, int32_t r, const figaro_relation_desc *rels,
                                 const figaro_plan_options *opts, hipStream_t stream) {
    if (!out) return set_error(nullptr, FIGARO_EINVAL, "out is NULL");
    *out = nullptr;
    if (r < 1 || !rels) return set_error(nullptr, FIGARO_EINVAL, "need at least one relation");
    figaro_plan_s *p = new figaro_plan_s();
    if (!(opts && opts->keys_on_host && opts->analyze_only)) (void)hipGetDevice(&p->device);
    figaro_status st;
    try {
        st = build(p, r, rels, opts, stream);
    } catch (const std::bad_alloc &) {
        st = set_error(p, FIGARO_ENOMEM, "host allocation failed");
    } catch (...) {
        st = set_error(p, FIGARO_EINVAL, "unexpected error while building the plan");
    }
    if (st != FIGARO_OK) {
        std::string msg = p->last_error;
        figaro_plan_destroy(p);
        g_thread_error = msg;
        return st;
    }
    *out = p;
    return FIGARO_OK;
}

void figaro_plan_destroy(figaro_plan_t p) {
    if (!p) return;
    for (auto e : p->prof_start) (void)hipEventDestroy(e);
    for (auto e : p->prof_stop) (void)hipEventDestroy(e);
    wide_qr_release(p->wqr);
    for (void *a : p->allocations) (void)hipFree(a);
    delete p;
}

int32_t figaro_plan_num_relations(figaro_plan_t p) { return p ? p->r : -1; }
int32_t figaro_plan_num_cols(figaro_plan_t p) { return p ? p->n : -1; }
int64_t figaro_plan_input_rows(figaro_plan_t p, int32_t i) {
    return (p && i >= 0 && i < p->r) ? p->rel[i].m_in : -1;
}
int64_t figaro_plan_rows(figaro_plan_t p, int32_t i) { return (p && i >= 0 && i < p->r) ? p->rel[i].m : -1; }
int64_t figaro_plan_dropped_rows(figaro_plan_t p, int32_t i) {
    return (p && i >= 0 && i < p->r) ? p->rel[i].m_in - p->rel[i].m : -1;
}
double figaro_plan_join_rows(figaro_plan_t p) { return p ? p->join_rows : -1.0; }
int64_t figaro_plan_workspace_bytes(figaro_plan_t p) { return p ? p->workspace_bytes : -1; }

figaro_status figaro_plan_permutation(figaro_plan_t p, int32_t i, int64_t *perm) {
    if (!p || i < 0 || i >= p->r || !perm) return set_error(p, FIGARO_EINVAL, "bad argument");
    if (figaro_status st = fetch_host_arrays(p, i); st != FIGARO_OK) return st;
    std::memcpy(perm, p->rel[i].perm.data(), sizeof(int64_t) * p->rel[i].perm.size());
    return FIGARO_OK;
}

int64_t figaro_plan_num_groups(figaro_plan_t p, int32_t i, int32_t which) {
    if (!p || i < 0 || i >= p->r) return -1;
    return which == 0 ? p->rel[i].G : (which == 1 ? p->rel[i].P : -1);
}

figaro_status figaro_plan_group_first_rows(figaro_plan_t p, int32_t i, int32_t which, int64_t *out) {
    if (!p || i < 0 || i >= p->r || !out || (which != 0 && which != 1))
        return set_error(p, FIGARO_EINVAL, "bad argument");
    if (figaro_status st = fetch_host_arrays(p, i); st != FIGARO_OK) return st;
    const auto &R = p->rel[i];
    if (which == 0) {
        for (int64_t g = 0; g < R.G; ++g) out[g] = R.perm[R.seg_off[g]];
    } else {
        for (int64_t q = 0; q < R.P; ++q) out[q] = R.perm[R.seg_off[R.par_off[q]]];
    }
    return FIGARO_OK;
}

figaro_status figaro_plan_counts(figaro_plan_t p, int32_t i, figaro_count_kind kind, int64_t *out) {
    if (!p || i < 0 || i >= p->r || !out) return set_error(p, FIGARO_EINVAL, "bad argument");
    if (figaro_status st = fetch_host_arrays(p, i); st != FIGARO_OK) return st;
    const auto &R = p->rel[i];
    const std::vector<int64_t> *v = nullptr;
    switch (kind) {
        case FIGARO_COUNT_ROWS_PER_KEY: v = &R.rpk; break;
        case FIGARO_COUNT_THETA_DOWN: v = &R.theta; break;
        case FIGARO_COUNT_PHI_CIRC: v = &R.phi_circ; break;
        case FIGARO_COUNT_PHI_UP: v = &R.phi_up; break;
        case FIGARO_COUNT_PHI_DOWN: v = &R.phi_down; break;
        default: return set_error(p, FIGARO_EINVAL, "unknown count kind");
    }
    if (R.parent < 0 && (kind == FIGARO_COUNT_PHI_UP || kind == FIGARO_COUNT_PHI_DOWN))
        return set_error(p, FIGARO_EINVAL, "the root has no parent groups");
    std::memcpy(out, v->data(), sizeof(int64_t) * v->size());
    return FIGARO_OK;
}

const char *figaro_last_error(figaro_plan_t p) {
    if (p) return p->last_error.c_str();
    return g_thread_error.c_str();
}

}  // extern "C"
