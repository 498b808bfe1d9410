// Launch sequence of the forward pass: post-order over the join tree
// (Algorithm 3), then the post-processing TSQR over the stack of partial R's.
// Everything is enqueued on the caller's stream; nothing is allocated and the
// host is never synchronised.
#include <string>

#include <algorithm>

#include "internal.hpp"
#include "bwd_batch.hpp"
#include "../../include/figaro_debug.h"

namespace figaro {
figaro_status set_error(figaro_plan_s *p, figaro_status st, const std::string &msg);
}

using namespace figaro;

namespace {

#define FIGARO_TRY(expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return set_error(p, FIGARO_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Timing of one launch when profiling is enabled (no-op otherwise).
struct ProfScope {
    figaro_plan_s *p;
    hipStream_t s;
    int slot = -1;
    int kind;
    double bytes, flops;
    ProfScope(figaro_plan_s *p_, hipStream_t s_, int kind_, double bytes_, double flops_)
        : p(p_), s(s_), kind(kind_), bytes(bytes_), flops(flops_) {
        if (p->prof_next < p->prof_start.size()) {
            slot = (int)p->prof_next++;
            if (hipEventRecord(p->prof_start[slot], s) != hipSuccess) slot = -1;
        }
    }
    ~ProfScope() {
        if (slot >= 0 && hipEventRecord(p->prof_stop[slot], s) == hipSuccess)
            p->prof_pending.push_back({kind, slot, bytes, flops});
    }
};

// Bit g of the two words: global column g (< n) is not one of `cols`.
// Wide plans (n > kMaxCols) clear their stack before every pass instead.
void set_other_cols(uint64_t (&w)[2], int n, const std::vector<int32_t> &cols) {
    w[0] = w[1] = 0;
    if (n > kMaxCols) return;
    for (int g = 0; g < n; ++g) w[g >> 6] |= 1ull << (g & 63);
    for (int32_t c : cols) w[c >> 6] &= ~(1ull << (c & 63));
}

struct Buffers {
    // per relation: own sums (key groups) and sigma (parent groups)
    std::vector<const double *> own;
    std::vector<int64_t> ld_own;
    std::vector<const double *> sigma;
    std::vector<int64_t> ld_sigma;
};

figaro_status check_inputs(figaro_plan_s *p, const double *const *values, const int64_t *ld) {
    if (p->analyze_only) return set_error(p, FIGARO_EINVAL, "the plan was built with analyze_only");
    if (!values || !ld) return set_error(p, FIGARO_EINVAL, "values/ld is NULL");
    for (int i = 0; i < p->r; ++i) {
        if (!values[i]) return set_error(p, FIGARO_EINVAL, "values[" + std::to_string(i) + "] is NULL");
        if (ld[i] < p->rel[i].m)
            return set_error(p, FIGARO_EINVAL, "ld[" + std::to_string(i) + "] is smaller than the plan rows");
    }
    return FIGARO_OK;
}

// The joined heads of relation v read in place (its first project-away
// level fused with process_and_join_children).
JoinSrc join_src(const figaro_plan_s *p, const RelPlan &Rl, int v, const Buffers &B) {
    JoinSrc js{};
    js.own = B.own[v];
    js.ld_own = B.ld_own[v];
    js.own_mult = Rl.d_own_mult;
    js.nchildren = (int32_t)Rl.children.size();
    for (size_t c = 0; c < Rl.children.size(); ++c) {
        js.sigma[c] = Rl.d_sigma_rm[c];
        js.ld_sigma[c] = p->rel[Rl.children[c]].nsub;
        js.cidx[c] = Rl.d_cidx[c];
        js.mult[c] = Rl.d_mult[c];
    }
    for (int c = 0; c < Rl.nsub && c < kMaxCols; ++c)
        js.code[c] = ((int32_t)Rl.col_src[c] + 1) << 8 | (uint8_t)Rl.col_idx[c];
    return js;
}

// Arguments of level li of head/tail task T reading its items from cur
// (ld); fold: the level folds its tails into workgroup R's (the first level
// of a fused narrow task).  With js, the first level reads its items
// through the join view.
HelmertArgs level_args(figaro_plan_s *p, Task &T, size_t li, const double *cur, int64_t ld, bool fuse, double *r0,
                       int64_t ld_r0, int32_t *block_of_row, const JoinSrc *js, bool &fold) {
    const Level &L = T.levels[li];
    // the tails of a wide plan's wide heads_and_tails task go to its region,
    // in the task's own columns
    const bool region = fuse && T.d_region != nullptr;
    const bool wide = T.ncols > kFusedMaxCols;
    HelmertArgs a{};
    a.in = cur;
    a.ld_in = ld;
    if (js && li == 0) {
        a.join = 1;
        a.js = *js;
    }
    a.ncols = T.ncols;
    a.items = L.items;
    a.pid = L.d_pid;
    a.piece_start = L.d_piece_start;
    a.phi_piece = L.d_phi_piece;
    a.alpha = L.d_alpha;
    a.beta = L.d_beta;
    a.chunk_start = L.d_chunk_start;
    a.chunk_piece0 = L.d_chunk_piece0;
    a.nchunks = L.nchunks;
    a.pieces_out = L.d_pieces;
    a.ld_pieces = L.npieces;
    a.stack = p->d_stack[0];
    a.ld_stack = p->stack_ld[0];
    a.stack_row0 = L.stack_row0;
    a.n_total = p->n;
    set_other_cols(a.other_cols, p->n, T.cols);
    if (!wide)
        for (int c = 0; c < T.ncols; ++c) a.colmap[c] = (uint16_t)T.cols[c];
    // upper levels of the fused pass write their tail rows into the
    // stack, and so do all levels of a wide task
    fold = fuse && li == 0 && !wide;
    const bool to_stack = fuse && !fold;
    a.r0 = to_stack ? (region ? T.d_region : p->d_stack[0]) : r0;
    a.ld_r0 = to_stack ? (region ? T.region_ld : p->stack_ld[0]) : ld_r0;
    a.r0_row0 = to_stack ? L.stack_row0 : L.r0_row0;
    if (fold && !r0) a.r0 = nullptr;
    a.block_of_row = to_stack ? nullptr : block_of_row;
    a.block_id = T.block_id;
    a.waves = L.waves;
    if (wide) {
        // column chunks, all in one launch: the tails of every column
        // depend on that column only; the first chunk also writes the
        // zeros of the columns outside the task
        a.in = a.join ? nullptr : cur;
        a.join_col0 = 0;
        a.ncols = kChunkCols;
        a.wide_cols = T.ncols;
        a.cols_ident = region ? 1 : 0;
        a.wide_colmap = T.d_cols16;
    }
    return a;
}

// One level of a head/tail task on its own.
figaro_status launch_level(figaro_plan_s *p, Task &T, size_t li, const HelmertArgs &a, bool fold, hipStream_t s) {
    const Level &L = T.levels[li];
    if (T.ncols > kFusedMaxCols && !T.d_cols16)
        return set_error(p, FIGARO_EINVAL, "wide task without a device column table");
    const int kind = li > 0 ? 2 : (L.unit ? 0 : 1);
    const double bytes = 8.0 * (double)L.items * T.ncols;
    const double flops = fold ? 2.0 * (double)L.items * T.ncols * T.ncols : 0.0;
    ProfScope ps(p, s, kind, bytes, flops);
    FIGARO_TRY(launch_helmert(a, L.unit, fold, L.variant, s));
    return FIGARO_OK;
}

// Run the levels of one head/tail task; returns the group sums.  With js,
// the first level reads its items through the join view (in is unused).
figaro_status run_task(figaro_plan_s *p, Task &T, const double *in, int64_t ld_in, bool fuse, double *r0,
                       int64_t ld_r0, int32_t *block_of_row, hipStream_t s, const double **group_sums,
                       int64_t *ld_groups, const JoinSrc *js = nullptr) {
    const double *cur = in;
    int64_t ld = ld_in;
    for (size_t li = 0; li < T.levels.size(); ++li) {
        bool fold = false;
        const HelmertArgs a = level_args(p, T, li, cur, ld, fuse, r0, ld_r0, block_of_row, js, fold);
        if (figaro_status st = launch_level(p, T, li, a, fold, s); st != FIGARO_OK) return st;
        cur = T.levels[li].d_pieces;
        ld = T.levels[li].npieces;
    }
    *group_sums = cur;
    *ld_groups = ld;
    return FIGARO_OK;
}

// heads_and_tails of every relation (they read the relation's own values
// only, so they are independent of each other and of the joins): level by
// level over all tasks, the same level of tasks of one tile shape sharing
// launches (upper levels are small and bound by latency; first levels that
// each fill the chip overlap one task's last tiles with the next one's
// first).  Leaves each relation's key-group sums in B.own.
figaro_status run_heads_and_tails(figaro_plan_s *p, const double *const *values, const int64_t *ld, bool fuse,
                                  double *r0, int64_t ld_r0, int32_t *block_of_row, hipStream_t s, Buffers &B) {
    std::vector<int> tasks;
    size_t levels = 0;
    for (int v : p->post) {
        B.own[v] = values[v];
        B.ld_own[v] = ld[v];
        if (p->rel[v].a2.active) {
            tasks.push_back(v);
            levels = std::max(levels, p->rel[v].a2.levels.size());
        }
    }
    struct Open {
        int shape, variant;
        bool unit, fold;
        HelmertBatch b;
        double bytes, flops;
    };
    for (size_t li = 0; li < levels; ++li) {
        std::vector<Open> open;
        auto flush = [&](Open &o) -> figaro_status {
            if (o.b.count == 0) return FIGARO_OK;
            ProfScope ps(p, s, li > 0 ? 2 : (o.unit ? 0 : 1), o.bytes, o.flops);
            FIGARO_TRY(launch_helmert_batch(o.b, o.unit, o.fold, o.variant, s));
            o.b.count = 0;
            o.b.wg0[0] = 0;
            o.bytes = o.flops = 0.0;
            return FIGARO_OK;
        };
        for (int v : tasks) {
            Task &T = p->rel[v].a2;
            if (li >= T.levels.size()) continue;
            const Level &L = T.levels[li];
            bool fold = false;
            const HelmertArgs a =
                level_args(p, T, li, B.own[v], B.ld_own[v], fuse, r0, ld_r0, block_of_row, nullptr, fold);
            if (T.ncols > kFusedMaxCols || L.waves <= 0 || L.nchunks <= 0) {
                if (figaro_status st = launch_level(p, T, li, a, fold, s); st != FIGARO_OK) return st;
            } else {
                const int shape = helmert_shape_class(T.ncols);
                size_t k = 0;
                while (k < open.size() && !(open[k].shape == shape && open[k].variant == L.variant &&
                                            open[k].unit == L.unit && open[k].fold == fold))
                    ++k;
                if (k == open.size()) open.push_back(Open{shape, L.variant, L.unit, fold, HelmertBatch{}, 0.0, 0.0});
                Open &o = open[k];
                o.b.a[o.b.count] = a;
                o.b.wg0[o.b.count + 1] = o.b.wg0[o.b.count] + (L.waves + waves_per_block() - 1) / waves_per_block();
                ++o.b.count;
                o.bytes += 8.0 * (double)L.items * T.ncols;
                o.flops += fold ? 2.0 * (double)L.items * T.ncols * T.ncols : 0.0;
                if (o.b.count == kHelmertBatch)
                    if (figaro_status st = flush(o); st != FIGARO_OK) return st;
            }
            B.own[v] = L.d_pieces;
            B.ld_own[v] = L.npieces;
        }
        for (Open &o : open)
            if (figaro_status st = flush(o); st != FIGARO_OK) return st;
    }
    return FIGARO_OK;
}

// Post-processing of a wide plan: the R of every region onto the diagonal
// of the stack's first n rows, then the QR of the whole stack, whose first
// n rows are upper triangular (triangular-pentagonal form).
figaro_status wide_post(figaro_plan_s *p, double *R, hipStream_t s) {
    const int32_t n = p->n;
    std::string err;
    // the regions side by side (in post order, as their workspaces)
    std::vector<WideQrJob> jobs;
    std::vector<Task *> tasks;
    double flops = 0.0, bytes = 0.0;
    for (int v : p->post) {
        Task &T = p->rel[v].a2;
        if (!T.active || !T.d_region) continue;
        const double h = (double)T.region_ld, c = T.ncols;
        jobs.push_back({&p->region_qr[tasks.size()], T.d_region, T.region_ld, T.region_ld, T.ncols, false});
        tasks.push_back(&T);
        flops += 2.0 * h * c * c - 2.0 / 3.0 * c * c * c;
        bytes += 8.0 * h * c;
    }
    if (!jobs.empty()) {
        ProfScope ps(p, s, 5, bytes, flops);
        figaro_status st = wide_qr_many(jobs, s, err);
        if (st != FIGARO_OK) return set_error(p, st, err);
    }
    for (Task *T : tasks)
        FIGARO_TRY(launch_copy_upper(T->d_region, T->region_ld, T->region_ld, T->ncols, p->d_stack[0],
                                     p->stack_ld[0], T->cols[0], T->cols[0], s));
    {
        const double g = (double)(p->stack_rows - n);
        ProfScope ps(p, s, 5, 8.0 * (double)p->stack_rows * n, 2.0 * g * n * (double)n);
        figaro_status st =
            wide_qr_many({{&p->wqr, p->d_stack[0], p->stack_ld[0], p->stack_rows, n, true}}, s, err);
        if (st != FIGARO_OK) return set_error(p, st, err);
    }
    FIGARO_TRY(launch_final_r(p->d_stack[0], p->stack_ld[0], n, n, R, s));
    return FIGARO_OK;
}

figaro_status forward(figaro_plan_s *p, const double *const *values, const int64_t *ld, bool fuse, double *R,
                      double *r0, int64_t ld_r0, int32_t *block_of_row, hipStream_t s, bool stop_before_tsqr = false,
                      Buffers *keep = nullptr) {
    // produce-only mode (fuse false, r0 null): piece sums and joined heads only.
    // The joined heads are read in place (fused relations) except when the
    // pass recomputes them for the backward pass (keep), which reads them
    // again and wants them stored.
    const bool join_in_place = keep == nullptr;
    if (p->wide && fuse) {
        // tasks write their columns only: the rest of the stack is zero
        ProfScope ps(p, s, 5, 8.0 * (double)p->stack_rows * p->n, 0.0);
        FIGARO_TRY(launch_fill(p->d_stack[0], (int64_t)p->n * p->stack_ld[0], 0.0, s));
    }
    Buffers B;
    B.own.assign(p->r, nullptr);
    B.ld_own.assign(p->r, 0);
    B.sigma.assign(p->r, nullptr);
    B.ld_sigma.assign(p->r, 0);
    // heads_and_tails: own key-group sums and the tails of every S_v
    if (figaro_status st = run_heads_and_tails(p, values, ld, fuse, r0, ld_r0, block_of_row, s, B); st != FIGARO_OK)
        return st;
    for (int v : p->post) {
        RelPlan &Rl = p->rel[v];
        const double *items = B.own[v];
        int64_t ld_items = B.ld_own[v];
        const bool in_place = Rl.fuse_join && join_in_place;
        if (!Rl.children.empty() && !in_place) {
            // process_and_join_children
            JoinArgs j{};
            j.groups = Rl.G;
            j.nsub = Rl.nsub;
            j.s = Rl.d_s;
            j.ld_s = Rl.ld_s;
            j.own = B.own[v];
            j.ld_own = B.ld_own[v];
            j.own_cols = Rl.ncols;
            j.own_pos = Rl.own_pos;
            j.own_mult = Rl.d_own_mult;
            j.nchildren = (int32_t)Rl.children.size();
            j.col_src = Rl.d_col_src;
            j.col_idx = Rl.d_col_idx;
            for (size_t c = 0; c < Rl.children.size(); ++c) {
                int ch = Rl.children[c];
                j.sigma[c] = B.sigma[ch];
                j.ld_sigma[c] = B.ld_sigma[ch];
                j.child_cols[c] = p->rel[ch].nsub;
                j.colpos[c] = Rl.d_colpos[c];
                j.cidx[c] = Rl.d_cidx[c];
                j.mult[c] = Rl.d_mult[c];
            }
            {
                ProfScope ps(p, s, 3, 8.0 * (double)Rl.G * (Rl.ncols + 2.0 * Rl.nsub), 0.0);
                FIGARO_TRY(launch_join(j, s));
            }
            items = Rl.d_s;
            ld_items = Rl.ld_s;
        }
        if (Rl.parent >= 0) {
            // project_away_join_attributes (only non-leaves with P < G have tails)
            if (Rl.a4.active) {
                JoinSrc js;
                if (in_place) {
                    // the children's sums, row-major
                    for (size_t c = 0; c < Rl.children.size(); ++c) {
                        const int ch = Rl.children[c];
                        FIGARO_TRY(launch_rowmajor(B.sigma[ch], B.ld_sigma[ch], p->rel[ch].P, p->rel[ch].nsub,
                                                   Rl.d_sigma_rm[c], s));
                    }
                    js = join_src(p, Rl, v, B);
                }
                figaro_status st = run_task(p, Rl.a4, items, ld_items, fuse, r0, ld_r0, block_of_row, s,
                                            &B.sigma[v], &B.ld_sigma[v], in_place ? &js : nullptr);
                if (st != FIGARO_OK) return st;
            } else {
                B.sigma[v] = items;
                B.ld_sigma[v] = ld_items;
            }
        } else if (fuse || r0) {
            RootArgs ra{};
            ra.groups = Rl.G;
            ra.n = p->n;
            ra.s = items;
            ra.ld_s = ld_items;
            ra.inv_sqrt_c = Rl.d_inv_sqrt_c;
            ra.dst = fuse ? p->d_stack[0] : r0;
            ra.ld_dst = fuse ? p->stack_ld[0] : ld_r0;
            ra.row0 = fuse ? Rl.root_row0 : Rl.r0_root_row0;
            ra.block_of_row = fuse ? nullptr : block_of_row;
            ra.block_id = 3 * v + 2;
            {
                ProfScope ps(p, s, 4, 16.0 * (double)Rl.G * p->n, 0.0);
                FIGARO_TRY(launch_root(ra, !fuse, s));
            }
        }
    }
    if (keep) *keep = B;
    if (!fuse || stop_before_tsqr) return FIGARO_OK;
    if (p->wide) return wide_post(p, R, s);
    // post-processing TSQR over the stack
    int cur = 0;
    for (size_t d = 0; d < p->dense.size(); ++d) {
        const DenseLevel &D = p->dense[d];
        DenseArgs a{};
        a.in = p->d_stack[cur];
        a.ld_in = p->stack_ld[cur];
        a.rows = D.rows;
        a.n = p->n;
        a.out = p->d_stack[1 - cur];
        a.ld_out = p->stack_ld[1 - cur];
        a.waves = D.waves;
        a.tiles_per_wave = D.tiles_per_wave;
        a.final_r = R;
        {
            ProfScope ps(p, s, 5, 8.0 * (double)D.rows * p->n, 2.0 * (double)D.rows * p->n * p->n);
            FIGARO_TRY(launch_dense(a, p->variant, s));
        }
        cur = 1 - cur;
    }
    return FIGARO_OK;
}

// Where a gradient goes: column-major [cols][ld] unless rowmajor ([rows][ld]).
// The gradients of the joined heads (d_gs) are row-major, which keeps the
// gathers of the join's adjoint within one row per key group.
struct Target {
    double *p;
    int64_t ld;
    bool rowmajor = false;
};

// Where the gradient of the key-group sums of relation v goes: the top level
// of its heads_and_tails task, or the caller's value gradient if every key
// group has one row.
Target own_grad_target(figaro_plan_s *p, int v, double *const *dvalues, const int64_t *ld_dv) {
    RelPlan &R = p->rel[v];
    if (R.a2.active) return {R.a2.levels.back().d_gpieces, R.a2.levels.back().npieces};
    return {dvalues[v], ld_dv[v]};
}

// Where the gradient of sigma_v (what relation v hands to its parent) goes.
Target sigma_grad_target(figaro_plan_s *p, int v, double *const *dvalues, const int64_t *ld_dv) {
    RelPlan &R = p->rel[v];
    if (R.children.empty()) return own_grad_target(p, v, dvalues, ld_dv);
    if (R.a4.active) return {R.a4.levels.back().d_gpieces, R.a4.levels.back().npieces};
    return {R.d_gs, R.nsub, true};
}

// Backward of the levels of one task, top level first; level 0 writes the
// gradient of the task's items to `out`.
figaro_status run_task_bwd(figaro_plan_s *p, Task &T, const double *in, int64_t ld_in, Target out, hipStream_t s) {
    for (int l = (int)T.levels.size() - 1; l >= 0; --l) {
        Level &L = T.levels[l];
        HelmertBwdArgs a{};
        a.in = (l == 0) ? in : T.levels[l - 1].d_pieces;
        a.ld_in = (l == 0) ? ld_in : T.levels[l - 1].npieces;
        a.ncols = T.ncols;
        a.pid = L.d_pid;
        a.piece_start = L.d_piece_start;
        a.phi_piece = L.d_phi_piece;
        a.alpha = L.d_alpha;
        a.beta = L.d_beta;
        a.chunk_start = L.d_chunk_start;
        a.nchunks = L.nchunks;
        a.K = p->d_K;
        a.n_total = p->n;
        for (int c = 0; c < T.ncols; ++c) a.colmap[c] = (uint8_t)T.cols[c];
        a.gpieces = L.d_gpieces;
        a.ld_gp = L.npieces;
        a.gout = (l == 0) ? out.p : T.levels[l - 1].d_gpieces;
        a.ld_gout = (l == 0) ? out.ld : T.levels[l - 1].npieces;
        a.gout_rowmajor = (l == 0 && out.rowmajor) ? 1 : 0;
        a.waves = (int32_t)std::min<int64_t>(L.nchunks, 8192);
        ProfScope ps(p, s, 6, 8.0 * (double)L.items * T.ncols * 2.0, 2.0 * (double)L.items * T.ncols * T.ncols);
        FIGARO_TRY(launch_helmert_bwd(a, L.unit, s));
    }
    return FIGARO_OK;
}

// Arguments of the backward of level l of task T (items of level 0: in).
HelmertBwdArgs level_bwd_args(figaro_plan_s *p, Task &T, int l, const double *in, int64_t ld_in, Target out) {
    Level &L = T.levels[l];
    HelmertBwdArgs a{};
    a.in = (l == 0) ? in : T.levels[l - 1].d_pieces;
    a.ld_in = (l == 0) ? ld_in : T.levels[l - 1].npieces;
    a.ncols = T.ncols;
    a.pid = L.d_pid;
    a.piece_start = L.d_piece_start;
    a.phi_piece = L.d_phi_piece;
    a.alpha = L.d_alpha;
    a.beta = L.d_beta;
    a.chunk_start = L.d_chunk_start;
    a.nchunks = L.nchunks;
    a.K = p->d_K;
    a.n_total = p->n;
    for (int c = 0; c < T.ncols; ++c) a.colmap[c] = (uint8_t)T.cols[c];
    a.gpieces = L.d_gpieces;
    a.ld_gp = L.npieces;
    a.gout = (l == 0) ? out.p : T.levels[l - 1].d_gpieces;
    a.ld_gout = (l == 0) ? out.ld : T.levels[l - 1].npieces;
    a.gout_rowmajor = (l == 0 && out.rowmajor) ? 1 : 0;
    a.waves = (int32_t)std::min<int64_t>(L.nchunks, 8192);
    return a;
}

// Backward of every relation's heads_and_tails task (step r: level
// levels - 1 - r of each task that has it), the same step of tasks of one
// shape class and count mode in shared launches.
figaro_status run_heads_and_tails_bwd(figaro_plan_s *p, const double *const *values, const int64_t *ld,
                                      double *const *dvalues, const int64_t *ld_dv, hipStream_t s) {
    std::vector<int> tasks;
    size_t steps = 0;
    for (int v : p->post)
        if (p->rel[v].a2.active) {
            tasks.push_back(v);
            steps = std::max(steps, p->rel[v].a2.levels.size());
        }
    struct Open {
        int shape;
        bool unit;
        HelmertBwdBatch b;
        double bytes, flops;
    };
    for (size_t r = 0; r < steps; ++r) {
        std::vector<Open> open;
        auto flush = [&](Open &o) -> figaro_status {
            if (o.b.count == 0) return FIGARO_OK;
            ProfScope ps(p, s, 6, o.bytes, o.flops);
            FIGARO_TRY(launch_helmert_bwd_batch(o.b, o.unit, s));
            o.b.count = 0;
            o.b.wg0[0] = 0;
            o.bytes = o.flops = 0.0;
            return FIGARO_OK;
        };
        for (int v : tasks) {
            Task &T = p->rel[v].a2;
            if (r >= T.levels.size()) continue;
            const int l = (int)(T.levels.size() - 1 - r);
            Level &L = T.levels[l];
            const HelmertBwdArgs a = level_bwd_args(p, T, l, values[v], ld[v], Target{dvalues[v], ld_dv[v]});
            const double bytes = 8.0 * (double)L.items * T.ncols * 2.0;
            const double flops = 2.0 * (double)L.items * T.ncols * T.ncols;
            const int shape = helmert_bwd_shape_class(T.ncols);
            if (shape == 0 || a.waves <= 0 || a.nchunks <= 0) {
                ProfScope ps(p, s, 6, bytes, flops);
                FIGARO_TRY(launch_helmert_bwd(a, L.unit, s));
                continue;
            }
            size_t k = 0;
            while (k < open.size() && !(open[k].shape == shape && open[k].unit == L.unit)) ++k;
            if (k == open.size()) open.push_back(Open{shape, L.unit, HelmertBwdBatch{}, 0.0, 0.0});
            Open &o = open[k];
            o.b.a[o.b.count] = a;
            o.b.wg0[o.b.count + 1] = o.b.wg0[o.b.count] + (a.waves + waves_per_block() - 1) / waves_per_block();
            ++o.b.count;
            o.bytes += bytes;
            o.flops += flops;
            if (o.b.count == kHelmertBwdBatch)
                if (figaro_status st = flush(o); st != FIGARO_OK) return st;
        }
        for (Open &o : open)
            if (figaro_status st = flush(o); st != FIGARO_OK) return st;
    }
    return FIGARO_OK;
}

figaro_status backward(figaro_plan_s *p, const double *const *values, const int64_t *ld, const double *R,
                       const double *dR, double *const *dvalues, const int64_t *ld_dv, hipStream_t s) {
    // recompute the forward intermediates (piece sums, joined heads)
    Buffers B;
    figaro_status st = forward(p, values, ld, false, nullptr, nullptr, 0, nullptr, s, false, &B);
    if (st != FIGARO_OK) return st;
    {
        ProfScope ps(p, s, 6, 0.0, 0.0);
        FIGARO_TRY(launch_qr_adjoint(R, dR, p->n, p->d_K, p->d_W, p->d_status, s));
    }
    for (auto it = p->post.rbegin(); it != p->post.rend(); ++it) {   // parents before children
        const int v = *it;
        RelPlan &Rl = p->rel[v];
        const bool leaf = Rl.children.empty();
        // items of v after the join (s), and where their gradient lives
        const double *items = leaf ? B.own[v] : Rl.d_s;
        const int64_t ld_items = leaf ? B.ld_own[v] : Rl.ld_s;
        const Target gs = leaf ? own_grad_target(p, v, dvalues, ld_dv) : Target{Rl.d_gs, Rl.nsub, true};
        if (Rl.parent < 0) {
            RootBwdArgs ra{};
            ra.groups = Rl.G;
            ra.n = p->n;
            ra.s = items;
            ra.ld_s = ld_items;
            ra.inv_sqrt_c = Rl.d_inv_sqrt_c;
            ra.K = p->d_K;
            ra.ds = gs.p;
            ra.ld_ds = gs.ld;
            ra.ds_rowmajor = gs.rowmajor ? 1 : 0;
            ProfScope ps(p, s, 6, 16.0 * (double)Rl.G * p->n, 0.0);
            FIGARO_TRY(launch_root_bwd(ra, s));
        } else if (!leaf && Rl.a4.active) {
            st = run_task_bwd(p, Rl.a4, items, ld_items, gs, s);
            if (st != FIGARO_OK) return st;
        }
        if (!leaf) {
            JoinBwdArgs j{};
            j.groups = Rl.G;
            j.ds = Rl.d_gs;
            j.ld_ds = Rl.nsub;
            const Target own = own_grad_target(p, v, dvalues, ld_dv);
            j.dOwn = own.p;
            j.ld_own = own.ld;
            j.own_cols = Rl.ncols;
            j.own_pos = Rl.own_pos;
            j.own_mult = Rl.d_own_mult;
            j.nchildren = (int32_t)Rl.children.size();
            for (size_t c = 0; c < Rl.children.size(); ++c) {
                const int ch = Rl.children[c];
                const Target t = sigma_grad_target(p, ch, dvalues, ld_dv);
                j.dsigma[c] = t.p;
                j.ld_dsigma[c] = t.ld;
                j.dsigma_rowmajor[c] = t.rowmajor ? 1 : 0;
                j.child_groups[c] = p->rel[ch].P;
                j.child_cols[c] = p->rel[ch].nsub;
                j.colpos[c] = Rl.d_colpos[c];
                j.inv_off[c] = Rl.d_inv_off[c];
                j.inv_idx[c] = Rl.d_inv_idx[c];
                j.nchunks[c] = Rl.join_nchunks[c];
                j.chunk_off[c] = Rl.d_chunk_off[c];
                j.chunk_q[c] = Rl.d_chunk_q[c];
                j.part[c] = Rl.d_join_part[c];
                j.mult[c] = Rl.d_mult[c];
            }
            ProfScope ps(p, s, 6, 16.0 * (double)Rl.G * Rl.nsub, 0.0);
            FIGARO_TRY(launch_join_bwd(j, s));
        }
    }
    // heads_and_tails of every relation last: each needs only the gradient
    // of its key-group sums, complete now; their levels from the top down,
    // the same step of tasks of one tile shape sharing launches
    return run_heads_and_tails_bwd(p, values, ld, dvalues, ld_dv, s);
}

}  // namespace

namespace figaro {

figaro_status run_forward(figaro_plan_s *p, const double *const *values, const int64_t *ld, double *R,
                          hipStream_t s) {
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    return forward(p, values, ld, true, R, nullptr, 0, nullptr, s);
}

figaro_status run_backward(figaro_plan_s *p, const double *const *values, const int64_t *ld, const double *R,
                           const double *dR, double *const *dvalues, const int64_t *ld_dv, hipStream_t s) {
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    if (p->wide) return set_error(p, FIGARO_EUNSUPPORTED, "the backward pass handles at most 128 columns");
    for (int i = 0; i < p->r; ++i)
        if (!dvalues[i] || ld_dv[i] < p->rel[i].m)
            return set_error(p, FIGARO_EINVAL, "dvalues[" + std::to_string(i) + "] is NULL or its ld too small");
    return backward(p, values, ld, R, dR, dvalues, ld_dv, s);
}

}  // namespace figaro

extern "C" {

figaro_status figaro_r_backward(figaro_plan_t p, const double *const *values, const int64_t *ld, const double *R,
                                const double *dR, double *const *dvalues, const int64_t *ld_dvalues,
                                hipStream_t stream) {
    if (!p) return set_error(nullptr, FIGARO_EINVAL, "plan is NULL");
    if (!R || !dR || !dvalues || !ld_dvalues) return set_error(p, FIGARO_EINVAL, "NULL argument");
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    if (p->wide) return set_error(p, FIGARO_EUNSUPPORTED, "the backward pass handles at most 128 columns");
    for (int i = 0; i < p->r; ++i)
        if (!dvalues[i] || ld_dvalues[i] < p->rel[i].m)
            return set_error(p, FIGARO_EINVAL, "dvalues[" + std::to_string(i) + "] is NULL or its ld too small");
    return backward(p, values, ld, R, dR, dvalues, ld_dvalues, stream);
}

figaro_status figaro_backward_status(figaro_plan_t p, hipStream_t stream) {
    if (!p || p->analyze_only) return set_error(p, FIGARO_EINVAL, "bad argument");
    int32_t st = 0;
    if (hipMemcpyAsync(&st, p->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return set_error(p, FIGARO_EHIP, "reading the backward status failed");
    return st ? set_error(p, FIGARO_ESINGULAR, "R has a zero diagonal entry") : FIGARO_OK;
}

figaro_status figaro_r(figaro_plan_t p, const double *const *values, const int64_t *ld, double *R,
                       hipStream_t stream) {
    if (!p) return set_error(nullptr, FIGARO_EINVAL, "plan is NULL");
    if (!R) return set_error(p, FIGARO_EINVAL, "R is NULL");
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    return forward(p, values, ld, true, R, nullptr, 0, nullptr, stream);
}

int64_t figaro_r0_rows(figaro_plan_t p) { return p ? p->r0_rows : -1; }

figaro_status figaro_r0(figaro_plan_t p, const double *const *values, const int64_t *ld, double *R0,
                        int64_t ld_r0, int32_t *block_of_row, hipStream_t stream) {
    if (!p) return set_error(nullptr, FIGARO_EINVAL, "plan is NULL");
    if (!R0 || ld_r0 < p->r0_rows) return set_error(p, FIGARO_EINVAL, "R0 is NULL or ld_r0 too small");
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    hipError_t e = launch_fill(R0, (int64_t)p->n * ld_r0, 0.0, stream);
    if (e != hipSuccess) return set_error(p, FIGARO_EHIP, hipGetErrorString(e));
    if (block_of_row) {
        e = launch_fill_i32(block_of_row, p->r0_rows, -1, stream);
        if (e != hipSuccess) return set_error(p, FIGARO_EHIP, hipGetErrorString(e));
    }
    return forward(p, values, ld, false, nullptr, R0, ld_r0, block_of_row, stream);
}

figaro_status figaro_permute_values(figaro_plan_t p, int32_t rel, const double *src, int64_t ld_src, double *dst,
                                    int64_t ld_dst, hipStream_t stream) {
    if (!p || rel < 0 || rel >= p->r || !src || !dst || p->analyze_only)
        return set_error(p, FIGARO_EINVAL, "bad argument");
    const RelPlan &R = p->rel[rel];
    if (ld_src < R.m_in || ld_dst < R.m) return set_error(p, FIGARO_EINVAL, "leading dimension too small");
    hipError_t e = launch_permute(src, ld_src, dst, ld_dst, R.d_perm, R.m, R.ncols, false, R.m_in, stream);
    return e == hipSuccess ? FIGARO_OK : set_error(p, FIGARO_EHIP, hipGetErrorString(e));
}

figaro_status figaro_unpermute_values(figaro_plan_t p, int32_t rel, const double *src, int64_t ld_src, double *dst,
                                      int64_t ld_dst, hipStream_t stream) {
    if (!p || rel < 0 || rel >= p->r || !src || !dst || p->analyze_only)
        return set_error(p, FIGARO_EINVAL, "bad argument");
    const RelPlan &R = p->rel[rel];
    if (ld_src < R.m || ld_dst < R.m_in) return set_error(p, FIGARO_EINVAL, "leading dimension too small");
    hipError_t e = launch_permute(src, ld_src, dst, ld_dst, R.d_perm, R.m, R.ncols, true, R.m_in, stream);
    return e == hipSuccess ? FIGARO_OK : set_error(p, FIGARO_EHIP, hipGetErrorString(e));
}

int64_t figaro_debug_stack_rows(figaro_plan_t p) { return p ? p->stack_rows : -1; }

int64_t figaro_debug_tile_rows(int32_t n, int32_t variant) {
    if (n < 1 || n > kMaxCols || variant < 0 || variant >= num_variants()) return -1;
    return dense_tile_rows_for(n, variant);
}

int64_t figaro_debug_dense_rows(int32_t n, int32_t variant, int64_t tiles_per_wave) {
    if (n < 1 || n > kMaxCols || variant < 0 || variant >= num_variants() || tiles_per_wave < 1) return -1;
    return (int64_t)dense_waves_per_block(n) * tiles_per_wave * dense_tile_rows_for(n, variant);
}

figaro_status figaro_debug_dense_step(int32_t n, int64_t rows, const double *in, int64_t ld_in, int32_t workgroups,
                                      int64_t tiles_per_wave, int32_t variant, double *out, int64_t ld_out,
                                      double *final_r, hipStream_t stream) {
    if (n < 1 || n > kMaxCols || rows < 0 || !in || ld_in < rows || workgroups < 1 || tiles_per_wave < 1 ||
        variant < 0 || variant >= num_variants())
        return set_error(nullptr, FIGARO_EINVAL, "bad argument");
    const int64_t per_wg = (int64_t)dense_waves_per_block(n) * tiles_per_wave * dense_tile_rows_for(n, variant);
    if ((int64_t)workgroups * per_wg < rows) return set_error(nullptr, FIGARO_EINVAL, "workgroups do not cover the rows");
    const bool fin = workgroups == 1 && final_r;
    if (!fin && (!out || ld_out < (int64_t)workgroups * n)) return set_error(nullptr, FIGARO_EINVAL, "bad output");
    DenseArgs a{};
    a.in = in;
    a.ld_in = ld_in;
    a.rows = rows;
    a.n = n;
    a.out = out;
    a.ld_out = ld_out;
    a.waves = workgroups;
    a.tiles_per_wave = tiles_per_wave;
    a.final_r = fin ? final_r : nullptr;
    hipError_t e = launch_dense(a, variant, stream);
    return e == hipSuccess ? FIGARO_OK : set_error(nullptr, FIGARO_EHIP, hipGetErrorString(e));
}

int32_t figaro_debug_stack_layout(figaro_plan_t p, int64_t *out, int32_t max_regions) {
    if (!p || !out || p->wide) return -1;
    int32_t k = 0;
    for (int v : p->post) {
        RelPlan &R = p->rel[v];
        for (Task *T : {&R.a2, &R.a4}) {
            if (!T->active) continue;
            for (size_t l = 0; l < T->levels.size(); ++l) {
                const Level &L = T->levels[l];
                const int64_t rows = (l == 0 && T->ncols <= kFusedMaxCols)
                                         ? (int64_t)((L.waves + waves_per_block() - 1) / waves_per_block()) * T->ncols
                                              : L.items;
                if (k < max_regions) {
                    out[3 * k] = T->block_id;
                    out[3 * k + 1] = L.stack_row0;
                    out[3 * k + 2] = rows;
                }
                ++k;
            }
        }
        if (R.parent < 0) {
            if (k < max_regions) {
                out[3 * k] = 3 * v + 2;
                out[3 * k + 1] = R.root_row0;
                out[3 * k + 2] = R.G;
            }
            ++k;
        }
    }
    return k;
}

figaro_status figaro_debug_stack(figaro_plan_t p, const double *const *values, const int64_t *ld, double *host_out,
                                 hipStream_t stream) {
    if (!p || !host_out) return set_error(p, FIGARO_EINVAL, "bad argument");
    if (p->wide) return set_error(p, FIGARO_EUNSUPPORTED, "wide plans reduce their stack in place");
    figaro_status st = check_inputs(p, values, ld);
    if (st != FIGARO_OK) return st;
    st = forward(p, values, ld, true, nullptr, nullptr, 0, nullptr, stream, true);
    if (st != FIGARO_OK) return st;
    if (hipStreamSynchronize(stream) != hipSuccess) return set_error(p, FIGARO_EHIP, "sync failed");
    for (int c = 0; c < p->n; ++c)
        if (hipMemcpy(host_out + (size_t)c * p->stack_rows, p->d_stack[0] + (size_t)c * p->stack_ld[0],
                      sizeof(double) * (size_t)p->stack_rows, hipMemcpyDeviceToHost) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "copy failed");
    return FIGARO_OK;
}

figaro_status figaro_profile_enable(figaro_plan_t p, int32_t capacity) {
    if (!p || capacity < 0) return set_error(p, FIGARO_EINVAL, "bad argument");
    for (auto e : p->prof_start) (void)hipEventDestroy(e);
    for (auto e : p->prof_stop) (void)hipEventDestroy(e);
    p->prof_start.clear();
    p->prof_stop.clear();
    p->prof_pending.clear();
    p->prof_next = 0;
    for (int32_t q = 0; q < capacity; ++q) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return set_error(p, FIGARO_EHIP, "hipEventCreate failed");
        if (hipEventCreate(&b) != hipSuccess) return set_error(p, FIGARO_EHIP, "hipEventCreate failed");
        p->prof_start.push_back(a);
        p->prof_stop.push_back(b);
    }
    return FIGARO_OK;
}

static figaro_status prof_drain(figaro_plan_s *p) {
    for (const auto &q : p->prof_pending) {
        if (hipEventSynchronize(p->prof_stop[q.slot]) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->prof_start[q.slot], p->prof_stop[q.slot]) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "hipEventElapsedTime failed");
        p->prof_ms[q.kind] += ms;
        p->prof_launches[q.kind] += 1;
        p->prof_bytes[q.kind] += q.bytes;
        p->prof_flops[q.kind] += q.flops;
    }
    p->prof_pending.clear();
    p->prof_next = 0;
    return FIGARO_OK;
}

figaro_status figaro_profile_read(figaro_plan_t p, int32_t kind, double *ms, int64_t *launches, double *bytes,
                                  double *flops) {
    if (!p || kind < 0 || kind >= kProfClasses) return set_error(p, FIGARO_EINVAL, "bad argument");
    figaro_status st = prof_drain(p);
    if (st != FIGARO_OK) return st;
    if (ms) *ms = p->prof_ms[kind];
    if (launches) *launches = p->prof_launches[kind];
    if (bytes) *bytes = p->prof_bytes[kind];
    if (flops) *flops = p->prof_flops[kind];
    return FIGARO_OK;
}

figaro_status figaro_profile_reset(figaro_plan_t p) {
    if (!p) return set_error(p, FIGARO_EINVAL, "bad argument");
    figaro_status st = prof_drain(p);
    for (int k = 0; k < kProfClasses; ++k) {
        p->prof_ms[k] = 0;
        p->prof_launches[k] = 0;
        p->prof_bytes[k] = 0;
        p->prof_flops[k] = 0;
    }
    return st;
}

}  // extern "C"
