// Internal structures shared by the plan builder, the launch sequence and the
// kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/figaro.h"

namespace figaro {

// Widest column count the register-tile kernels handle (the narrow regime:
// dense TSQR of the stack in registers, backward pass).
constexpr int kMaxCols = 128;
// Widest column count of a plan; above kMaxCols the stack is reduced by the
// blocked Householder QR of wideqr.hip.
constexpr int kMaxWideCols = 16384;
// Head/tail tasks with more columns than this write their tails to the stack
// of the post-processing TSQR, in column chunks of kChunkCols, instead of
// folding them into a register-tile QR.
constexpr int kFusedMaxCols = 40;
constexpr int kChunkCols = 32;

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value).
// ---------------------------------------------------------------------------

// One launch of the segmented head/tail + QR-accumulate kernel.
//
// Items are rows of `in` (column-major [ncols][ld_in]).  Each item has a
// count c (1 for input rows) and a vector of column sums s.  Items are
// grouped into pieces (consecutive items of one key group inside one chunk).
// For the t-th item of a piece with W items' worth of count before it and
// P the sum of the s of those items, the tail row is
//     (W s - c P) / (sqrt(c) sqrt(W) sqrt(W + c)) * phi      (phi: group scale)
// which is the generalized tail of Definition 2 written with sums instead of
// heads.  The first item of a piece has no tail.  The kernel writes the sum
// of every piece to `pieces_out` and either folds the tail rows into a
// per-wave Householder R (mode FUSE) or writes them to an R0 buffer.
// The joined heads of a relation read in place: process_and_join_children
// (Algorithm 3) fused into the first level of project_away_join_attributes.
// Column c of item (key group) g is
//   own[idx[c] * ld_own + g] * own_mult[g]                       if src[c] < 0,
//   sigma_j[cidx_j[g] * ld_sigma_j + idx[c]] * mult_j[g]         if src[c] = j,
// the same products the separate join kernel would store.  The children's
// sums are row-major here, so the columns of one child group share a cache
// line.
constexpr int kFuseMaxChildren = 4;
struct JoinSrc {
    const double *own;
    int64_t ld_own;
    const double *own_mult;
    int32_t nchildren;
    const double *sigma[kFuseMaxChildren];
    int64_t ld_sigma[kFuseMaxChildren];
    const int32_t *cidx[kFuseMaxChildren];
    const double *mult[kFuseMaxChildren];
    // per joined column: (source + 1) << 8 | column within the source, with
    // source -1 for the own sums and j for child j (32-bit words, so the
    // kernel reads them with scalar loads)
    int32_t code[kMaxCols];
};

struct HelmertArgs {
    const double *in;
    int64_t ld_in;
    int32_t ncols;
    int64_t items;
    const int32_t *pid;          // [items] piece id of each item
    const int64_t *piece_start;  // [npieces+1] first item of every piece
    const double *phi_piece;     // unit-count mode: tail scale of every piece
    const double *alpha;         // weighted mode: per-item tail coefficient of s
    const double *beta;          // weighted mode: per-item tail coefficient of P
    const int64_t *chunk_start;  // [nchunks+1]
    const int32_t *chunk_piece0; // [nchunks+1] first piece id of every chunk
    int64_t nchunks;
    double *pieces_out;          // [ncols][ld_pieces] (may be null: no piece output)
    int64_t ld_pieces;
    // QR output: each wave writes its R (ncols rows, n_total columns) at rows
    // stack_row0 + wave*ncols of `stack`.
    double *stack;
    int64_t ld_stack;
    int64_t stack_row0;
    int32_t n_total;
    uint64_t other_cols[2];      // bit g set: global column g is not a column of this block
    uint16_t colmap[kFusedMaxCols];   // output column of every local column
    // R0 output (materialisation for inspection)
    double *r0;
    int64_t ld_r0;
    int64_t r0_row0;
    int32_t *block_of_row;
    int32_t block_id;
    int32_t waves;
    // items read through a join view (first project-away level), columns
    // join_col0 .. join_col0 + ncols - 1 of the joined heads
    int32_t join;
    int32_t join_col0;
    JoinSrc js;
    // a task of more than kFusedMaxCols columns (tails not folded): one
    // launch takes all of its kChunkCols-column chunks, blockIdx.y the chunk
    // (0: not chunked).  Output column of task column c: c itself
    // (cols_ident, a region) or wide_colmap[c].
    int32_t wide_cols;
    int32_t cols_ident;
    const uint16_t *wide_colmap;
};

// Upper head/tail levels of independent tasks in one launch (kernel
// arguments stay under 4 KB): task t owns workgroups [wg0[t], wg0[t + 1]).
constexpr int kHelmertBatch = 3;
struct HelmertBatch {
    HelmertArgs a[kHelmertBatch];
    int32_t wg0[kHelmertBatch + 1];
    int32_t count;
};

// Dense TSQR step: QR of `rows` rows of `in` ([n][ld_in]); workgroup b (of
// `waves` workgroups; n <= 16: 4 waves on separate tiles, tiles_per_wave
// tiles per wave; n > 16: waves sharing each tile, tiles_per_wave tiles per
// workgroup) writes its
// R (n rows) to `out` rows b*n, or the final R (sign-normalised) to `final_r`
// when there is a single workgroup.
struct DenseArgs {
    const double *in;
    int64_t ld_in;
    int64_t rows;
    int32_t n;
    double *out;
    int64_t ld_out;
    int32_t waves;
    int64_t tiles_per_wave;
    double *final_r;
};

// Backward of one head/tail level: recompute the tails of every chunk, take
// dT = T K_blk (K_blk: K restricted to the block's columns), and write the
// gradient of every item:  ds_t = alpha_t dT_t - sum_{u > t in its piece}
// beta_u dT_u + dsigma[piece of t].
struct HelmertBwdArgs {
    const double *in;
    int64_t ld_in;
    int32_t ncols;
    const int32_t *pid;
    const int64_t *piece_start;
    const double *phi_piece;
    const double *alpha;
    const double *beta;
    const int64_t *chunk_start;
    int64_t nchunks;
    const double *K;             // n_total x n_total, column-major
    int32_t n_total;
    uint8_t colmap[kMaxCols];
    const double *gpieces;       // gradient of the piece sums, [ncols][ld_gp]
    int64_t ld_gp;
    double *gout;                // gradient of the items, [ncols][ld_gout] (or [items][ld_gout])
    int64_t ld_gout;
    int32_t gout_rowmajor;       // 1: item t, column c at gout[t * ld_gout + c]
    int32_t waves;
};

constexpr int kMaxChildren = 16;

// process_and_join_children: per key group g of relation i,
//   s[own columns][g]   = own_sum[g] * own_mult[g]
//   s[child j cols][g]  = sigma_j[cidx_j[g]] * mult_j[g]
struct JoinArgs {
    int64_t groups;
    int32_t nsub;
    double *s;
    int64_t ld_s;
    const double *own;
    int64_t ld_own;
    int32_t own_cols;
    int32_t own_pos;
    const double *own_mult;
    int32_t nchildren;
    const double *sigma[kMaxChildren];
    int64_t ld_sigma[kMaxChildren];
    int32_t child_cols[kMaxChildren];
    const int32_t *colpos[kMaxChildren];
    const int32_t *cidx[kMaxChildren];
    const double *mult[kMaxChildren];
    const int16_t *col_src;      // [nsub] per output column: -1 own, else the child
    const int16_t *col_idx;      // [nsub] per output column: column within its source
};

// Root emit: rows s[.][g] / sqrt(c_g) into the stack (or R0).
struct RootArgs {
    int64_t groups;
    int32_t n;
    const double *s;
    int64_t ld_s;
    const double *inv_sqrt_c;    // [groups] (may be null: factor 1)
    double *dst;
    int64_t ld_dst;
    int64_t row0;
    int32_t *block_of_row;
    int32_t block_id;
};

// Backward of process_and_join_children: own-column gradient scaled by
// own_mult, and for every child group q the sum over the parent key groups
// that join it (plan-time inverse index, deterministic order).
struct JoinBwdArgs {
    int64_t groups;
    const double *ds;            // row-major [groups][ld_ds] (ld_ds >= nsub)
    int64_t ld_ds;
    double *dOwn;                // [own_cols][ld_own]
    int64_t ld_own;
    int32_t own_cols;
    int32_t own_pos;
    const double *own_mult;
    int32_t nchildren;
    double *dsigma[kMaxChildren];
    int64_t ld_dsigma[kMaxChildren];
    int32_t dsigma_rowmajor[kMaxChildren];
    int64_t child_groups[kMaxChildren];
    int32_t child_cols[kMaxChildren];
    const int32_t *colpos[kMaxChildren];
    const int64_t *inv_off[kMaxChildren];   // [child groups + 1]
    const int32_t *inv_idx[kMaxChildren];   // parent key groups sorted by child group
    const double *mult[kMaxChildren];
    // children whose inverse lists run long: the lists cut into chunks of
    // kJoinChunk entries (chunk k belongs to child group chunk_q[k]; the
    // chunks of group q are chunk_off[q] .. chunk_off[q + 1] - 1), a
    // partial sum per (chunk, column) in part, summed in chunk order
    int64_t nchunks[kMaxChildren];           // 0: one thread per child group walks its list
    const int64_t *chunk_off[kMaxChildren];
    const int32_t *chunk_q[kMaxChildren];
    double *part[kMaxChildren];              // [nchunks][child columns]
    int64_t part_block0[kMaxChildren + 2];   // first block of every part (set by the launcher)
};

// Backward of the root heads: row_g = s_g / sqrt(c_g), d row_g = row_g K,
// ds_g = d row_g / sqrt(c_g).
struct RootBwdArgs {
    int64_t groups;
    int32_t n;
    const double *s;
    int64_t ld_s;
    const double *inv_sqrt_c;
    const double *K;
    double *ds;
    int64_t ld_ds;
    int32_t ds_rowmajor;         // 1: group g, column c at ds[g * ld_ds + c]
};

struct WideQr;

// ---------------------------------------------------------------------------
// Launchers (kernels.hip)
// ---------------------------------------------------------------------------
hipError_t launch_helmert(const HelmertArgs &a, bool unit, bool fuse, int variant, hipStream_t s);
// One level of up to kHelmertBatch tasks of one tile shape (columns <=
// kFusedMaxCols, same nb_for(ncols), variant, unit counts and folding).
hipError_t launch_helmert_batch(const HelmertBatch &b, bool unit, bool fuse, int variant, hipStream_t s);
int helmert_shape_class(int ncols);
hipError_t launch_dense(const DenseArgs &a, int variant, hipStream_t s);
hipError_t launch_join(const JoinArgs &a, hipStream_t s);
hipError_t launch_rowmajor(const double *src, int64_t ld_src, int64_t rows, int32_t ncols, double *dst, hipStream_t s);
hipError_t launch_root(const RootArgs &a, bool to_r0, hipStream_t s);
hipError_t launch_permute(const double *src, int64_t ld_src, double *dst, int64_t ld_dst,
                          const int64_t *perm, int64_t rows, int32_t ncols, bool inverse,
                          int64_t total_rows, hipStream_t s);
hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t s);
hipError_t launch_qr_adjoint(const double *R, const double *dR, int32_t n, double *K, double *W, int32_t *status,
                             hipStream_t s);
hipError_t launch_helmert_bwd(const HelmertBwdArgs &a, bool unit, hipStream_t s);
hipError_t launch_join_bwd(const JoinBwdArgs &a, hipStream_t s);
hipError_t launch_root_bwd(const RootBwdArgs &a, hipStream_t s);
hipError_t launch_copy_cols(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t rows,
                            int32_t ncols, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
// Blocked Householder QR (wideqr.hip).
int64_t wide_qr_panel_rows(int64_t h, int32_t n, bool tp);
int64_t wide_qr_workspace_doubles(int64_t max_nv, int32_t n);
// Workspace carving; blas: a rocBLAS handle to share, or null to create one.
figaro_status wide_qr_init(WideQr &w, double *ws, int64_t max_nv, int32_t n, void *blas, std::string &err);
void wide_qr_release(WideQr &w);
// One QR of the blocked kind: A (h x n, lda) in place, general (tp false)
// or with rows [0, n) an upper triangular block (tp true).
struct WideQrJob {
    const WideQr *w;
    double *A;
    int64_t lda, h;
    int32_t n;
    bool tp;
};
// Independent QRs side by side: their panels share launches.
figaro_status wide_qr_many(const std::vector<WideQrJob> &jobs, hipStream_t s, std::string &err);
hipError_t launch_copy_upper(const double *src, int64_t ld_src, int64_t rows, int32_t cols, double *dst,
                             int64_t ld_dst, int64_t row0, int64_t col0, hipStream_t s);
hipError_t launch_final_r(const double *A, int64_t lda, int64_t rows, int32_t n, double *R, hipStream_t s);
// Whole passes on one plan (run.cpp), used by the batched entry points.
figaro_status run_forward(figaro_plan_s *p, const double *const *values, const int64_t *ld, double *R,
                          hipStream_t s);
figaro_status run_backward(figaro_plan_s *p, const double *const *values, const int64_t *ld, const double *R,
                           const double *dR, double *const *dvalues, const int64_t *ld_dv, hipStream_t s);

int tile_items_for(int ncols, int variant);   // items per chunk of the register-tile kernel
int num_variants();                           // number of register-tile kernel variants
int dense_tile_rows_for(int ncols, int variant);   // rows per tile of the dense kernel
int dense_waves_per_block(int ncols);   // waves of a workgroup that fold separate tiles
bool dense_coop(int ncols);            // dense steps share each tile among a workgroup's waves
int waves_per_block();                // waves per workgroup of the QR kernels

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------

// One level of a segmented head/tail task.
struct Level {
    int64_t items = 0, npieces = 0, nchunks = 0;
    bool unit = false;
    int32_t variant = 0;          // tile shape of the head/tail kernel at this level
    int32_t waves = 0;
    int64_t stack_row0 = 0;       // first stack row of this launch's R's
    int64_t r0_row0 = 0;          // first R0 row of this level
    int32_t *d_pid = nullptr;
    int64_t *d_piece_start = nullptr;
    int64_t *d_chunk_start = nullptr;
    int32_t *d_chunk_piece0 = nullptr;   // [nchunks+1] first piece of every chunk
    double *d_phi_piece = nullptr;       // [npieces+1] (one entry of padding)
    double *d_alpha = nullptr, *d_beta = nullptr;
    double *d_pieces = nullptr;   // [ncols][npieces]
    double *d_gpieces = nullptr;  // gradient of the piece sums, [ncols][npieces]
};

// heads_and_tails (A2) or project_away_join_attributes (A4) of one relation.
struct Task {
    bool active = false;
    // wide plans: the tails of a wide heads_and_tails task go to a region
    // of their own (task columns, ld region_ld) that is reduced by itself
    double *d_region = nullptr;
    int64_t region_ld = 0;
    int32_t variant = 0;          // tile shape of the head/tail kernel
    int32_t ncols = 0;
    int32_t block_id = 0;
    std::vector<int32_t> cols;    // global columns, ascending
    uint16_t *d_cols16 = nullptr; // cols on the device (tasks of more than kFusedMaxCols columns)
    int32_t *d_colmap = nullptr;
    int32_t *d_inv_colmap = nullptr;
    std::vector<Level> levels;
};

struct RelPlan {
    // as given
    int64_t m_in = 0;
    int32_t nkeys = 0;
    std::vector<int32_t> attrs;   // as given
    int32_t ncols = 0;
    int32_t parent = -1;
    std::vector<int32_t> children;
    int32_t col0 = 0;             // first global column
    // reduction, order, groups
    int64_t m = 0;                // rows kept
    std::vector<int64_t> perm;    // plan row -> caller row (kept rows first)
    int64_t *d_perm = nullptr;
    int64_t G = 0, P = 0;         // key groups, parent groups
    std::vector<int64_t> seg_off; // [G+1] row offsets of key groups
    std::vector<int64_t> par_off; // [P+1] key-group offsets of parent groups
    // counts (exact)
    std::vector<int64_t> rpk, theta, phi_circ, fjs;  // [G]
    std::vector<int64_t> phi_up, phi_down;           // [P]
    // heads/tails of S_i
    bool singleton = false;       // every key group has one row
    Task a2;
    // join with children
    int32_t nsub = 0;
    std::vector<int32_t> sub_cols;   // global columns of the subtree, ascending
    int32_t own_pos = 0;
    double *d_own_mult = nullptr;
    std::vector<int32_t *> d_cidx;
    std::vector<double *> d_mult;
    std::vector<int32_t *> d_colpos;
    std::vector<double *> d_sigma_rm;   // fused join: row-major copy of every child's sums [P_child][nsub_child]
    std::vector<int16_t> col_src;    // [nsub] per subtree column: -1 own, else child index
    std::vector<int16_t> col_idx;    // [nsub] per subtree column: column within its source
    int16_t *d_col_src = nullptr, *d_col_idx = nullptr;
    bool fuse_join = false;          // joined heads read in place by the first project-away level
    double *d_s = nullptr;           // [nsub][ld_s]
    int64_t ld_s = 0;                // G rounded up to 16 (aligned columns)
    double *d_gs = nullptr;          // gradient of s, [nsub][G]
    std::vector<int64_t *> d_inv_off;   // per child: [P_child+1]
    std::vector<int32_t *> d_inv_idx;   // per child: [G]
    // per child: the inverse lists in chunks, where some list is longer
    // than kJoinChunk (else nchunks 0 and null pointers)
    std::vector<int64_t> join_nchunks;
    std::vector<int64_t *> d_chunk_off;
    std::vector<int32_t *> d_chunk_q;
    std::vector<double *> d_join_part;
    // projection onto X_p
    Task a4;
    // root
    double *d_inv_sqrt_c = nullptr;
    int64_t root_row0 = 0;
    int64_t r0_root_row0 = 0;
    // plans built on the device: segment offsets and counts stay there, and
    // the host copies above are fetched when a query asks for them
    int64_t *d_seg_off = nullptr, *d_par_off = nullptr;   // [G+1], [P+1]
    int64_t *d_theta = nullptr, *d_phi_circ = nullptr;     // [G]
    int64_t *d_theta_excl = nullptr;  // [G+1] exclusive prefix sums of Theta (join-row enumeration)
    int64_t *d_phi_up = nullptr, *d_phi_down = nullptr;   // [P]
    bool host_arrays = true;         // perm, seg_off, par_off and the counts are on the host
};

constexpr int kProfClasses = 8;

struct ProfPending {
    int kind;
    int slot;
    double bytes, flops;
};

// Workspace of the blocked Householder QR (wideqr.hip).
struct WideQr {
    double *V = nullptr;      // [32][ldv] reflectors of one panel (virtual rows)
    int64_t ldv = 0;
    double *tau = nullptr;    // [n]
    double *T = nullptr;      // V^T V of the current panel, [32][32]
    double *G = nullptr;      // partial products V^T V, [parts][32][32]
    double *W = nullptr;      // T^T V^T C, [n][32]
    double *Wp = nullptr;     // partial products V^T C, [parts][n][32]
    int64_t wp_stride = 0;
    double *part = nullptr;   // partial sums of the per-column passes
    double *head = nullptr;
    void *blas = nullptr;     // rocblas_handle
};

struct DenseLevel {
    int64_t rows;
    int32_t waves;
    int64_t tiles_per_wave;
};

}  // namespace figaro

struct figaro_plan_s {
    int32_t r = 0;
    int32_t n = 0;
    int32_t root = -1;
    std::vector<int32_t> post;           // post-order of relations
    std::vector<figaro::RelPlan> rel;
    double join_rows = 0.0;
    int device = 0;
    int32_t tile_items = 0;
    int32_t waves_cap = 0;
    bool analyze_only = false;
    bool separate_join = false;
    bool device_plan = false;        // keys segmented and counted on the device
    int32_t variant = 0;
    // stack for the post-processing TSQR
    int64_t stack_rows = 0;
    double *d_stack[2] = {nullptr, nullptr};
    int64_t stack_ld[2] = {0, 0};
    std::vector<figaro::DenseLevel> dense;
    // wide regime (n > kMaxCols): rows [0, n) of stack 0 hold the R's of the
    // wide heads_and_tails tasks on the diagonal, the other stack rows
    // follow; the whole stack is reduced by the blocked QR
    bool wide = false;
    figaro::WideQr wqr;                       // the final QR of the stack (owns the rocBLAS handle)
    std::vector<figaro::WideQr> region_qr;    // one per region, in post order of their relations
    int64_t r0_rows = 0;
    double *d_K = nullptr;           // n x n, backward
    double *d_W = nullptr;           // n x n scratch of the QR adjoint
    int32_t *d_status = nullptr;     // device status word of the backward pass
    int64_t workspace_bytes = 0;
    std::vector<void *> allocations;
    // autotuner result (figaro_plan_create_tuned), tuned_ms < 0 otherwise
    double tuned_ms = -1.0;
    figaro_plan_options tuned_options{};
    std::string last_error;
    // profiling
    std::vector<hipEvent_t> prof_start, prof_stop;
    size_t prof_next = 0;
    std::vector<figaro::ProfPending> prof_pending;
    double prof_ms[figaro::kProfClasses] = {0};
    int64_t prof_launches[figaro::kProfClasses] = {0};
    double prof_bytes[figaro::kProfClasses] = {0};
    double prof_flops[figaro::kProfClasses] = {0};
};

namespace figaro {

// Device allocations owned by a plan (freed by figaro_plan_destroy).
template <typename T>
inline hipError_t dev_upload(figaro_plan_s *p, T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    size_t bytes = sizeof(T) * std::max<size_t>(src.size(), 1);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    p->allocations.push_back(*dst);
    p->workspace_bytes += (int64_t)bytes;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return e;
}

inline hipError_t dev_alloc(figaro_plan_s *p, void **dst, size_t bytes) {
    *dst = nullptr;
    hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return e;
    p->allocations.push_back(*dst);
    p->workspace_bytes += (int64_t)std::max<size_t>(bytes, 8);
    return e;
}


figaro_status set_error(figaro_plan_s *p, figaro_status st, const std::string &msg);

// Inverse lists longer than this are summed in chunks by the join adjoint.
constexpr int64_t kJoinChunk = 1024;
// Chunks of relation R's inverse list for child c from its offsets (host
// copy, P_child + 1 entries), appended to R's per-child vectors (plan.cpp).
figaro_status join_chunks(figaro_plan_s *p, RelPlan &R, size_t c, const std::vector<int64_t> &off);

// Levels of a segmented head/tail task from level `first` on (plan.cpp):
// items grouped by group_off (ngroups + 1 offsets), per-item counts (empty:
// every item counts 1), per-group tail scale, the chunk size of level 0.
figaro_status build_task_levels(figaro_plan_s *p, Task &T, int first, int64_t items, std::vector<int64_t> goff,
                                std::vector<int64_t> cnt, bool unit, const std::vector<double> &phi, int tile);
figaro_status finish_task(figaro_plan_s *p, Task &T, int32_t n_total);
// Stack and R0 layout, dense TSQR levels and the remaining workspace, once
// every task is built (plan.cpp).
figaro_status finish_plan(figaro_plan_s *p);
// Key segmentation, count queries and the tasks' first levels on the device
// (dplan.hip), from the validated tree and columns of p.
figaro_status build_keys_on_device(figaro_plan_s *p, const figaro_relation_desc *rels, hipStream_t stream);
// Host copies of the device plan's arrays for the query calls.
figaro_status fetch_host_arrays(figaro_plan_s *p, int32_t rel);
// Device arrays the enumeration of join rows reads (segment and parent-group
// offsets, Theta and its prefix sums, Phi-down), for plans of either builder
// (dplan.hip).
figaro_status enumeration_arrays(figaro_plan_s *p, hipStream_t stream);

}  // namespace figaro
