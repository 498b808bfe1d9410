/*
 * figaro.h -- C ABI of the MI355X library that computes the upper-triangular
 * factor R of the QR decomposition of the data columns of an acyclic natural
 * join, without materialising the join.
 *
 * The problem statement follows the paper's setup section ("Input" and
 * "Output"): the input is a database of relations S_1..S_r together with a
 * join tree; the output is the R of A[:Y], the data columns of the join.  R is
 * returned upper triangular with a non-negative diagonal, which makes it unique
 * whenever A has full column rank.
 *
 * Model.
 *  - A relation has `rows` tuples, `num_keys` join attributes (identified by
 *    global attribute ids; equal ids are compared for equality, which is the
 *    natural join) and `num_cols` real data columns.
 *  - Key attributes are join attributes only: every key attribute of a
 *    relation must be shared with its parent or with one of its children in
 *    the join tree.  A relation with no key attributes joins its parent by
 *    Cartesian product.
 *  - The join tree is given by `parent` (-1 for exactly one root).  For every
 *    attribute, the relations containing it must form a connected subtree
 *    (running intersection).
 *  - Tuples are a bag: duplicate tuples each count.  Dangling tuples (tuples
 *    that occur in no join row) are removed by the plan (semi-join reduction);
 *    the paper assumes a fully reduced database, and R is unchanged by the
 *    removal.
 *  - Columns of R are ordered by relation index, then by column order within
 *    a relation; key attributes are not columns of R.
 *
 * Layouts.  Key columns are device arrays, column-major [num_keys][rows] of
 * int32 or int64.  Data values are FP64, column-major: column c of relation i
 * starts at values[i] + c * ld[i], ld[i] >= rows.  R is FP64 column-major
 * n x n (leading dimension n), n = sum of num_cols.
 *
 * Row order.  The compute calls take the values of every relation in *plan
 * order*: rows sorted by the relation's key attributes (the paper's
 * algorithms assume sorted inputs), with only the rows that survive the
 * reduction.  figaro_plan_permutation() gives the permutation and
 * figaro_permute_values() applies it on the device.
 *
 * Ownership and concurrency.  The caller owns every buffer it passes.  The
 * plan owns a device workspace, allocated in figaro_plan_create(); the compute
 * calls allocate nothing and do not synchronise the host, and enqueue all work
 * on the given stream.  Calls that use the same plan share its workspace and
 * must be serialised on one stream.
 *
 * Errors.  Every call returns a figaro_status; nothing is thrown across the
 * ABI.  figaro_last_error() returns a message for the last failing call on a
 * plan (or, for a NULL plan, the last failing call of the calling thread).
 * NaN or Inf values propagate into R and are not an error.
 */
#ifndef FIGARO_H
#define FIGARO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct figaro_plan_s *figaro_plan_t;

typedef enum {
    FIGARO_OK = 0,
    FIGARO_EINVAL = 1,          /* bad argument (NULL pointer, size, dtype, ld) */
    FIGARO_ENOTTREE = 2,        /* parents do not form one tree, or running intersection fails */
    FIGARO_EUNSHARED_KEY = 3,   /* a key attribute shared with no neighbour in the tree */
    FIGARO_EEMPTY_JOIN = 4,     /* the join has no rows */
    FIGARO_EOVERFLOW = 5,       /* a count query value reaches 2^53 */
    FIGARO_ESINGULAR = 6,       /* R has a zero diagonal entry (backward pass) */
    FIGARO_ENOMEM = 7,          /* device allocation failed */
    FIGARO_EHIP = 8,            /* a HIP runtime call failed */
    FIGARO_EUNSUPPORTED = 9     /* a size beyond what this build supports */
} figaro_status;

/* One relation of the database. */
typedef struct {
    int64_t rows;               /* number of tuples m_i >= 0 */
    int32_t num_keys;           /* number of join attributes k_i >= 0 */
    const int32_t *key_attr;    /* host [k_i]: global attribute ids, distinct */
    const void *key_cols;       /* device [k_i][rows] int32 or int64 */
    int32_t key_dtype;          /* 4 (int32) or 8 (int64) */
    int32_t num_cols;           /* number of FP64 data columns n_i >= 1 */
    int32_t parent;             /* index of the parent relation, -1 for the root */
} figaro_relation_desc;

/* Tuning knobs of a plan; pass NULL for defaults. */
typedef struct {
    int32_t tile_items;         /* items per tile of the segmented head/tail
                                   kernels; 0 = default (chosen per column
                                   count).  Smaller tiles split key groups
                                   across tiles, which exercises the
                                   two-level head/tail combination. */
    int32_t waves_per_task;     /* upper bound on waves of one head/tail
                                   launch, 0 = default */
    int32_t keys_on_host;       /* 1: key_cols are host pointers */
    int32_t variant;            /* form of the register-tile Householder QR:
                                   0 fully unrolled (triangular work), 1
                                   compact runtime column loop (smaller code,
                                   twice the arithmetic), 2 fully unrolled
                                   with a register budget for two waves per
                                   SIMD; other values give FIGARO_EINVAL */
    int32_t analyze_only;       /* 1: stop after the count queries; the plan
                                   then answers the info and count queries
                                   only, holds no device memory, and the
                                   compute calls return FIGARO_EINVAL */
    int32_t separate_join;      /* 1: always store the joined heads of a
                                   relation (process_and_join_children) before
                                   projecting the join attributes away; 0
                                   (default): a non-root relation with at most
                                   four children has its first project-away
                                   level read them in place instead */
    int32_t host_plan;          /* 1: build the plan on the host even when
                                   the keys are on the device (the keys are
                                   copied over); 0 (default): device keys are
                                   sorted, segmented and counted on the
                                   device.  Both give the same plan. */
} figaro_plan_options;

/* Count-query selectors for figaro_plan_counts(). */
typedef enum {
    FIGARO_COUNT_ROWS_PER_KEY = 0,   /* |S_i^{x_i}|, per key group x_i */
    FIGARO_COUNT_THETA_DOWN = 1,     /* Theta_i^down(x_i), per key group */
    FIGARO_COUNT_PHI_CIRC = 2,       /* Phi_i^o(x_i), per key group */
    FIGARO_COUNT_PHI_UP = 3,         /* Phi_i^up(x_p), per parent group */
    FIGARO_COUNT_PHI_DOWN = 4        /* Phi_i^down(x_p), per parent group */
} figaro_count_kind;

/*
 * Build a plan from the keys (section "Scaling Factors as Count Queries",
 * Algorithm 2, and the sort order both algorithms assume): validate the tree,
 * reduce dangling tuples, sort each relation on (attributes shared with the
 * parent, then its other key attributes, then row index), segment it into key
 * groups, evaluate the count queries exactly in 64-bit integers, derive the
 * scale factors, and allocate the workspace.  With device keys (the default)
 * the dictionary encoding, the reduction, the radix sort, the segments, the
 * child indices, the counts and the first level of every head/tail task are
 * computed on the device, on `stream`, which the call synchronises a few
 * times; host keys (or host_plan) run the same steps on the host.
 */
figaro_status figaro_plan_create(figaro_plan_t *out, int32_t r,
                                 const figaro_relation_desc *rels,
                                 const figaro_plan_options *opts,
                                 hipStream_t stream);
void figaro_plan_destroy(figaro_plan_t plan);

int32_t figaro_plan_num_relations(figaro_plan_t plan);
int32_t figaro_plan_num_cols(figaro_plan_t plan);                 /* n */
int64_t figaro_plan_input_rows(figaro_plan_t plan, int32_t rel);  /* m_i as given */
int64_t figaro_plan_rows(figaro_plan_t plan, int32_t rel);        /* rows kept in plan order */
int64_t figaro_plan_dropped_rows(figaro_plan_t plan, int32_t rel);/* dangling tuples removed */
double  figaro_plan_join_rows(figaro_plan_t plan);                /* |A|, exact below 2^53 */
int64_t figaro_plan_workspace_bytes(figaro_plan_t plan);

/* perm_host[p] (p < input rows) is the caller row placed at plan row p; the
 * kept rows come first, the dropped rows after them.  Host output. */
figaro_status figaro_plan_permutation(figaro_plan_t plan, int32_t rel, int64_t *perm_host);

/* Number of key groups (which = 0: groups of x_i) or parent groups (which = 1:
 * groups of x_p) of relation rel; -1 on error. */
int64_t figaro_plan_num_groups(figaro_plan_t plan, int32_t rel, int32_t which);
/* Caller row index of the first plan row of every group (host output). */
figaro_status figaro_plan_group_first_rows(figaro_plan_t plan, int32_t rel, int32_t which,
                                           int64_t *rows_host);
/* Exact count-query values per group (host output). */
figaro_status figaro_plan_counts(figaro_plan_t plan, int32_t rel, figaro_count_kind kind,
                                 int64_t *out_host);

/* dst (plan order, leading dim ld_dst) <- src (caller order, leading dim
 * ld_src) for the kept rows of relation rel; device pointers, enqueued. */
figaro_status figaro_permute_values(figaro_plan_t plan, int32_t rel, const double *src,
                                    int64_t ld_src, double *dst, int64_t ld_dst,
                                    hipStream_t stream);
/* dst (caller order) <- src (plan order); rows dropped by the reduction get 0.
 * Used to return gradients in the caller's row order. */
figaro_status figaro_unpermute_values(figaro_plan_t plan, int32_t rel, const double *src,
                                      int64_t ld_src, double *dst, int64_t ld_dst,
                                      hipStream_t stream);

/*
 * Forward: R of the join (Algorithm 3 followed by the post-processing QR of
 * the section "Post-processing", then a non-negative diagonal).
 *   values[i]: device, plan order, column-major with leading dim ld[i] >= rows
 *   R: device, n x n column-major; the strictly lower part is written as 0.
 * Enqueued on `stream`; no allocation, no host synchronisation.
 */
figaro_status figaro_r(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                       double *R, hipStream_t stream);

/*
 * Backward: gradients of a scalar loss with respect to every relation's values,
 * given dR = dLoss/dR.  Only the upper triangle of dR is used (the strictly
 * lower part of R is structurally zero).  The paper has no backward pass; this
 * is the adjoint of the forward computation: with
 *   K = R^{-1} copyltu(R triu(dR)^T) R^{-T},  copyltu(M) = tril(M) + tril(M,-1)^T,
 * the gradient of the join matrix is A K (the adjoint of the R factor of a QR
 * decomposition), and the library pushes the gradients of the R0 rows (R0 K on
 * each row's non-zero columns) back through the head/tail recurrences, the
 * join of the children's heads and the root heads, recomputing the forward
 * intermediates instead of storing them.
 *   values, ld : as for figaro_r (plan order)
 *   R          : the R that figaro_r returned for these values (n x n)
 *   dR         : device n x n column-major
 *   dvalues[i] : device output, plan order, leading dim ld_dvalues[i] >= rows;
 *                every kept row is written
 * Enqueued on `stream`; no allocation, no host synchronisation.  A zero on
 * the diagonal of R makes the gradient non-finite; figaro_backward_status()
 * synchronises `stream` and reports FIGARO_ESINGULAR in that case.
 */
figaro_status figaro_r_backward(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                                const double *R, const double *dR, double *const *dvalues,
                                const int64_t *ld_dvalues, hipStream_t stream);
figaro_status figaro_backward_status(figaro_plan_t plan, hipStream_t stream);

/*
 * The intermediate matrix R0 of Theorem 6 (heads and tails before the
 * post-processing QR), materialised for inspection: figaro_r0_rows() rows of
 * n columns, column-major with leading dimension ld_r0.  block_of_row
 * (device int32, may be NULL) receives for each row the id of the block that
 * produced it: 3*i + 0 for tails of relation i (heads_and_tails), 3*i + 1 for
 * generalized tails of relation i (project_away_join_attributes), 3*i + 2 for
 * the heads emitted at the root.  Rows that carry no tail are zero.
 */
int64_t figaro_r0_rows(figaro_plan_t plan);
figaro_status figaro_r0(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                        double *R0, int64_t ld_r0, int32_t *block_of_row, hipStream_t stream);

/*
 * The post-processing QR (section "Post-processing") of a plain matrix: R
 * of the rows x n FP64 matrix A (device, column-major, leading dimension lda
 * >= max(rows, 1)), e.g. the R0 that figaro_r0() materialises, by the same
 * TSQR levels as figaro_r(): partial R's of row tiles, folded level by level,
 * the last level sign-normalised.  R: device n x n column-major, the strictly
 * lower part written as 0.  1 <= n <= 128 (FIGARO_EUNSUPPORTED otherwise);
 * rows may be 0 (R = 0; A may then be NULL).  The partial R's of the levels live in `workspace`
 * (device, caller-owned, at least figaro_tsqr_workspace_bytes(rows, n)
 * bytes, at most 8 MiB for any size; FIGARO_EINVAL if smaller), which the
 * call may overwrite; it must not be used by another call in flight.
 * Enqueued on `stream`; no allocation, no host synchronisation.
 */
int64_t figaro_tsqr_workspace_bytes(int64_t rows, int32_t n);   /* -1 for an unsupported n */
figaro_status figaro_tsqr(int64_t rows, int32_t n, const double *A, int64_t lda, double *R,
                          void *workspace, int64_t workspace_bytes, hipStream_t stream);

/*
 * figaro_tsqr() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same levels and kernels, and the same R bit for bit, with the partial
 * R's in a static 8 MiB device array of the library instead of a workspace.
 * Each GPU holds its own copy of the array from the first call on it (its
 * address is looked up then, with that device current) until the process
 * ends.  Arguments as for figaro_tsqr(); any row count works (the levels are
 * shaped to fit the array), n beyond 128 gives FIGARO_EUNSUPPORTED.  Every
 * call on a GPU uses that GPU's one array: calls that may overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * Allocates nothing; enqueued on `stream`, no host synchronisation.
 */
figaro_status figaro_tsqr_noalloc(int64_t rows, int32_t n, const double *A, int64_t lda, double *R,
                                  hipStream_t stream);

/*
 * From R to Q, SVD and PCA (section "From R to Q, SVD and PCA").
 *
 * figaro_svd_r(): R = U_R Sigma V^T for an n x n matrix R (device, column-
 * major, 1 <= n <= 128), by one-sided Jacobi rotations; sigma (device [n])
 * in decreasing order, V and U_R (device n x n column-major; U may be NULL)
 * with matching columns.  For the R of a join matrix A, sigma and V are the
 * singular values and right singular vectors of A, and V's columns its
 * principal components.  Each column of U_R and V is determined up to sign
 * (up to a rotation within repeated singular values).  work: device, at
 * least 2 n^2 doubles, overwritten.  Enqueued on `stream`.
 *
 * figaro_r_inverse(): R^-1 of an upper-triangular n x n R with non-zero
 * diagonal (device, column-major), enqueued on `stream`.
 *
 * figaro_join_multiply(): rows row0 .. row0 + nrows - 1 of A M, for the join
 * matrix A of the plan (never materialised) and an n x k matrix M (device,
 * column-major, leading dimension ldm >= n, 1 <= k <= 128), each column c
 * multiplied by col_scale[c] when col_scale (device [k]) is not NULL:
 * out (device, column-major [k][ld_out], ld_out >= nrows).  With M = R^-1
 * the rows are those of Q (A = QR); with M = V and col_scale = 1 / sigma
 * those of the left singular vectors U; with M = V[:, :k] the PCA
 * projection.  The join rows come in a fixed order: root key groups in
 * plan order; within a key group its tuples in plan order, each followed by
 * the combinations of its children's subtree rows (first child slowest).
 * tuple_ids (device int64 [r][ld_ids], may be NULL) receives, for every
 * output row, the caller row index of the tuple each relation contributes.
 * values / ld as for figaro_r (plan order).  work: device, at least
 * figaro_join_multiply_workspace_bytes(plan, k) bytes (the dot products of
 * every tuple with the rows of M).  At most 16 relations.  Enqueued on
 * `stream`; no allocation.
 */
figaro_status figaro_svd_r(int32_t n, const double *R, double *sigma, double *U, double *V, double *work,
                           hipStream_t stream);
figaro_status figaro_r_inverse(int32_t n, const double *R, double *Rinv, hipStream_t stream);
int64_t figaro_join_multiply_workspace_bytes(figaro_plan_t plan, int32_t k);   /* -1 on error */
figaro_status figaro_join_multiply(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                                   const double *M, int64_t ldm, int32_t k, const double *col_scale,
                                   int64_t row0, int64_t nrows, double *out, int64_t ld_out,
                                   int64_t *tuple_ids, int64_t ld_ids, void *work, int64_t work_bytes,
                                   hipStream_t stream);

/*
 * Per-kernel timing for benchmarks.  While enabled, the compute calls record a
 * pair of HIP events on the caller's stream around every kernel launch, in a
 * pool of `capacity` pairs (events are created here, not in the compute
 * calls; launches beyond the pool are not timed).  figaro_profile_read()
 * waits for the recorded events, adds their durations to the totals of each
 * kernel class, and frees the pool slots.  Classes:
 *   0 heads_and_tails, first level (unit-count tails + QR accumulation)
 *   1 project_away_join_attributes, first level (weighted tails + QR)
 *   2 upper levels of both (combination of tiles of one key group)
 *   3 process_and_join_children
 *   4 root heads
 *   5 post-processing TSQR over the stack of partial R factors
 *   6 backward kernels
 * For each class the totals hold: elapsed milliseconds, launches, the
 * algorithmic bytes (values read, for classes 0-2; gathered and written rows
 * for 3-4; stack rows read for 5) and the QR flops (2 m n^2 per launch).
 */
figaro_status figaro_profile_enable(figaro_plan_t plan, int32_t capacity);   /* 0 disables */
figaro_status figaro_profile_read(figaro_plan_t plan, int32_t kernel_class, double *ms,
                                  int64_t *launches, double *bytes, double *flops);
figaro_status figaro_profile_reset(figaro_plan_t plan);

/* Message of the last failing call on `plan` (NULL: on the calling thread). */
const char *figaro_last_error(figaro_plan_t plan);

/*
 * Batches: many independent join instances (each with its own plan) in one
 * call, for serving.  Each instance is the computation of figaro_r (or
 * figaro_r_backward) on its own plan; the paper treats one join at a time,
 * and a batch is simply the independent instances side by side.
 *
 * figaro_batch_create() takes `count` distinct plans (the batch does not own
 * them; they must outlive it) and creates `streams` HIP streams (<= 0: 8) of
 * default priority; instances are assigned to streams longest-first by an
 * estimate of their work.  Errors: FIGARO_EINVAL for a NULL, analyze-only or
 * repeated plan; FIGARO_EHIP if a stream or event cannot be created.
 * Messages go to figaro_last_error(NULL).
 *
 * figaro_r_batched(): R[i] <- R of instance i, with values[i] / ld[i] as for
 * figaro_r on plans[i] (plan order, device).  The batch forks from `stream`
 * with an event, runs every instance on its assigned stream, and joins back
 * into `stream`: work enqueued later on `stream` sees every R.  No
 * allocation, no host synchronisation.  On an argument error in instance i
 * the other instances still run; the first error is returned.
 *
 * figaro_r_backward_batched(): the same for figaro_r_backward, per instance.
 *
 * Per-launch timing (figaro_profile_enable) must be disabled on every plan
 * of a batch: figaro_r_batched(), figaro_r_backward_batched() and
 * figaro_batch_capture() return FIGARO_EINVAL otherwise (a plan's timing
 * events are recorded on one stream and read back on the host).
 *
 * figaro_batch_capture(): captures the sequence of figaro_r_batched() with
 * these pointers into a HIP graph (stream capture on `stream`, which must not
 * be the null stream), replacing any graph captured before.  figaro_batch_launch() replays it on a stream:
 * the buffers captured are read and written again.  Concurrent use of one
 * batch (or of its plans) must be serialised by the caller.
 */
typedef struct figaro_batch_s *figaro_batch_t;
figaro_status figaro_batch_create(figaro_batch_t *out, int32_t count, const figaro_plan_t *plans,
                                  int32_t streams);
void figaro_batch_destroy(figaro_batch_t batch);
int32_t figaro_batch_stream_of(figaro_batch_t batch, int32_t instance);   /* -1 if out of range */
figaro_status figaro_r_batched(figaro_batch_t batch, const double *const *const *values,
                               const int64_t *const *ld, double *const *R, hipStream_t stream);
figaro_status figaro_r_backward_batched(figaro_batch_t batch, const double *const *const *values,
                                        const int64_t *const *ld, const double *const *R,
                                        const double *const *dR, double *const *const *dvalues,
                                        const int64_t *const *ld_dvalues, hipStream_t stream);
figaro_status figaro_batch_capture(figaro_batch_t batch, const double *const *const *values,
                                   const int64_t *const *ld, double *const *R, hipStream_t stream);
figaro_status figaro_batch_launch(figaro_batch_t batch, hipStream_t stream);

/*
 * Join-tree selection (experiments section, "Effect of join trees": the
 * method runs fastest on the join tree with the smallest intermediate
 * results, which keeps a large fact table away from the root so that its
 * join attributes are aggregated away early).  A join tree here is a
 * spanning tree over the relations in which the relations holding any one
 * attribute stay connected (running intersection) and every key attribute is
 * shared with a neighbour; any relation may be the root.  The score of a
 * rooted tree is the work of the QR of R0, rows x columns^2 summed over its
 * blocks:
 *   sum_i (m_i - G_i) n_i^2 + sum_{i not root} (G_i - P_i) nsub_i^2 + G_root n^2
 * with m_i the rows, n_i the columns and G_i the distinct values of the join
 * attributes of relation i, P_i the distinct values of those it shares with
 * its parent, nsub_i the columns of its subtree, n the total (dangling
 * tuples are not removed first: for a database that is not fully reduced the
 * score is an estimate).  Keys as in figaro_relation_desc (host arrays when
 * keys_on_host is 1, else device arrays read on `stream`, which is then
 * synchronised); r <= 12.
 *
 * figaro_join_tree_cost(): the score of the tree given by rels[i].parent
 * (FIGARO_ENOTTREE if it is not a join tree).
 * figaro_choose_join_tree(): the lowest-scoring join tree over every join
 * tree and root (rels[i].parent is ignored); parents_out[i] receives the
 * parent of relation i (-1 for the root), *cost_out (may be NULL) its score.
 * Relations that share no attributes are linked by Cartesian products only
 * when the shared attributes alone leave them disconnected.
 * FIGARO_ENOTTREE if no join tree exists (a cyclic join).  Host only.
 */
figaro_status figaro_join_tree_cost(int32_t r, const figaro_relation_desc *rels, int32_t keys_on_host,
                                    double *cost_out, hipStream_t stream);
figaro_status figaro_choose_join_tree(int32_t r, const figaro_relation_desc *rels, int32_t keys_on_host,
                                      int32_t *parents_out, double *cost_out, hipStream_t stream);

/*
 * Autotuner: builds the plan under each option set of `candidates`
 * (ncandidates <= 0 or NULL: register-tile variants 0 and 2 times wave caps
 * 512, 1024, 2048; analyze_only is ignored), times `reps` forward passes of
 * each on the caller's values (values[i]: device, caller order, column-major,
 * ld[i] >= rows; they are copied into plan order in a temporary buffer), and
 * returns the fastest plan.  Candidates the instance cannot use are skipped;
 * FIGARO_EUNSUPPORTED if none works.  Allocates and synchronises `stream`
 * (a planning call, not a compute call).  figaro_plan_tuning() reports the
 * option set chosen and its time per pass in milliseconds (FIGARO_EINVAL for
 * a plan not built here).
 */
figaro_status figaro_plan_create_tuned(figaro_plan_t *out, int32_t r, const figaro_relation_desc *relations,
                                       const double *const *values, const int64_t *ld, int32_t ncandidates,
                                       const figaro_plan_options *candidates, int32_t reps, hipStream_t stream);
figaro_status figaro_plan_tuning(figaro_plan_t plan, figaro_plan_options *chosen, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* FIGARO_H */
