/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, single-threaded reference code for the upper-triangular factor
 * R of the QR decomposition of the data columns of an acyclic natural join.
 * Only the test-suite, the smoke check and the CPU baseline leg of the
 * benchmark may load this library.  It shares no code with the HIP library.
 *
 * What is computed, and from which passage of the paper:
 *   - the natural join of the relations, by index nested loops along the join
 *     tree (setup section: relations, natural join, join tree; bag semantics);
 *   - the textbook Householder QR of the join matrix (Golub & Van Loan), with
 *     R normalised to a non-negative diagonal, which makes R unique for a
 *     full-rank input (setup section, "Output");
 *   - a brute-force Givens QR with the rotation of Definition 1 and Bindel's
 *     sign choice (related-work section), used to cross-check the above;
 *   - A^T A in long double and log det(A^T A) by LU in long double;
 *   - an at-scale reference that never materialises the join: A^T A is summed
 *     by distributivity over the join tree (first moments only, anchored at
 *     each relation in turn), then factorised by a Cholesky decomposition in
 *     __float128.  R = chol(A^T A) is the plain definition of R.
 *
 * Conventions: matrices are column-major; relation keys are int64 arrays of
 * shape [k][m]; relation values are double arrays of shape [n][m].
 */
#define _GNU_SOURCE
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t m;              /* rows */
    int32_t k;              /* number of key attributes */
    const int32_t *attrs;   /* [k] global attribute ids */
    const int64_t *keys;    /* [k][m] */
    int32_t n;              /* number of data columns */
    const double *vals;     /* [n][m] */
    int32_t parent;         /* -1 for the root */
} orel;

/* ------------------------------------------------------------------------ */
/* Small helpers: attribute positions, key-tuple sorting and lookup.         */
/* ------------------------------------------------------------------------ */

static int attr_pos(const orel *R, int32_t a) {
    for (int i = 0; i < R->k; ++i)
        if (R->attrs[i] == a) return i;
    return -1;
}

/* shared attributes between relations a and b, as positions in each */
static int shared_attrs(const orel *A, const orel *B, int *pa, int *pb) {
    int c = 0;
    for (int i = 0; i < A->k; ++i) {
        int j = attr_pos(B, A->attrs[i]);
        if (j >= 0) { pa[c] = i; pb[c] = j; ++c; }
    }
    return c;
}

typedef struct {
    const orel *R;
    const int *pos;
    int npos;
} sort_ctx;

static int cmp_rows(const void *x, const void *y, void *arg) {
    const sort_ctx *c = (const sort_ctx *)arg;
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    for (int i = 0; i < c->npos; ++i) {
        int64_t ka = c->R->keys[(int64_t)c->pos[i] * c->R->m + a];
        int64_t kb = c->R->keys[(int64_t)c->pos[i] * c->R->m + b];
        if (ka < kb) return -1;
        if (ka > kb) return 1;
    }
    return (a > b) - (a < b);
}

/* An index of relation R's rows, sorted by the key attributes at `pos`. */
typedef struct {
    const orel *R;
    int pos[64];
    int npos;
    int64_t *order;   /* [m] row ids sorted by key tuple */
} row_index;

static int rindex_build(row_index *ix, const orel *R, const int *pos, int npos) {
    ix->R = R;
    ix->npos = npos;
    for (int i = 0; i < npos; ++i) ix->pos[i] = pos[i];
    ix->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->m > 0 ? R->m : 1));
    if (!ix->order) return -1;
    for (int64_t i = 0; i < R->m; ++i) ix->order[i] = i;
    sort_ctx c = {R, ix->pos, npos};
    qsort_r(ix->order, (size_t)R->m, sizeof(int64_t), cmp_rows, &c);
    return 0;
}

/* compare the key tuple of row `r` (in the index's relation) to a probe tuple */
static int cmp_probe(const row_index *ix, int64_t r, const int64_t *probe) {
    for (int i = 0; i < ix->npos; ++i) {
        int64_t k = ix->R->keys[(int64_t)ix->pos[i] * ix->R->m + r];
        if (k < probe[i]) return -1;
        if (k > probe[i]) return 1;
    }
    return 0;
}

/* range [lo, hi) of index entries whose key tuple equals probe */
static void rindex_range(const row_index *ix, const int64_t *probe, int64_t *lo, int64_t *hi) {
    int64_t a = 0, b = ix->R->m;
    while (a < b) {
        int64_t mid = (a + b) / 2;
        if (cmp_probe(ix, ix->order[mid], probe) < 0) a = mid + 1; else b = mid;
    }
    *lo = a;
    b = ix->R->m;
    while (a < b) {
        int64_t mid = (a + b) / 2;
        if (cmp_probe(ix, ix->order[mid], probe) <= 0) a = mid + 1; else b = mid;
    }
    *hi = a;
}

/* ------------------------------------------------------------------------ */
/* Join materialisation by index nested loops along the join tree.           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int r;
    const orel *rels;
    int *order;            /* pre-order of the join tree */
    row_index *ix;            /* per relation: index on the attributes shared with its parent */
    int (*ppos)[64];       /* per relation: positions of the shared attrs in the parent */
    int *npp;
    int64_t *cur;          /* current row per relation */
    int64_t *col_off;      /* global column offset per relation */
    double *A;             /* output, column-major, may be NULL (count only) */
    int64_t *idx;          /* output tuple indices [r][lda], may be NULL */
    int64_t lda;
    int64_t rows;          /* rows emitted so far */
    int64_t max_rows;
    int overflow;
} join_ctx;

static void join_rec(join_ctx *c, int depth) {
    if (c->overflow) return;
    if (depth == c->r) {
        if (c->idx) {
            if (c->rows >= c->max_rows) { c->overflow = 1; return; }
            for (int i = 0; i < c->r; ++i) c->idx[(int64_t)i * c->lda + c->rows] = c->cur[i];
        }
        if (c->A) {
            if (c->rows >= c->max_rows) { c->overflow = 1; return; }
            for (int i = 0; i < c->r; ++i) {
                const orel *R = &c->rels[i];
                for (int col = 0; col < R->n; ++col)
                    c->A[(c->col_off[i] + col) * c->lda + c->rows] = R->vals[(int64_t)col * R->m + c->cur[i]];
            }
        }
        c->rows++;
        return;
    }
    int i = c->order[depth];
    const orel *R = &c->rels[i];
    if (R->parent < 0) {
        for (int64_t t = 0; t < R->m; ++t) { c->cur[i] = t; join_rec(c, depth + 1); }
        return;
    }
    const orel *P = &c->rels[R->parent];
    int64_t probe[64];
    for (int a = 0; a < c->npp[i]; ++a)
        probe[a] = P->keys[(int64_t)c->ppos[i][a] * P->m + c->cur[R->parent]];
    int64_t lo, hi;
    rindex_range(&c->ix[i], probe, &lo, &hi);
    for (int64_t q = lo; q < hi; ++q) { c->cur[i] = c->ix[i].order[q]; join_rec(c, depth + 1); }
}

static int preorder(int r, const orel *rels, int *order) {
    int root = -1, cnt = 0;
    for (int i = 0; i < r; ++i)
        if (rels[i].parent < 0) { if (root >= 0) return -1; root = i; }
    if (root < 0) return -1;
    int *stack = (int *)malloc(sizeof(int) * (size_t)r);
    int sp = 0;
    stack[sp++] = root;
    while (sp) {
        int v = stack[--sp];
        if (cnt >= r) { free(stack); return -1; }
        order[cnt++] = v;
        for (int j = r - 1; j >= 0; --j)
            if (rels[j].parent == v) stack[sp++] = j;
    }
    free(stack);
    return cnt == r ? 0 : -1;
}

/* Enumerate the join. If A != NULL, write rows (column-major, leading dim lda,
 * at most max_rows). Returns the number of join rows, or -1 on error, -2 if
 * max_rows was exceeded. */
int64_t or_join(int r, const orel *rels, double *A, int64_t lda, int64_t max_rows) {
    join_ctx c;
    memset(&c, 0, sizeof c);
    c.r = r;
    c.rels = rels;
    c.order = (int *)malloc(sizeof(int) * (size_t)r);
    c.ix = (row_index *)calloc((size_t)r, sizeof(row_index));
    c.ppos = malloc(sizeof(int[64]) * (size_t)r);
    c.npp = (int *)calloc((size_t)r, sizeof(int));
    c.cur = (int64_t *)calloc((size_t)r, sizeof(int64_t));
    c.col_off = (int64_t *)calloc((size_t)r, sizeof(int64_t));
    int64_t result = -1;
    if (preorder(r, rels, c.order) != 0) goto done;
    for (int i = 1; i < r; ++i) c.col_off[i] = c.col_off[i - 1] + rels[i - 1].n;
    for (int i = 0; i < r; ++i) {
        if (rels[i].parent < 0) continue;
        int pc[64], pp[64];
        int ns = shared_attrs(&rels[i], &rels[rels[i].parent], pc, pp);
        c.npp[i] = ns;
        for (int a = 0; a < ns; ++a) c.ppos[i][a] = pp[a];
        if (rindex_build(&c.ix[i], &rels[i], pc, ns) != 0) goto done;
    }
    c.A = A;
    c.lda = lda;
    c.max_rows = max_rows;
    join_rec(&c, 0);
    result = c.overflow ? -2 : c.rows;
done:
    for (int i = 0; i < r; ++i) free(c.ix[i].order);
    free(c.order); free(c.ix); free(c.ppos); free(c.npp); free(c.cur); free(c.col_off);
    return result;
}

/* The join as tuple indices: idx[i*lda + row] is the tuple of relation i in
 * join row `row` (same row order as or_join). */
int64_t or_join_idx(int r, const orel *rels, int64_t *idx, int64_t lda, int64_t max_rows) {
    join_ctx c;
    memset(&c, 0, sizeof c);
    c.r = r;
    c.rels = rels;
    c.order = (int *)malloc(sizeof(int) * (size_t)r);
    c.ix = (row_index *)calloc((size_t)r, sizeof(row_index));
    c.ppos = malloc(sizeof(int[64]) * (size_t)r);
    c.npp = (int *)calloc((size_t)r, sizeof(int));
    c.cur = (int64_t *)calloc((size_t)r, sizeof(int64_t));
    c.col_off = (int64_t *)calloc((size_t)r, sizeof(int64_t));
    int64_t result = -1;
    if (preorder(r, rels, c.order) != 0) goto done;
    for (int i = 0; i < r; ++i) {
        if (rels[i].parent < 0) continue;
        int pc[64], pp[64];
        int ns = shared_attrs(&rels[i], &rels[rels[i].parent], pc, pp);
        c.npp[i] = ns;
        for (int a = 0; a < ns; ++a) c.ppos[i][a] = pp[a];
        if (rindex_build(&c.ix[i], &rels[i], pc, ns) != 0) goto done;
    }
    c.idx = idx;
    c.lda = lda;
    c.max_rows = max_rows;
    join_rec(&c, 0);
    result = c.overflow ? -2 : c.rows;
done:
    for (int i = 0; i < r; ++i) free(c.ix[i].order);
    free(c.order); free(c.ix); free(c.ppos); free(c.npp); free(c.cur); free(c.col_off);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Textbook Householder QR (R only), then a non-negative diagonal.           */
/* ------------------------------------------------------------------------ */

/* 2-norm with scaling, as the reference BLAS dnrm2 does, to avoid overflow */
static double scaled_norm(const double *x, int64_t len) {
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < len; ++i) {
        if (x[i] != 0.0) {
            double a = fabs(x[i]);
            if (scale < a) { ssq = 1.0 + ssq * (scale / a) * (scale / a); scale = a; }
            else { ssq += (a / scale) * (a / scale); }
        }
    }
    return scale * sqrt(ssq);
}

static void sign_normalise(int n, double *R) {
    for (int i = 0; i < n; ++i) {
        if (R[(int64_t)i * n + i] < 0.0)
            for (int j = i; j < n; ++j) R[(int64_t)j * n + i] = -R[(int64_t)j * n + i];
    }
}

/* A is m x n, column-major with leading dimension lda; it is overwritten.
 * R receives the n x n upper-triangular factor (column-major, ld n), with a
 * non-negative diagonal and zeros below the diagonal.  Returns the number of
 * zero diagonal entries (0 for a full-rank input).  Requires m >= 0. */
int or_householder_r(int64_t m, int32_t n, double *A, int64_t lda, double *R) {
    double *v = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int j = 0; j < n && j < m; ++j) {
        double *x = A + (int64_t)j * lda + j;
        int64_t len = m - j;
        double nrm = scaled_norm(x, len);
        if (nrm == 0.0) continue;
        double alpha = (x[0] >= 0.0) ? -nrm : nrm;       /* sign(0) = +1 */
        for (int64_t i = 0; i < len; ++i) v[i] = x[i];
        v[0] -= alpha;
        double vtv = 0.0;
        for (int64_t i = 0; i < len; ++i) vtv += v[i] * v[i];
        double beta = 2.0 / vtv;
        for (int k = j; k < n; ++k) {
            double *a = A + (int64_t)k * lda + j;
            double w = 0.0;
            for (int64_t i = 0; i < len; ++i) w += v[i] * a[i];
            w *= beta;
            for (int64_t i = 0; i < len; ++i) a[i] -= w * v[i];
        }
    }
    free(v);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            R[(int64_t)j * n + i] = (i <= j && i < m) ? A[(int64_t)j * lda + i] : 0.0;
    sign_normalise(n, R);
    int zeros = 0;
    for (int i = 0; i < n; ++i) if (R[(int64_t)i * n + i] == 0.0) ++zeros;
    return zeros;
}

/* Brute-force Givens QR: for each column j, zero the entries below the
 * diagonal from the bottom up, rotating row i against the pivot row j.
 * The rotation follows Definition 1 with Bindel's choice:
 *   h = sqrt(a^2 + b^2), cos = |a| / h, sin = -sign(a) b / h, sign(0) = +1,
 * which maps (a, b) to (sign(a) h, 0).  A is overwritten. */
int or_givens_r(int64_t m, int32_t n, double *A, int64_t lda, double *R) {
    for (int j = 0; j < n && j < m; ++j) {
        for (int64_t i = m - 1; i > j; --i) {
            double a = A[(int64_t)j * lda + j];
            double b = A[(int64_t)j * lda + i];
            if (b == 0.0) continue;
            double h = hypot(a, b);
            double sg = (a >= 0.0) ? 1.0 : -1.0;
            double cs = fabs(a) / h;
            double sn = -sg * b / h;
            for (int k = j; k < n; ++k) {
                double xi = A[(int64_t)k * lda + j];   /* pivot row */
                double xj = A[(int64_t)k * lda + i];   /* row to zero */
                A[(int64_t)k * lda + j] = xi * cs - xj * sn;
                A[(int64_t)k * lda + i] = xi * sn + xj * cs;
            }
            A[(int64_t)j * lda + i] = 0.0;
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            R[(int64_t)j * n + i] = (i <= j && i < m) ? A[(int64_t)j * lda + i] : 0.0;
    sign_normalise(n, R);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Checks in long double.                                                    */
/* ------------------------------------------------------------------------ */

/* G = A^T A (n x n, column-major) accumulated in long double, returned as a
 * pair of doubles (hi + lo) per entry. */
void or_gram_ld(int64_t m, int32_t n, const double *A, int64_t lda, double *Ghi, double *Glo) {
    for (int a = 0; a < n; ++a)
        for (int b = 0; b <= a; ++b) {
            long double s = 0.0L;
            for (int64_t i = 0; i < m; ++i)
                s += (long double)A[(int64_t)a * lda + i] * (long double)A[(int64_t)b * lda + i];
            double hi = (double)s;
            double lo = (double)(s - (long double)hi);
            Ghi[(int64_t)a * n + b] = Ghi[(int64_t)b * n + a] = hi;
            Glo[(int64_t)a * n + b] = Glo[(int64_t)b * n + a] = lo;
        }
}

/* || R^T R - G ||_F / || G ||_F with R^T R formed in long double and G given
 * as hi + lo pairs. */
double or_gram_relerr(int32_t n, const double *R, const double *Ghi, const double *Glo) {
    long double num = 0.0L, den = 0.0L;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            long double s = 0.0L;
            for (int k = 0; k < n; ++k)
                s += (long double)R[(int64_t)a * n + k] * (long double)R[(int64_t)b * n + k];
            long double g = (long double)Ghi[(int64_t)a * n + b] + (long double)Glo[(int64_t)a * n + b];
            num += (s - g) * (s - g);
            den += g * g;
        }
    return den > 0.0L ? (double)sqrtl(num / den) : (double)sqrtl(num);
}

/* log |det G| by LU with partial pivoting in long double; G given as hi+lo. */
double or_logabsdet(int32_t n, const double *Ghi, const double *Glo) {
    long double *M = (long double *)malloc(sizeof(long double) * (size_t)n * (size_t)n);
    for (int64_t i = 0; i < (int64_t)n * n; ++i) M[i] = (long double)Ghi[i] + (long double)Glo[i];
    long double logdet = 0.0L;
    for (int j = 0; j < n; ++j) {
        int p = j;
        for (int i = j + 1; i < n; ++i)
            if (fabsl(M[(int64_t)j * n + i]) > fabsl(M[(int64_t)j * n + p])) p = i;
        long double piv = M[(int64_t)j * n + p];
        if (piv == 0.0L) { free(M); return -INFINITY; }
        if (p != j)
            for (int k = 0; k < n; ++k) {
                long double t = M[(int64_t)k * n + j];
                M[(int64_t)k * n + j] = M[(int64_t)k * n + p];
                M[(int64_t)k * n + p] = t;
            }
        logdet += logl(fabsl(piv));
        for (int i = j + 1; i < n; ++i) {
            long double f = M[(int64_t)j * n + i] / piv;
            for (int k = j; k < n; ++k) M[(int64_t)k * n + i] -= f * M[(int64_t)k * n + j];
        }
    }
    free(M);
    return (double)logdet;
}

/* ------------------------------------------------------------------------ */
/* At-scale reference: A^T A by distributivity over the join tree, then a    */
/* Cholesky factorisation in __float128.                                      */
/* ------------------------------------------------------------------------ */

/*
 * Anchor relation k.  Re-root the tree at k.  For every other relation j,
 * bottom-up, build a message keyed by the attributes j shares with its new
 * parent: for each key value, the number of rows of the join of the subtree
 * of j with that key (count) and the sums of every data column of the
 * subtree over those rows.  At the anchor, each of its rows t contributes
 *   w_t * y_t y_t^T                           to block (k, k),
 *   y_t (sums of the other side)^T            to blocks (k, l),
 * where w_t is the number of join rows that contain t.  Every quantity is a
 * sum over join rows, grouped by key, so this is A^T A by definition.
 * Counts are exact in __float128 (< 2^113); column sums are accumulated in
 * long double per row and per key in __float128.
 */

typedef struct {
    int64_t nkeys;
    int64_t *key_rows;   /* representative row of S_j for each key value */
    int kpos[64];        /* positions of the shared attributes within S_j */
    int nk;
    __float128 *cnt;     /* [nkeys] */
    __float128 *sum;     /* [nkeys][width] */
    int width;           /* number of data columns in the subtree */
    int *cols;           /* [width] global column ids of the subtree, ascending */
    row_index ix;           /* index of S_j rows on kpos (for grouping) */
    int64_t *grp_of_row; /* [m_j] key group of each row */
} message;

typedef struct {
    int r;
    const orel *rels;
    int *col_off;
    int **adj;
    int *deg;
} tree_info;

static int key_equal_rows(const orel *R, const int *pos, int np, int64_t a, int64_t b) {
    for (int i = 0; i < np; ++i)
        if (R->keys[(int64_t)pos[i] * R->m + a] != R->keys[(int64_t)pos[i] * R->m + b]) return 0;
    return 1;
}

/* find key group in message `msg` for a probe row `t` of relation P, where
 * ppos are the positions in P of msg's shared attributes; -1 if absent. */
static int64_t msg_lookup(const message *msg, const orel *P, const int *ppos, int64_t t) {
    int64_t probe[64];
    for (int i = 0; i < msg->nk; ++i) probe[i] = P->keys[(int64_t)ppos[i] * P->m + t];
    int64_t lo, hi;
    rindex_range(&msg->ix, probe, &lo, &hi);
    if (lo >= hi) return -1;
    return msg->grp_of_row[msg->ix.order[lo]];
}

/* Rows of R grouped by all of R's key attributes: order[] sorted by key,
 * gstart[g]..gstart[g+1] the rows of group g. */
typedef struct {
    row_index ix;
    int64_t *gstart;
    int64_t ngroups;
} full_groups;

static int full_groups_build(full_groups *F, const orel *R) {
    int pos[64];
    for (int i = 0; i < R->k; ++i) pos[i] = i;
    if (rindex_build(&F->ix, R, pos, R->k) != 0) return -1;
    F->gstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->m + 1));
    int64_t g = 0;
    for (int64_t q = 0; q < R->m; ++q)
        if (q == 0 || !key_equal_rows(R, pos, R->k, F->ix.order[q], F->ix.order[q - 1])) F->gstart[g++] = q;
    F->gstart[g] = R->m;
    F->ngroups = g;
    return 0;
}

static void full_groups_free(full_groups *F) { free(F->ix.order); free(F->gstart); }

/* build messages for the subtree of j (re-rooted, coming from `from`), post-order */
static int build_message(tree_info *T, message *msgs, int j, int from) {
    const orel *R = &T->rels[j];
    int nch = 0;
    int ch[64];
    for (int d = 0; d < T->deg[j]; ++d)
        if (T->adj[j][d] != from) ch[nch++] = T->adj[j][d];
    for (int c = 0; c < nch; ++c)
        if (build_message(T, msgs, ch[c], j) != 0) return -1;
    message *M = &msgs[j];
    int pj[64], pf[64];
    M->nk = shared_attrs(R, &T->rels[from], pj, pf);
    for (int i = 0; i < M->nk; ++i) M->kpos[i] = pj[i];
    int w = R->n;
    for (int c = 0; c < nch; ++c) w += msgs[ch[c]].width;
    M->width = w;
    M->cols = (int *)malloc(sizeof(int) * (size_t)(w > 0 ? w : 1));
    int p = 0;
    for (int col = 0; col < R->n; ++col) M->cols[p++] = T->col_off[j] + col;
    for (int c = 0; c < nch; ++c)
        for (int q = 0; q < msgs[ch[c]].width; ++q) M->cols[p++] = msgs[ch[c]].cols[q];
    for (int a = 1; a < w; ++a) {
        int v = M->cols[a], b = a - 1;
        while (b >= 0 && M->cols[b] > v) { M->cols[b + 1] = M->cols[b]; --b; }
        M->cols[b + 1] = v;
    }
    /* message key groups: rows of R grouped by the attributes shared with `from` */
    if (rindex_build(&M->ix, R, M->kpos, M->nk) != 0) return -1;
    M->grp_of_row = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->m > 0 ? R->m : 1));
    M->key_rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->m > 0 ? R->m : 1));
    int64_t g = -1;
    for (int64_t q = 0; q < R->m; ++q) {
        int64_t row = M->ix.order[q];
        if (q == 0 || !key_equal_rows(R, M->kpos, M->nk, row, M->ix.order[q - 1])) {
            ++g;
            M->key_rows[g] = row;
        }
        M->grp_of_row[row] = g;
    }
    M->nkeys = g + 1;
    M->cnt = (__float128 *)calloc((size_t)(M->nkeys > 0 ? M->nkeys : 1), sizeof(__float128));
    M->sum = (__float128 *)calloc((size_t)(M->nkeys > 0 ? M->nkeys : 1) * (size_t)(w > 0 ? w : 1), sizeof(__float128));
    int *own_at = (int *)malloc(sizeof(int) * (size_t)(R->n > 0 ? R->n : 1));
    for (int col = 0; col < R->n; ++col)
        for (int a = 0; a < w; ++a) if (M->cols[a] == T->col_off[j] + col) own_at[col] = a;
    int *ch_at[64];
    int ch_ppos[64][64];
    for (int c = 0; c < nch; ++c) {
        message *C = &msgs[ch[c]];
        ch_at[c] = (int *)malloc(sizeof(int) * (size_t)(C->width > 0 ? C->width : 1));
        for (int q = 0; q < C->width; ++q)
            for (int a = 0; a < w; ++a) if (M->cols[a] == C->cols[q]) ch_at[c][q] = a;
        for (int i = 0; i < C->nk; ++i) ch_ppos[c][i] = attr_pos(R, T->rels[ch[c]].attrs[C->kpos[i]]);
    }
    /* every row of one full-key group of R joins the same child groups */
    full_groups F;
    if (full_groups_build(&F, R) != 0) return -1;
    long double *ysum = (long double *)malloc(sizeof(long double) * (size_t)(R->n > 0 ? R->n : 1));
    for (int64_t fg = 0; fg < F.ngroups; ++fg) {
        int64_t rep = F.ix.order[F.gstart[fg]];
        int64_t cnt_rows = F.gstart[fg + 1] - F.gstart[fg];
        __float128 wt = 1;
        int64_t cg[64];
        int ok = 1;
        for (int c = 0; c < nch; ++c) {
            cg[c] = msg_lookup(&msgs[ch[c]], R, ch_ppos[c], rep);
            if (cg[c] < 0) { ok = 0; break; }
            wt *= msgs[ch[c]].cnt[cg[c]];
        }
        if (!ok) continue;
        for (int col = 0; col < R->n; ++col) ysum[col] = 0.0L;
        for (int64_t q = F.gstart[fg]; q < F.gstart[fg + 1]; ++q) {
            int64_t t = F.ix.order[q];
            for (int col = 0; col < R->n; ++col) ysum[col] += (long double)R->vals[(int64_t)col * R->m + t];
        }
        int64_t g2 = M->grp_of_row[rep];
        M->cnt[g2] += wt * (__float128)cnt_rows;
        __float128 *S = M->sum + g2 * w;
        for (int col = 0; col < R->n; ++col) S[own_at[col]] += (__float128)ysum[col] * wt;
        for (int c = 0; c < nch; ++c) {
            message *C = &msgs[ch[c]];
            __float128 other = (__float128)cnt_rows;
            for (int c2 = 0; c2 < nch; ++c2)
                if (c2 != c) other *= msgs[ch[c2]].cnt[cg[c2]];
            for (int q = 0; q < C->width; ++q) S[ch_at[c][q]] += C->sum[cg[c] * C->width + q] * other;
        }
    }
    free(ysum);
    full_groups_free(&F);
    free(own_at);
    for (int c = 0; c < nch; ++c) free(ch_at[c]);
    return 0;
}

static void free_message(message *M) {
    free(M->key_rows); free(M->cols); free(M->cnt); free(M->sum);
    free(M->ix.order); free(M->grp_of_row);
    memset(M, 0, sizeof *M);
}

/* Full A^T A (n x n, column-major) in __float128, plus the join size.
 * Anchor k contributes the diagonal block (k, k) and the blocks (k, l) for
 * every other relation l; the latter are written at rows of k, columns of l. */
static int factorized_gram(int r, const orel *rels, __float128 *G, __float128 *join_rows) {
    tree_info T;
    T.r = r;
    T.rels = rels;
    T.col_off = (int *)calloc((size_t)r + 1, sizeof(int));
    for (int i = 0; i < r; ++i) T.col_off[i + 1] = T.col_off[i] + rels[i].n;
    int n = T.col_off[r];
    T.adj = (int **)malloc(sizeof(int *) * (size_t)r);
    T.deg = (int *)calloc((size_t)r, sizeof(int));
    for (int i = 0; i < r; ++i) T.adj[i] = (int *)malloc(sizeof(int) * (size_t)r);
    for (int i = 0; i < r; ++i)
        if (rels[i].parent >= 0) {
            int p = rels[i].parent;
            T.adj[i][T.deg[i]++] = p;
            T.adj[p][T.deg[p]++] = i;
        }
    __float128 *Gw = (__float128 *)calloc((size_t)n * (size_t)n, sizeof(__float128));
    message *msgs = (message *)calloc((size_t)r, sizeof(message));
    int status = 0;
    for (int k = 0; k < r && status == 0; ++k) {
        const orel *K = &rels[k];
        for (int d = 0; d < T.deg[k]; ++d)
            if (build_message(&T, msgs, T.adj[k][d], k) != 0) { status = -1; break; }
        if (status) break;
        int nch = T.deg[k];
        int ch_ppos[64][64];
        for (int c = 0; c < nch; ++c) {
            message *C = &msgs[T.adj[k][c]];
            for (int i = 0; i < C->nk; ++i) ch_ppos[c][i] = attr_pos(K, rels[T.adj[k][c]].attrs[C->kpos[i]]);
        }
        int nk = K->n;
        long double *yy = (long double *)malloc(sizeof(long double) * (size_t)(nk > 0 ? nk * nk : 1));
        long double *ys = (long double *)malloc(sizeof(long double) * (size_t)(nk > 0 ? nk : 1));
        __float128 total = 0;
        full_groups F;
        if (full_groups_build(&F, K) != 0) { status = -1; break; }
        for (int64_t fg = 0; fg < F.ngroups; ++fg) {
            int64_t rep = F.ix.order[F.gstart[fg]];
            int64_t cnt_rows = F.gstart[fg + 1] - F.gstart[fg];
            __float128 wt = 1;
            int64_t cg[64];
            int ok = 1;
            for (int c = 0; c < nch; ++c) {
                cg[c] = msg_lookup(&msgs[T.adj[k][c]], K, ch_ppos[c], rep);
                if (cg[c] < 0) { ok = 0; break; }
                wt *= msgs[T.adj[k][c]].cnt[cg[c]];
            }
            if (!ok) continue;
            total += wt * (__float128)cnt_rows;
            for (int a = 0; a < nk * nk; ++a) yy[a] = 0.0L;
            for (int a = 0; a < nk; ++a) ys[a] = 0.0L;
            for (int64_t q = F.gstart[fg]; q < F.gstart[fg + 1]; ++q) {
                int64_t t = F.ix.order[q];
                for (int a = 0; a < nk; ++a) {
                    long double ya = K->vals[(int64_t)a * K->m + t];
                    ys[a] += ya;
                    for (int b = 0; b <= a; ++b) yy[a * nk + b] += ya * (long double)K->vals[(int64_t)b * K->m + t];
                }
            }
            for (int a = 0; a < nk; ++a)
                for (int b = 0; b <= a; ++b)
                    Gw[(int64_t)(T.col_off[k] + b) * n + (T.col_off[k] + a)] += (__float128)yy[a * nk + b] * wt;
            for (int c = 0; c < nch; ++c) {
                message *C = &msgs[T.adj[k][c]];
                __float128 other = 1;
                for (int c2 = 0; c2 < nch; ++c2)
                    if (c2 != c) other *= msgs[T.adj[k][c2]].cnt[cg[c2]];
                for (int q = 0; q < C->width; ++q) {
                    __float128 s = C->sum[cg[c] * C->width + q] * other;
                    int gc = C->cols[q];
                    for (int a = 0; a < nk; ++a) Gw[(int64_t)gc * n + (T.col_off[k] + a)] += (__float128)ys[a] * s;
                }
            }
        }
        full_groups_free(&F);
        *join_rows = total;
        free(yy);
        free(ys);
        for (int i = 0; i < r; ++i) free_message(&msgs[i]);
    }
    /* Gw holds, for each anchor k: the lower triangle of block (k,k) and the
     * full blocks at rows of k / columns of other relations.  Assemble the
     * symmetric matrix: diagonal blocks from their lower triangle; for a pair
     * of relations the block was produced once from each side; the two agree
     * in exact arithmetic, take their mean. */
    for (int k = 0; k < r; ++k)
        for (int a = T.col_off[k]; a < T.col_off[k + 1]; ++a)
            for (int b = T.col_off[k]; b <= a; ++b) {
                __float128 v = Gw[(int64_t)b * n + a];
                G[(int64_t)b * n + a] = v;
                G[(int64_t)a * n + b] = v;
            }
    for (int k = 0; k < r; ++k)
        for (int l = k + 1; l < r; ++l)
            for (int a = T.col_off[k]; a < T.col_off[k + 1]; ++a)
                for (int b = T.col_off[l]; b < T.col_off[l + 1]; ++b) {
                    __float128 v = (Gw[(int64_t)b * n + a] + Gw[(int64_t)a * n + b]) / 2;
                    G[(int64_t)b * n + a] = v;
                    G[(int64_t)a * n + b] = v;
                }
    free(Gw);
    free(msgs);
    for (int i = 0; i < r; ++i) free(T.adj[i]);
    free(T.adj); free(T.deg); free(T.col_off);
    return status;
}

/* A^T A by distributivity (hi + lo doubles) and the exact join size. */
int or_factorized_gram(int r, const orel *rels, double *Ghi, double *Glo, double *join_rows) {
    int n = 0;
    for (int i = 0; i < r; ++i) n += rels[i].n;
    __float128 *G = (__float128 *)malloc(sizeof(__float128) * (size_t)n * (size_t)n);
    __float128 jr = 0;
    int st = factorized_gram(r, rels, G, &jr);
    for (int64_t i = 0; i < (int64_t)n * n; ++i) {
        Ghi[i] = (double)G[i];
        Glo[i] = (double)(G[i] - (__float128)Ghi[i]);
    }
    *join_rows = (double)jr;
    free(G);
    return st;
}

/* R = chol(A^T A), upper triangular with positive diagonal, computed in
 * __float128 from the factorised Gram matrix; rounded to double.  Returns 0,
 * or 1 if the Gram matrix is not positive definite (rank-deficient join). */
int or_factorized_r(int r, const orel *rels, double *Rout, double *join_rows) {
    int n = 0;
    for (int i = 0; i < r; ++i) n += rels[i].n;
    __float128 *G = (__float128 *)malloc(sizeof(__float128) * (size_t)n * (size_t)n);
    __float128 jr = 0;
    int st = factorized_gram(r, rels, G, &jr);
    *join_rows = (double)jr;
    if (st != 0) { free(G); return -1; }
    __float128 *R = (__float128 *)calloc((size_t)n * (size_t)n, sizeof(__float128));
    int pd = 1;
    for (int j = 0; j < n && pd; ++j) {
        __float128 d = G[(int64_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= R[(int64_t)j * n + k] * R[(int64_t)j * n + k];
        if (!(d > 0)) { pd = 0; break; }
        __float128 rjj = sqrtq(d);
        R[(int64_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            __float128 s = G[(int64_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= R[(int64_t)j * n + k] * R[(int64_t)i * n + k];
            R[(int64_t)i * n + j] = s / rjj;
        }
    }
    for (int64_t i = 0; i < (int64_t)n * n; ++i) Rout[i] = (double)R[i];
    free(R);
    free(G);
    return pd ? 0 : 1;
}
