// From R to Q, SVD and PCA (section "From R to Q, SVD and PCA").
//
//  * figaro_svd_r: the SVD of the n x n upper-triangular R, whose singular
//    values and right singular vectors are those of the join matrix A.
//    One-sided Jacobi (Hestenes): columns of a working copy of R are rotated
//    in pairs until every pair is orthogonal to working precision (pairs in
//    round-robin order, disjoint pairs of a step in parallel, one workgroup);
//    then sigma_i = ||a_i||, U_R = a_i / sigma_i, V = the product of the
//    rotations, sorted by decreasing sigma.  The paper uses a
//    divide-and-conquer SVD; Jacobi reaches the same factors to rounding and
//    is accurate in the small singular values too.
//  * figaro_r_inverse: R^-1 by back substitution, one column per thread.
//  * figaro_join_multiply: rows of A M for the join matrix A, which is never
//    materialised.  As in the paper, every tuple s of every relation first
//    takes the dot products of its data values with the rows of M at its
//    columns (D_i = S_i M[cols_i, :]); a row of A M is then the sum of the
//    D rows of the tuples that make up that join row.  The join rows are
//    enumerated in a fixed order from the plan's exact counts: a row index
//    is split, from the root down, into a key group (by the prefix sums of
//    Theta), the group's tuple and one row index per child subtree (mixed
//    radix over the children's Phi-down), so every thread rebuilds its row
//    independently.  Q = A R^-1, U = A V Sigma^-1 and the PCA projection
//    A V[:, 1:k] are such products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace figaro {
extern thread_local std::string g_thread_error;
}  // namespace figaro

using namespace figaro;

namespace {

figaro_status fail(figaro_plan_s *p, figaro_status st, const std::string &msg) {
    if (p) return set_error(p, st, msg);
    g_thread_error = msg;
    return st;
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of an n x n matrix (n <= 128), one workgroup
// ---------------------------------------------------------------------------

constexpr int kSvdThreads = 1024;
constexpr int kSvdWaves = kSvdThreads / 64;
constexpr int kMaxSweeps = 60;

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// work: A (n x n, column-major), then V (n x n); lane l holds rows l and l + 64
__global__ __launch_bounds__(kSvdThreads) void k_jacobi(int n, const double *R, double *work, int *sweeps_out) {
    __shared__ int rotated;
    double *A = work, *V = work + (size_t)n * n;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
        A[i] = R[i];
        V[i] = (i % n == i / n) ? 1.0 : 0.0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int np = n + (n & 1);   // players in the round-robin (a dummy when n is odd)
    const double tol = 2.220446049250313e-16 * sqrt((double)n);
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int t = 0; t < np - 1; ++t) {
            for (int k = wave; k < np / 2; k += kSvdWaves) {
                // pair k of round t (circle method: player 0 fixed)
                const int i = k == 0 ? 0 : ((k + t) % (np - 1)) + 1;
                const int j = ((np - 1 - k + t) % (np - 1)) + 1;
                if (i >= n || j >= n) continue;
                const int a = min(i, j), b = max(i, j);
                const double x0 = lane < n ? A[(size_t)a * n + lane] : 0.0;
                const double y0 = lane < n ? A[(size_t)b * n + lane] : 0.0;
                const double x1 = lane + 64 < n ? A[(size_t)a * n + lane + 64] : 0.0;
                const double y1 = lane + 64 < n ? A[(size_t)b * n + lane + 64] : 0.0;
                const double al = wsum(fma(x0, x0, x1 * x1));
                const double be = wsum(fma(y0, y0, y1 * y1));
                const double ga = wsum(fma(x0, y0, x1 * y1));
                // rotate unless the pair is orthogonal to working precision
                // (the butterfly sums are the same bits in every lane, so the
                // whole wave takes the same branch)
                if (ga == 0.0 || fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
                const double c = 1.0 / sqrt(fma(tt, tt, 1.0)), s = c * tt;
                if (lane < n) {
                    A[(size_t)a * n + lane] = c * x0 - s * y0;
                    A[(size_t)b * n + lane] = s * x0 + c * y0;
                }
                if (lane + 64 < n) {
                    A[(size_t)a * n + lane + 64] = c * x1 - s * y1;
                    A[(size_t)b * n + lane + 64] = s * x1 + c * y1;
                }
                for (int r = lane; r < n; r += 64) {
                    const double va = V[(size_t)a * n + r], vb = V[(size_t)b * n + r];
                    V[(size_t)a * n + r] = c * va - s * vb;
                    V[(size_t)b * n + r] = s * va + c * vb;
                }
                if (lane == 0) rotated = 1;
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    if (threadIdx.x == 0 && sweeps_out) *sweeps_out = sweep;
}

// sigma, U = A / sigma, V, columns in decreasing order of sigma (ties keep
// their order); one thread per column
__global__ void k_svd_sort(int n, const double *work, double *sigma, double *U, double *V) {
    __shared__ double nrm[128];
    const double *A = work, *Vw = work + (size_t)n * n;
    const int j = threadIdx.x;
    if (j < n) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s = fma(A[(size_t)j * n + r], A[(size_t)j * n + r], s);
        nrm[j] = sqrt(s);
    }
    __syncthreads();
    if (j >= n) return;
    const double sj = nrm[j];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += (nrm[q] > sj || (nrm[q] == sj && q < j)) ? 1 : 0;
    sigma[rank] = sj;
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    for (int r = 0; r < n; ++r) {
        if (U) U[(size_t)rank * n + r] = A[(size_t)j * n + r] * inv;
        V[(size_t)rank * n + r] = Vw[(size_t)j * n + r];
    }
}

__global__ void k_tri_inverse(int n, const double *R, double *X) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int i = n - 1; i >= 0; --i) {
        double v = (i == j) ? 1.0 : 0.0;
        if (i < j || i == j) {
            for (int k = i + 1; k <= j; ++k) v = fma(-R[(size_t)k * n + i], X[(size_t)j * n + k], v);
            v /= R[(size_t)i * n + i];
        } else {
            v = 0.0;
        }
        X[(size_t)j * n + i] = v;
    }
}

// ---------------------------------------------------------------------------
// Join-row enumeration
// ---------------------------------------------------------------------------

constexpr int kEnumRels = 16;

struct EnumRel {
    const int64_t *seg_off;     // [G+1]
    const int64_t *theta_excl;  // [G+1]
    const int64_t *par_off;     // [P+1] (non-root)
    const int64_t *phi_down;    // [P]   (non-root)
    const int64_t *perm;        // plan row -> caller row
    const int32_t *cidx_from_parent;   // parent key group -> this relation's parent group
    const double *D;            // [k][m] dot products of this relation's rows with M
    int64_t m;
    int64_t G;
};

struct EnumArgs {
    EnumRel rel[kEnumRels];
    int8_t kids[kEnumRels][kEnumRels];
    int8_t nkids[kEnumRels];
    int8_t pre[kEnumRels];      // pre-order of the join tree
    int32_t r;
    int32_t k;
    const double *col_scale;    // [k] or null
    int64_t row0, nrows;
    double *out;
    int64_t ld_out;
    int64_t *ids;               // [r][ld_ids] or null
    int64_t ld_ids;
};

// D_i[p, c] = sum over the relation's columns t of S_i[p, t] M[col0 + t, c],
// one thread per (p, c)
__global__ void k_rel_dots(const double *S, int64_t ld, int64_t m, int ncols, int col0, const double *M, int64_t ldm,
                           double *D) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= m) return;
    double acc = 0.0;
    for (int t = 0; t < ncols; ++t) acc = fma(S[(int64_t)t * ld + p], M[(int64_t)c * ldm + col0 + t], acc);
    D[(int64_t)c * m + p] = acc;
}

// the last index in [lo, hi) whose prefix value is <= v
__device__ __forceinline__ int64_t floor_search(const int64_t *pre, int64_t lo, int64_t hi, int64_t v) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pre[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_enumerate(EnumArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nrows) return;
    const int64_t row = a.row0 + t;
    int64_t g[kEnumRels], rem[kEnumRels], prow[kEnumRels];
    const int root = a.pre[0];
    g[root] = floor_search(a.rel[root].theta_excl, 0, a.rel[root].G, row);
    rem[root] = row - a.rel[root].theta_excl[g[root]];
    for (int q = 0; q < a.r; ++q) {
        const int v = a.pre[q];
        const EnumRel &R = a.rel[v];
        const int64_t gv = g[v];
        // rows of the children's subtrees for this key group, first child most significant
        int64_t prodc = 1;
        int64_t pg[kEnumRels];
        for (int c = 0; c < a.nkids[v]; ++c) {
            const int ch = a.kids[v][c];
            pg[c] = a.rel[ch].cidx_from_parent[gv];
            prodc *= a.rel[ch].phi_down[pg[c]];
        }
        int64_t r = rem[v] % prodc;
        prow[v] = R.seg_off[gv] + rem[v] / prodc;
        for (int c = a.nkids[v] - 1; c >= 0; --c) {
            const int ch = a.kids[v][c];
            const EnumRel &C = a.rel[ch];
            const int64_t pd = C.phi_down[pg[c]];
            const int64_t rc = r % pd;
            r /= pd;
            const int64_t lo = C.par_off[pg[c]], hi = C.par_off[pg[c] + 1];
            const int64_t want = C.theta_excl[lo] + rc;
            g[ch] = floor_search(C.theta_excl, lo, hi, want);
            rem[ch] = want - C.theta_excl[g[ch]];
        }
    }
    for (int c = 0; c < a.k; ++c) {
        double acc = 0.0;
        for (int q = 0; q < a.r; ++q) {
            const int v = a.pre[q];
            acc += a.rel[v].D[(int64_t)c * a.rel[v].m + prow[v]];
        }
        a.out[(int64_t)c * a.ld_out + t] = a.col_scale ? acc * a.col_scale[c] : acc;
    }
    if (a.ids)
        for (int v = 0; v < a.r; ++v) a.ids[(int64_t)v * a.ld_ids + t] = a.rel[v].perm[prow[v]];
}

}  // namespace

extern "C" {

figaro_status figaro_svd_r(int32_t n, const double *R, double *sigma, double *U, double *V, double *work,
                           hipStream_t stream) {
    if (n < 1 || n > kMaxCols) return fail(nullptr, FIGARO_EUNSUPPORTED, "n must be between 1 and 128");
    if (!R || !sigma || !V || !work) return fail(nullptr, FIGARO_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kSvdThreads), 0, stream, n, R, work, (int *)nullptr);
    hipLaunchKernelGGL(k_svd_sort, dim3(1), dim3(128), 0, stream, n, (const double *)work, sigma, U, V);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FIGARO_OK : fail(nullptr, FIGARO_EHIP, hipGetErrorString(e));
}

figaro_status figaro_r_inverse(int32_t n, const double *R, double *Rinv, hipStream_t stream) {
    if (n < 1 || n > kMaxCols) return fail(nullptr, FIGARO_EUNSUPPORTED, "n must be between 1 and 128");
    if (!R || !Rinv) return fail(nullptr, FIGARO_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_tri_inverse, dim3(1), dim3(128), 0, stream, n, R, Rinv);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FIGARO_OK : fail(nullptr, FIGARO_EHIP, hipGetErrorString(e));
}

int64_t figaro_join_multiply_workspace_bytes(figaro_plan_t p, int32_t k) {
    if (!p || p->analyze_only || k < 1) return -1;
    int64_t rows = 0;
    for (const auto &R : p->rel) rows += R.m;
    return 8 * rows * (int64_t)k;
}

figaro_status figaro_join_multiply(figaro_plan_t p, const double *const *values, const int64_t *ld, const double *M,
                                   int64_t ldm, int32_t k, const double *col_scale, int64_t row0, int64_t nrows,
                                   double *out, int64_t ld_out, int64_t *tuple_ids, int64_t ld_ids, void *work,
                                   int64_t work_bytes, hipStream_t stream) {
    if (!p) return fail(nullptr, FIGARO_EINVAL, "plan is NULL");
    if (p->analyze_only) return fail(p, FIGARO_EINVAL, "the plan was built with analyze_only");
    if (p->r > kEnumRels) return fail(p, FIGARO_EUNSUPPORTED, "more than 16 relations");
    if (!values || !ld || !M || !out || k < 1 || k > kMaxCols || ldm < p->n || nrows < 0 || row0 < 0 ||
        ld_out < std::max<int64_t>(nrows, 1) || (tuple_ids && ld_ids < std::max<int64_t>(nrows, 1)))
        return fail(p, FIGARO_EINVAL, "bad argument");
    if ((double)(row0 + nrows) > p->join_rows) return fail(p, FIGARO_EINVAL, "rows beyond the join");
    if (!work || work_bytes < figaro_join_multiply_workspace_bytes(p, k))
        return fail(p, FIGARO_EINVAL, "workspace smaller than figaro_join_multiply_workspace_bytes()");
    for (int i = 0; i < p->r; ++i)
        if (!values[i] || ld[i] < p->rel[i].m) return fail(p, FIGARO_EINVAL, "values or ld of a relation");
    if (nrows == 0) return FIGARO_OK;
    EnumArgs a{};
    a.r = p->r;
    a.k = k;
    a.col_scale = col_scale;
    a.row0 = row0;
    a.nrows = nrows;
    a.out = out;
    a.ld_out = ld_out;
    a.ids = tuple_ids;
    a.ld_ids = ld_ids;
    double *D = static_cast<double *>(work);
    for (int i = 0; i < p->r; ++i) {
        const RelPlan &R = p->rel[i];
        EnumRel &e = a.rel[i];
        e.seg_off = R.d_seg_off;
        e.theta_excl = R.d_theta_excl;
        e.par_off = R.d_par_off;
        e.phi_down = R.d_phi_down;
        e.perm = R.d_perm;
        e.D = D;
        e.m = R.m;
        e.G = R.G;
        a.nkids[i] = (int8_t)R.children.size();
        for (size_t c = 0; c < R.children.size(); ++c) {
            a.kids[i][c] = (int8_t)R.children[c];
            a.rel[R.children[c]].cidx_from_parent = R.d_cidx[c];
        }
        const int bs = 256;
        if (R.m > 0)
            hipLaunchKernelGGL(k_rel_dots, dim3((unsigned)((R.m + bs - 1) / bs), (unsigned)k), dim3(bs), 0, stream,
                               values[i], ld[i], R.m, R.ncols, R.col0, M, ldm, D);
        D += R.m * (int64_t)k;
    }
    std::vector<int32_t> pre;
    std::vector<int32_t> stack{p->root};
    while (!stack.empty()) {
        const int v = stack.back();
        stack.pop_back();
        pre.push_back(v);
        for (auto it = p->rel[v].children.rbegin(); it != p->rel[v].children.rend(); ++it) stack.push_back(*it);
    }
    for (int q = 0; q < p->r; ++q) a.pre[q] = (int8_t)pre[q];
    const int bs = 256;
    hipLaunchKernelGGL(k_enumerate, dim3((unsigned)((nrows + bs - 1) / bs)), dim3(bs), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FIGARO_OK : fail(p, FIGARO_EHIP, hipGetErrorString(e));
}

}  // extern "C"
