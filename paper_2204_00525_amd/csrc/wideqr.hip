// Blocked Householder QR for the wide regime: plans with more columns than
// the register-tile kernels hold.  Post-processing of the paper ("Post-
// processing" section: the R0 that the head/tail phase leaves is reduced by
// a QR decomposition; the wide synthetic experiments run it through a
// blocked LAPACK-style QR).  Only R is kept.
//
// The matrix A (h x n, column-major, leading dimension lda) is reduced in
// panels of kNb columns, right-looking:
//   * panel: one Householder reflector per column, H = I - tau v v^T with
//     v = [1; x / (alpha - beta)], beta = -sign(alpha) ||[alpha; x]||,
//     tau = (beta - alpha) / beta (tau = 0 when x = 0);
//   * compact WY form of the panel's reflectors, Q = I - V T V^T (T upper
//     triangular, built column by column from V^T V and tau);
//   * trailing columns C := Q^T C = C - V (T^T (V^T C)), the two products
//     with V as plain rocBLAS GEMMs.
//
// Two row structures:
//   general (tp = 0): reflector j acts on rows j .. h-1;
//   triangular-pentagonal (tp = 1): rows 0 .. n-1 already form an upper
//     triangular block, so reflector j acts on row j and rows n .. h-1 only
//     (the block's other rows are zero in column j and stay so).
// In both, the rows a panel's reflectors touch are numbered "virtual rows":
// t < kb is row k + t (the panel's own rows), t >= kb is row s0 + t - kb
// (s0 = k + kb in general form, n in triangular-pentagonal form), so that V
// is one contiguous (kb + h - s0) x kb block.
//
// A panel column needs one reduction over all its rows (the norm of x and
// the dot products of x with the panel's later columns, from which both the
// reflector and its effect on those columns follow).  Short panels run in
// one workgroup; tall ones take one launch per column over many workgroups,
// each launch first finishing the previous column's reflector from the
// partial sums every workgroup left, applying it to its rows, then leaving
// its partial sums for the next column.  Nothing spins on another
// workgroup.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>

#include "internal.hpp"

namespace figaro {
namespace {

constexpr int kNb = 32;             // panel width
constexpr int kPassThreads = 256;   // threads of a panel workgroup (4 waves)
constexpr int kSmallRows = 1024;    // virtual rows up to which one workgroup factors a panel
constexpr int kMaxPassWgs = 128;    // workgroups of a per-column pass
constexpr int kPartStride = kNb + 1;

struct PanelArgs {
    double *A;
    int64_t lda;
    int64_t k;      // first column (and first row) of the panel
    int32_t kb;     // panel width
    int64_t s0;     // first row of the tail range
    int32_t tp;     // triangular-pentagonal form
    int64_t nv;     // virtual rows
    double *V;      // [kb][ldv]
    int64_t ldv;
    double *tau;    // [kb]
    double *part;   // [2][wgs][kPartStride]: per-workgroup partial sums of one column
    double *head;   // [2][kPartStride]: the reflector's own row, columns 0..kb-1
    int32_t wgs;
    int64_t rows_per_wg;
};

// The scalars of one reflector as every workgroup derives them.
struct Refl {
    double tau, scale, beta;
    double w[kNb];   // w_c = v^T a_c for the panel's later columns c
};

__device__ __forceinline__ int64_t real_row(const PanelArgs &a, int64_t t) {
    return t < a.kb ? a.k + t : a.s0 + (t - a.kb);
}

// Whether virtual row t lies in the tail of reflector q (below its own row
// and, in triangular-pentagonal form, outside the triangular block).
__device__ __forceinline__ bool in_tail(const PanelArgs &a, int64_t t, int q) {
    return t > q && (!a.tp || t >= a.kb);
}

// Reflector q from its row (head[c], c >= q) and the reduced sums over its
// tail: tot[q] = ||x||^2, tot[c] = x^T a_c for c > q.  Run by thread 0.
__device__ void make_reflector(const PanelArgs &a, int q, const double *head, const double *tot, Refl &r) {
    const double alpha = head[q], sig2 = tot[q];
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (sig2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    r.tau = tau;
    r.scale = scale;
    r.beta = beta;
    for (int c = q + 1; c < a.kb; ++c) r.w[c] = head[c] + scale * tot[c];
}

// One column step on virtual rows [t0, t1) of a workgroup: apply reflector
// q = p - 1 (p > 0) with the scalars in r, write column q of V, then add
// this workgroup's sums for reflector p (p < kb) into acc and keep row p's
// values in head_out.
__device__ __forceinline__ void column_step(const PanelArgs &a, int p, int64_t t0, int64_t t1, const Refl &r,
                                            double (&acc)[kNb], double *head_out) {
    const int q = p - 1;
    const int c_lo = p > 0 ? q : p;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kPassThreads) {
        double *base = a.A + real_row(a, t) + a.k * a.lda;
        double x[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c)
            if (c >= c_lo && c < a.kb) x[c] = base[c * a.lda];
        if (p > 0) {
            double v;
            bool changed = true;
            if (t == q) {
                v = 1.0;
                x[q] = r.beta;
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c > q && c < a.kb) x[c] -= r.tau * r.w[c];
            } else if (in_tail(a, t, q)) {
                v = x[q] * r.scale;
                x[q] = v;
                const double tv = r.tau * v;
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c > q && c < a.kb) x[c] -= tv * r.w[c];
            } else {
                v = 0.0;
                changed = false;
            }
            a.V[(int64_t)q * a.ldv + t] = v;
            if (changed) {
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c >= q && c < a.kb) base[c * a.lda] = x[c];
            }
        }
        if (p < a.kb) {
            if (t == p) {
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c >= p && c < a.kb) head_out[c] = x[c];
            } else if (in_tail(a, t, p)) {
                const double xp = x[p];
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c >= p && c < a.kb) acc[c] += xp * x[c];
            }
        }
    }
}

// Sum acc[c] (c in [p, kb)) over the workgroup into out[c] (LDS scratch red).
__device__ void block_sum(const PanelArgs &a, int p, double (&acc)[kNb], double (*red)[kPassThreads / 64],
                          double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kNb; ++c) {
        if (c < p || c >= a.kb) continue;
        double v = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[c][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x >= p && threadIdx.x < a.kb) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kPassThreads / 64; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

// Whole panel in one workgroup (nv <= kSmallRows).
__global__ __launch_bounds__(kPassThreads) void k_panel_one(PanelArgs a) {
    __shared__ double red[kNb][kPassThreads / 64];
    __shared__ double tot[kNb], head[kNb];
    __shared__ Refl r;
    for (int p = 0; p <= a.kb; ++p) {
        if (p > 0) {
            if (threadIdx.x == 0) {
                make_reflector(a, p - 1, head, tot, r);
                a.tau[p - 1] = r.tau;
            }
            __syncthreads();
        }
        double acc[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) acc[c] = 0.0;
        __shared__ double head_next[kNb];
        column_step(a, p, 0, a.nv, r, acc, head_next);
        if (p < a.kb) {
            block_sum(a, p, acc, red, tot);
            __syncthreads();
            if (threadIdx.x < kNb) head[threadIdx.x] = head_next[threadIdx.x];
            __syncthreads();
        }
    }
}

// One column step of a tall panel; workgroup b owns virtual rows
// [b * rows_per_wg, (b + 1) * rows_per_wg).  Partial sums and the
// reflector's row alternate between two buffers by column parity, so a
// launch never overwrites what a workgroup of the same launch still reads.
__global__ __launch_bounds__(kPassThreads) void k_panel_pass(PanelArgs a, int p) {
    __shared__ double red[kNb][kPassThreads / 64];
    __shared__ double tot[kNb], hd[kNb];
    __shared__ Refl r;
    if (p > 0) {
        const int q = p - 1;
        const double *prt = a.part + (int64_t)(q & 1) * a.wgs * kPartStride;
        const double *hq = a.head + (q & 1) * kPartStride;
        const int c = threadIdx.x;
        if (c >= q && c < a.kb) {
            double s = 0.0;
            for (int b = 0; b < a.wgs; ++b) s += prt[(int64_t)b * kPartStride + c];
            tot[c] = s;
            hd[c] = hq[c];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            make_reflector(a, q, hd, tot, r);
            if (blockIdx.x == 0) a.tau[q] = r.tau;
        }
        __syncthreads();
    }
    const int64_t t0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t t1 = std::min<int64_t>(a.nv, t0 + a.rows_per_wg);
    double acc[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) acc[c] = 0.0;
    column_step(a, p, t0, t1, r, acc, a.head + (p & 1) * kPartStride);
    if (p < a.kb) {
        __syncthreads();
        block_sum(a, p, acc, red, a.part + ((int64_t)(p & 1) * a.wgs + blockIdx.x) * kPartStride);
    }
}

// T of the compact WY form from G = V^T V and tau (one wave):
//   T[p][p] = tau_p,  T[0:p][p] = -tau_p T[0:p][0:p] G[0:p][p].
__global__ __launch_bounds__(64) void k_wy_t(const double *G, const double *tau, int kb, double *T) {
    __shared__ double sT[kNb][kNb + 1];
    const int i = threadIdx.x;
    if (i < kNb)
        for (int j = 0; j < kNb; ++j) sT[i][j] = 0.0;
    __syncthreads();
    for (int p = 0; p < kb; ++p) {
        const double tp = tau[p];
        double y = 0.0;
        if (i < p)
            for (int j = i; j < p; ++j) y += sT[i][j] * G[p * kNb + j];
        __syncthreads();
        if (i < p) sT[i][p] = -tp * y;
        if (i == p) sT[p][p] = tp;
        __syncthreads();
    }
    if (i < kNb)
        for (int j = 0; j < kNb; ++j) T[j * kNb + i] = sT[i][j];
}

// W := T^T W for the kb x nc block W (leading dimension kNb), one column per
// thread.
__global__ __launch_bounds__(256) void k_wy_tw(const double *T, int kb, double *W, int64_t nc) {
    __shared__ double sT[kNb * kNb];
    for (int i = threadIdx.x; i < kNb * kNb; i += blockDim.x) sT[i] = T[i];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double w[kNb], o[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) w[q] = q < kb ? W[c * kNb + q] : 0.0;
#pragma unroll
    for (int p = 0; p < kNb; ++p) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q <= p; ++q) s += sT[p * kNb + q] * w[q];
        o[p] = s;
    }
#pragma unroll
    for (int p = 0; p < kNb; ++p)
        if (p < kb) W[c * kNb + p] = o[p];
}

// Upper-triangular part of the first min(rows, cols) rows of src (cols
// columns) into dst at (row0 + j, col0 + c); zeros below the diagonal.
__global__ void k_copy_upper(const double *src, int64_t ld_src, int64_t rows, int32_t cols, double *dst,
                             int64_t ld_dst, int64_t row0, int64_t col0) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= cols) return;
    const double v = (j <= c && j < rows) ? src[(int64_t)c * ld_src + j] : 0.0;
    dst[(col0 + c) * ld_dst + row0 + j] = v;
}

// R (n x n, leading dimension n) from the upper triangle of A's first n
// rows, every row scaled by the sign of its diagonal entry (rows beyond
// `rows` are zero).
__global__ void k_final_r(const double *A, int64_t lda, int64_t rows, int32_t n, double *R) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n) return;
    double v = 0.0;
    if (j <= c && j < rows) {
        const double d = A[j * lda + j];
        v = (d < 0.0 ? -1.0 : 1.0) * A[(int64_t)c * lda + j];
    }
    R[(int64_t)c * n + j] = v;
}

bool gemm(rocblas_handle h, bool ta, int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
          const double *B, int64_t ldb, double beta, double *C, int64_t ldc) {
    if (m <= 0 || n <= 0) return true;
    if (k <= 0 && beta == 1.0) return true;
    return rocblas_dgemm(h, ta ? rocblas_operation_transpose : rocblas_operation_none, rocblas_operation_none,
                         (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &alpha, A, (rocblas_int)lda, B,
                         (rocblas_int)ldb, &beta, C, (rocblas_int)ldc) == rocblas_status_success;
}

}  // namespace

int64_t wide_qr_panel_rows(int64_t h, int32_t n, bool tp) {
    return tp ? kNb + std::max<int64_t>(0, h - n) : std::max<int64_t>(h, kNb);
}

int64_t wide_qr_workspace_doubles(int64_t max_nv, int32_t n) {
    return (int64_t)kNb * max_nv          // V
           + n                            // tau
           + 2 * kNb * kNb                // T, G
           + (int64_t)kNb * n             // W
           + 2 * kMaxPassWgs * kPartStride + 2 * kPartStride;
}

figaro_status wide_qr_init(WideQr &w, double *ws, int64_t max_nv, int32_t n, std::string &err) {
    w.ldv = std::max<int64_t>(max_nv, 1);
    w.V = ws;
    w.tau = w.V + kNb * w.ldv;
    w.T = w.tau + n;
    w.G = w.T + kNb * kNb;
    w.W = w.G + kNb * kNb;
    w.part = w.W + (int64_t)kNb * n;
    w.head = w.part + 2 * kMaxPassWgs * kPartStride;
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
        err = "rocblas_create_handle failed";
        return FIGARO_EHIP;
    }
    // fixed reduction order in every product: results repeat bit for bit
    if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success) {
        rocblas_destroy_handle(h);
        err = "rocblas_set_atomics_mode failed";
        return FIGARO_EHIP;
    }
    w.blas = h;
    return FIGARO_OK;
}

void wide_qr_release(WideQr &w) {
    if (w.blas) rocblas_destroy_handle((rocblas_handle)w.blas);
    w.blas = nullptr;
}

figaro_status wide_qr(const WideQr &w, double *A, int64_t lda, int64_t h, int32_t n, bool tp, hipStream_t s,
                      std::string &err) {
    rocblas_handle bh = (rocblas_handle)w.blas;
    if (!bh || h < (tp ? n : 1) || wide_qr_panel_rows(h, n, tp) > w.ldv) {
        err = "blocked QR: bad shape";
        return FIGARO_EINVAL;
    }
    if (lda > INT32_MAX || w.ldv > INT32_MAX) {   // rocBLAS takes 32-bit leading dimensions
        err = "blocked QR: more than 2^31 rows";
        return FIGARO_EUNSUPPORTED;
    }
    if (rocblas_set_stream(bh, s) != rocblas_status_success) {
        err = "rocblas_set_stream failed";
        return FIGARO_EHIP;
    }
    auto hip_fail = [&](const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(hipGetLastError());
        return FIGARO_EHIP;
    };
    auto blas_fail = [&]() {
        err = "rocblas_dgemm failed";
        return FIGARO_EHIP;
    };
    const int64_t kend = tp ? n : std::min<int64_t>(n, h);
    for (int64_t k = 0; k < kend; k += kNb) {
        PanelArgs a{};
        a.A = A;
        a.lda = lda;
        a.k = k;
        a.kb = (int32_t)std::min<int64_t>(kNb, kend - k);
        a.s0 = tp ? n : k + a.kb;
        a.tp = tp ? 1 : 0;
        a.nv = a.kb + (h - a.s0);
        a.V = w.V;
        a.ldv = w.ldv;
        a.tau = w.tau + k;
        a.part = w.part;
        a.head = w.head;
        if (a.nv <= kSmallRows) {
            a.wgs = 1;
            a.rows_per_wg = a.nv;
            hipLaunchKernelGGL(k_panel_one, dim3(1), dim3(kPassThreads), 0, s, a);
            if (hipGetLastError() != hipSuccess) return hip_fail("panel");
        } else {
            a.wgs = (int32_t)std::min<int64_t>(kMaxPassWgs, (a.nv + kPassThreads - 1) / kPassThreads);
            a.rows_per_wg = (a.nv + a.wgs - 1) / a.wgs;
            for (int p = 0; p <= a.kb; ++p) {
                hipLaunchKernelGGL(k_panel_pass, dim3(a.wgs), dim3(kPassThreads), 0, s, a, p);
                if (hipGetLastError() != hipSuccess) return hip_fail("panel pass");
            }
        }
        const int64_t nc = n - k - a.kb;
        if (nc <= 0) continue;
        double *C = A + (k + a.kb) * lda;   // trailing columns, row 0
        // T from V^T V
        if (!gemm(bh, true, a.kb, a.kb, a.nv, 1.0, w.V, w.ldv, w.V, w.ldv, 0.0, w.G, kNb)) return blas_fail();
        hipLaunchKernelGGL(k_wy_t, dim3(1), dim3(64), 0, s, w.G, a.tau, a.kb, w.T);
        if (hipGetLastError() != hipSuccess) return hip_fail("wy T");
        // W = V^T C over the panel's rows, then the tail rows
        if (!tp) {
            if (!gemm(bh, true, a.kb, nc, a.nv, 1.0, w.V, w.ldv, C + k, lda, 0.0, w.W, kNb)) return blas_fail();
        } else {
            if (!gemm(bh, true, a.kb, nc, a.kb, 1.0, w.V, w.ldv, C + k, lda, 0.0, w.W, kNb)) return blas_fail();
            if (!gemm(bh, true, a.kb, nc, h - n, 1.0, w.V + a.kb, w.ldv, C + n, lda, 1.0, w.W, kNb))
                return blas_fail();
        }
        hipLaunchKernelGGL(k_wy_tw, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, w.T, a.kb, w.W, nc);
        if (hipGetLastError() != hipSuccess) return hip_fail("wy T^T W");
        // C -= V W
        if (!tp) {
            if (!gemm(bh, false, a.nv, nc, a.kb, -1.0, w.V, w.ldv, w.W, kNb, 1.0, C + k, lda)) return blas_fail();
        } else {
            if (!gemm(bh, false, a.kb, nc, a.kb, -1.0, w.V, w.ldv, w.W, kNb, 1.0, C + k, lda)) return blas_fail();
            if (!gemm(bh, false, h - n, nc, a.kb, -1.0, w.V + a.kb, w.ldv, w.W, kNb, 1.0, C + n, lda))
                return blas_fail();
        }
    }
    return FIGARO_OK;
}

hipError_t launch_copy_upper(const double *src, int64_t ld_src, int64_t rows, int32_t cols, double *dst,
                             int64_t ld_dst, int64_t row0, int64_t col0, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 255) / 256), (unsigned)cols);
    hipLaunchKernelGGL(k_copy_upper, grid, dim3(256), 0, s, src, ld_src, rows, cols, dst, ld_dst, row0, col0);
    return hipGetLastError();
}

hipError_t launch_final_r(const double *A, int64_t lda, int64_t rows, int32_t n, double *R, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_final_r, grid, dim3(256), 0, s, A, lda, rows, n, R);
    return hipGetLastError();
}

}  // namespace figaro
