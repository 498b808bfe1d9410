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
//     triangular; T is applied through its inverse, diag(1 / tau) plus the
//     strict upper triangle of V^T V);
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
// one workgroup with their rows in registers; tall ones take one launch per
// column over many workgroups, each launch first finishing the previous
// column's reflector from the partial sums every workgroup left, applying
// it to its rows, then leaving its partial sums for the next column.
// Nothing spins on another workgroup.  A triangular-pentagonal QR with few
// rows below the triangle (one root row, for a Cartesian product) takes
// one wave per panel, a panel column per lane, and one fused launch for
// the trailing update.  The panels of independent QRs (a plan's per-
// relation regions) share launches.
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
constexpr int kTpSmall = 64;        // tail rows up to which the triangular-pentagonal form has its own kernels

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
    double *head;   // [2][kPartStride]: the reflector's own row, from its column on
    int32_t wgs;
    int64_t rows_per_wg;
};

// The panels of up to kMaxJobs independent QRs, factored by one launch:
// job j owns workgroups [wg0[j], wg0[j + 1]).
constexpr int kMaxJobs = 8;
struct PanelBatch {
    PanelArgs a[kMaxJobs];
    int32_t wg0[kMaxJobs + 1];
    int32_t count;
};

__device__ __forceinline__ int job_of(const PanelBatch &b, int wg) {
    int j = 0;
    while (j + 1 < b.count && wg >= b.wg0[j + 1]) ++j;
    return j;
}

// The scalars of one reflector, derived by every thread from the
// reflector's own row and the reduced sums over its tail, both relative to
// the reflector's column (head[0] = alpha, head[c] = its row in column
// q + c; tot[0] = ||x||^2, tot[c] = x^T a_{q+c}); w_c = v^T a_{q+c} is read
// as head[c] + scale * tot[c] where it is used.
struct Refl {
    double tau, scale, beta;
    const double *head, *tot;
};

__device__ __forceinline__ Refl make_reflector_scalars(double alpha, double sig2) {
    Refl r;
    r.tau = 0.0;
    r.scale = 0.0;
    r.beta = alpha;
    if (sig2 > 0.0) {
        r.beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
        r.tau = (r.beta - alpha) / r.beta;
        r.scale = 1.0 / (alpha - r.beta);
    }
    r.head = nullptr;
    r.tot = nullptr;
    return r;
}

__device__ __forceinline__ Refl make_reflector(const double *head, const double *tot) {
    Refl r = make_reflector_scalars(head[0], tot[0]);
    r.head = head;
    r.tot = tot;
    return r;
}

// Workgroup barrier for LDS traffic only.  The panel kernels' global
// stores (reflectors, finished columns) are read by later launches alone,
// so the barrier waits for the LDS operations of every wave and lets the
// stores drain in the background (a full __syncthreads would wait for
// them at every column).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// v where keep holds, else +0.  A bit mask rather than a branch, so a
// load feeding it stays unconditional and all of a row's loads are in
// flight together (a guarded load compiles to a branch and a wait each).
__device__ __forceinline__ double keep_or_zero(double v, bool keep) {
    return __longlong_as_double(__double_as_longlong(v) & -(long long)keep);
}

__device__ __forceinline__ int64_t real_row(const PanelArgs &a, int64_t t) {
    return t < a.kb ? a.k + t : a.s0 + (t - a.kb);
}

// Whether virtual row t lies in the tail of reflector q (below its own row
// and, in triangular-pentagonal form, outside the triangular block).
__device__ __forceinline__ bool in_tail(const PanelArgs &a, int64_t t, int q) {
    return t > q && (!a.tp || t >= a.kb);
}

// A row held relative to the current column: y[c] is the row's entry in
// column q + c of the panel, so the pivot is always y[0] and every
// register index is a compile-time constant.  Entries beyond the panel's
// live width are zero, in the rows and in the reflector's row and sums, so
// the loops below run over all kNb entries without a branch.
//
// w[c] = v^T a_{q+c}, the same for every row: taken once per step.
__device__ __forceinline__ void reflector_w(const Refl &r, double (&w)[kNb]) {
#pragma unroll
    for (int c = 0; c < kNb; ++c) w[c] = r.head[c] + r.scale * r.tot[c];
}

// Reflector q applied to virtual row t; returns the row's entry of v (1 on
// the reflector's own row, 0 outside its rows) and whether the row changed.
__device__ __forceinline__ double apply_row(const PanelArgs &a, int64_t t, int q, const Refl &r,
                                            const double (&w)[kNb], double (&y)[kNb], bool &changed) {
    const bool own = t == q, tail = in_tail(a, t, q);
    const double v = own ? 1.0 : (tail ? y[0] * r.scale : 0.0);
    const double f = own ? r.tau : r.tau * v;
    y[0] = own ? r.beta : (tail ? v : y[0]);
#pragma unroll
    for (int c = 1; c < kNb; ++c) y[c] -= f * w[c];
    changed = own || tail;
    return v;
}

// Drop the pivot column: y[c] = y[c + 1].
__device__ __forceinline__ void shift_row(double (&y)[kNb]) {
#pragma unroll
    for (int c = 0; c + 1 < kNb; ++c) y[c] = y[c + 1];
    y[kNb - 1] = 0.0;
}

// Row t's share of the sums of reflector p (y relative to column p):
// ||x||^2 and x^T a_{p+c} into acc[c] for its tail rows; its own row goes
// to head_out.
__device__ __forceinline__ void accumulate_row(const PanelArgs &a, int64_t t, int p, const double (&y)[kNb],
                                               double (&acc)[kNb], double *head_out) {
    if (t == p) {
#pragma unroll
        for (int c = 0; c < kNb; ++c) head_out[c] = y[c];
    }
    const double y0 = in_tail(a, t, p) ? y[0] : 0.0;
#pragma unroll
    for (int c = 0; c < kNb; ++c) acc[c] += y0 * y[c];
}

// Sum acc[c] over the workgroup of TH threads into out[c] (all kNb
// entries): every thread's values through LDS (buf, column-major by
// thread), then TH / 32 threads per column add 32 each and combine within
// their group of lanes.  Ends with the values in out visible to the thread
// that wrote them only; the caller synchronises before others read them.
// (Rows of buf are TH + 1 doubles long, so the 32 columns a wave reads at
// once fall in different LDS banks.)
template <int TH>
__device__ __forceinline__ void block_sum(const double (&acc)[kNb], double (*buf)[TH + 1], double *out) {
    constexpr int SEG = TH / kNb;
#pragma unroll
    for (int c = 0; c < kNb; ++c) buf[c][threadIdx.x] = acc[c];
    lds_barrier();
    const int c = threadIdx.x / SEG, sg = threadIdx.x % SEG;
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int k = 0; k < kNb; k += 2) {
        v0 += buf[c][k * SEG + sg];
        v1 += buf[c][(k + 1) * SEG + sg];
    }
    double v = v0 + v1;
#pragma unroll
    for (int off = 1; off < SEG; off <<= 1) v += __shfl_xor(v, off);
    if (sg == 0) out[c] = v;
}

template <int TH>
struct OneShared {
    double buf[kNb][TH + 1];
    double tot[2][kNb], head[2][kNb];
};

// Whole panel in one workgroup of TH threads (nv <= RPT * TH): thread i
// holds virtual rows i, i + TH, ... in registers, relative to the current
// column; a column leaves the registers for memory when it has been the
// pivot.  The sums and the reflector's row alternate between two LDS
// buffers by column parity.
template <int RPT, int TH>
__global__ __launch_bounds__(TH) void k_panel_one(PanelBatch batch) {
    __shared__ OneShared<TH> sh;
    const PanelArgs a = batch.a[blockIdx.x];
    double y[RPT][kNb];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t t = threadIdx.x + (int64_t)i * TH;
        const double *base = a.A + real_row(a, t < a.nv ? t : 0) + a.k * a.lda;
#pragma unroll
        for (int c = 0; c < kNb; ++c)
            y[i][c] = keep_or_zero(base[(int64_t)(c < a.kb ? c : a.kb - 1) * a.lda], t < a.nv && c < a.kb);
    }
    for (int p = 0; p <= a.kb; ++p) {
        Refl r{};
        double w[kNb];
        if (p > 0) {
            r = make_reflector(sh.head[(p - 1) & 1], sh.tot[(p - 1) & 1]);
            reflector_w(r, w);
            if (threadIdx.x == 0) a.tau[p - 1] = r.tau;
        }
        double acc[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) acc[c] = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t t = threadIdx.x + (int64_t)i * TH;
            if (t >= a.nv) continue;
            if (p > 0) {
                bool changed;
                a.V[(int64_t)(p - 1) * a.ldv + t] = apply_row(a, t, p - 1, r, w, y[i], changed);
                a.A[real_row(a, t) + (a.k + p - 1) * a.lda] = y[i][0];
                shift_row(y[i]);
            }
            accumulate_row(a, t, p, y[i], acc, sh.head[p & 1]);
        }
        if (p < a.kb) {
            block_sum<TH>(acc, sh.buf, sh.tot[p & 1]);
            lds_barrier();
        }
    }
}

// A double of lane `src` (wave-uniform) in every lane.
__device__ __forceinline__ double readlane_f64(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Panel of the triangular-pentagonal form with a short tail (g <= GM rows
// below the triangle), one wave per job, one panel column per lane: lane c
// holds the panel's own rows of its column (top, relative to the current
// pivot row, which leaves when it is final) and the g tail rows.  The
// sums of a reflector are then dot products within each lane over the
// tail; the pivot column's tail goes to every lane by lane reads (up to 16
// rows: no LDS round trip and no barrier per column) or through LDS.
template <int GM>
__global__ __launch_bounds__(64) void k_panel_tp(PanelBatch batch) {
    constexpr bool BCAST = GM <= 16;
    __shared__ double sx[BCAST ? 1 : GM];
    __shared__ double salpha;
    const PanelArgs a = batch.a[blockIdx.x];
    const int lane = threadIdx.x;
    const int g = (int)(a.nv - a.kb);
    const int c = lane < a.kb ? lane : a.kb - 1;   // clamped column of this lane
    const bool live = lane < a.kb;
    const double *col = a.A + (a.k + c) * a.lda;
    double top[kNb], tail[GM];
#pragma unroll
    for (int i = 0; i < kNb; ++i) top[i] = keep_or_zero(col[a.k + (i < a.kb ? i : a.kb - 1)], live && i < a.kb);
#pragma unroll
    for (int r = 0; r < GM; ++r) tail[r] = keep_or_zero(col[r < g ? a.s0 + r : a.k], live && r < g);
    for (int p = 0; p < a.kb; ++p) {
        double x[GM], alpha;
        if constexpr (BCAST) {
#pragma unroll
            for (int r = 0; r < GM; ++r) x[r] = readlane_f64(tail[r], p);
            alpha = readlane_f64(top[0], p);
        } else {
            if (lane == p) {
#pragma unroll
                for (int r = 0; r < GM; ++r) sx[r] = tail[r];
                salpha = top[0];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < GM; ++r) x[r] = sx[r];
            alpha = salpha;
        }
        double sig2 = 0.0, d = 0.0;
#pragma unroll
        for (int r = 0; r < GM; ++r) {
            sig2 += x[r] * x[r];
            d += x[r] * tail[r];
        }
        const Refl rf = make_reflector_scalars(alpha, sig2);
        // V column p: 1 on the pivot's own row, 0 on the triangle's other
        // rows, the scaled tail below
        if constexpr (BCAST) {
            if (lane < a.kb) a.V[(int64_t)p * a.ldv + lane] = lane == p ? 1.0 : 0.0;
            if (lane == p) {
#pragma unroll
                for (int r = 0; r < GM; ++r)
                    if (r < g) a.V[(int64_t)p * a.ldv + a.kb + r] = tail[r] * rf.scale;
            }
        } else {
            for (int64_t t = lane; t < a.nv; t += 64)
                a.V[(int64_t)p * a.ldv + t] = t < a.kb ? (t == p ? 1.0 : 0.0) : sx[t - a.kb] * rf.scale;
        }
        if (lane == 0) a.tau[p] = rf.tau;
        if (live && lane > p) {
            const double w = top[0] + rf.scale * d;
            const double f = rf.tau * w;
            top[0] -= f;
            const double fv = f * rf.scale;
#pragma unroll
            for (int r = 0; r < GM; ++r) tail[r] -= fv * x[r];
        }
        if (live && lane == p) top[0] = rf.beta;
        if (live && lane >= p) a.A[(a.k + p) + (a.k + lane) * a.lda] = top[0];
#pragma unroll
        for (int i = 0; i + 1 < kNb; ++i) top[i] = top[i + 1];
        top[kNb - 1] = 0.0;
        if constexpr (!BCAST) __syncthreads();
    }
}

// Column step p of a tall panel; workgroup b owns virtual rows
// [b * rows_per_wg, (b + 1) * rows_per_wg).  Partial sums and the
// reflector's row alternate between two buffers by column parity, so a
// launch never overwrites what a workgroup of the same launch still reads.
__global__ __launch_bounds__(kPassThreads) void k_panel_pass(PanelBatch batch, int p) {
    __shared__ double buf[kNb][kPassThreads + 1];
    __shared__ double tot[kNb], hd[kNb];
    const int job = job_of(batch, blockIdx.x);
    const PanelArgs a = batch.a[job];
    const int wg = blockIdx.x - batch.wg0[job];
    if (p > a.kb) return;   // a narrower panel of the batch is done
    const int q = p - 1;
    const int c_lo = p > 0 ? q : p;
    const int width = a.kb - c_lo;
    const int64_t t0 = (int64_t)wg * a.rows_per_wg;
    const int64_t t1 = std::min<int64_t>(a.nv, t0 + a.rows_per_wg);
    // the first row's loads go out before the partial sums are read, so
    // the two memory round trips overlap
    double y[kNb];
    {
        const int64_t t = t0 + threadIdx.x < t1 ? t0 + threadIdx.x : t0;
        const double *base = a.A + real_row(a, t < a.nv ? t : 0) + (a.k + c_lo) * a.lda;
#pragma unroll
        for (int c = 0; c < kNb; ++c) y[c] = keep_or_zero(base[(int64_t)(c < width ? c : width - 1) * a.lda], c < width);
    }
    Refl r{};
    double w[kNb];
    if (p > 0) {
        // the previous launch's partial sums: 8 threads per column
        const double *prt = a.part + (int64_t)(q & 1) * a.wgs * kPartStride;
        const int c = threadIdx.x >> 3, sg = threadIdx.x & 7;
        double v = 0.0;
        for (int b = sg; b < a.wgs; b += 8) v += prt[(int64_t)b * kPartStride + c];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (sg == 0) {
            tot[c] = v;
            hd[c] = a.head[(q & 1) * kPartStride + c];
        }
        lds_barrier();
        r = make_reflector(hd, tot);
        reflector_w(r, w);
        if (wg == 0 && threadIdx.x == 0) a.tau[q] = r.tau;
    }
    double acc[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) acc[c] = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kPassThreads) {
        double *base = a.A + real_row(a, t) + (a.k + c_lo) * a.lda;
        if (t != t0 + threadIdx.x) {
#pragma unroll
            for (int c = 0; c < kNb; ++c)
                y[c] = keep_or_zero(base[(int64_t)(c < width ? c : width - 1) * a.lda], c < width);
        }
        if (p > 0) {
            bool changed;
            a.V[(int64_t)q * a.ldv + t] = apply_row(a, t, q, r, w, y, changed);
            if (changed) {
                // highest column first: the clamped addresses of the
                // columns beyond the width all land on the last live
                // column, which its own store then sets
#pragma unroll
                for (int c = kNb - 1; c >= 0; --c)
                    base[(int64_t)(c < width ? c : width - 1) * a.lda] = c < width ? y[c] : 0.0;
            }
            shift_row(y);
        }
        if (p < a.kb) accumulate_row(a, t, p, y, acc, a.head + (p & 1) * kPartStride);
    }
    if (p < a.kb) block_sum<kPassThreads>(acc, buf, a.part + ((int64_t)(p & 1) * a.wgs + wg) * kPartStride);
}

// Partial Gram products of a panel's reflectors, P_b = V_b^T V_b over the
// virtual rows [b kGramRows, (b + 1) kGramRows) (V: kb live columns of
// leading dimension ldv, nv rows; columns from kb on count as zero), part b
// at P + b * kNb * kNb, summed by k_wy_g.  The rows are staged in LDS once;
// thread t forms four entries of row t / 8.
constexpr int kGramRows = 128;
__global__ __launch_bounds__(256) void k_vtv_parts(const double *V, int64_t ldv, int kb, int64_t nv, double *P) {
    __shared__ double sV[kNb][kGramRows + 1];
    const int64_t r0 = (int64_t)blockIdx.x * kGramRows;
    for (int e = threadIdx.x; e < kNb * kGramRows; e += blockDim.x) {
        const int c = e / kGramRows, r = e % kGramRows;
        sV[c][r] = (c < kb && r0 + r < nv) ? V[(int64_t)c * ldv + r0 + r] : 0.0;
    }
    __syncthreads();
    const int i = threadIdx.x >> 3, j = (threadIdx.x & 7) * 4;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
    for (int r = 0; r < kGramRows; ++r) {
        const double v = sV[i][r];
        a0 = fma(v, sV[j][r], a0);
        a1 = fma(v, sV[j + 1][r], a1);
        a2 = fma(v, sV[j + 2][r], a2);
        a3 = fma(v, sV[j + 3][r], a3);
    }
    double *out = P + (int64_t)blockIdx.x * kNb * kNb + i * kNb + j;
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
}

int64_t gram_parts(int64_t rows) { return std::max<int64_t>(1, (rows + kGramRows - 1) / kGramRows); }

// G = V^T V from its nparts partial products (part b at Gp + b * kNb * kNb);
// workgroup b sums the entries [256 b, 256 b + 256).
__global__ __launch_bounds__(256) void k_wy_g(const double *Gp, int nparts, double *G) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kNb * kNb; e += gridDim.x * blockDim.x) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        int b = 0;
        for (; b + 4 <= nparts; b += 4) {
            g0 += Gp[(int64_t)(b + 0) * kNb * kNb + e];
            g1 += Gp[(int64_t)(b + 1) * kNb * kNb + e];
            g2 += Gp[(int64_t)(b + 2) * kNb * kNb + e];
            g3 += Gp[(int64_t)(b + 3) * kNb * kNb + e];
        }
        for (; b < nparts; ++b) g0 += Gp[(int64_t)b * kNb * kNb + e];
        G[e] = (g0 + g1) + (g2 + g3);
    }
}

// Forward substitution of one column through T^T: T is never formed, its
// inverse being diag(1 / tau) plus the strict upper triangle of G = V^T V
// (the column recurrence of T, inverted block by block), so W2 = T^T W
// solves (diag(1 / tau) + strictly-lower(G^T)) W2 = W:
//   W2_i = tau_i (W_i - sum_{j < i} G(j, i) W2_j),
// which also gives W2_i = 0 for a reflector with tau_i = 0 (the identity).
// Taken column by column: W2_j is final once the columns before it have
// been subtracted.  sG[j][i] = G(i, j) in LDS (rows padded; G symmetric).
// (An empty asm statement per column keeps the compiler from hoisting all
// 496 LDS reads of G ahead of the arithmetic, which would spill.)
__device__ __forceinline__ void solve_t(const double (*sG)[kNb + 1], const double *stau, double (&w)[kNb]) {
#pragma unroll
    for (int j = 0; j < kNb; ++j) {
        w[j] *= stau[j];
#pragma unroll
        for (int i = j + 1; i < kNb; ++i) w[i] -= sG[j][i] * w[j];
        asm volatile("" ::: "memory");
    }
}

// W2 = T^T W for the kb x nc block W, W the sum of nparts partial products
// (part b at Wp + b * part_stride, kNb x nc, leading dimension kNb): 32
// threads per column (coalesced partial sums), 8 columns per workgroup;
// the substitution of a column runs over its 32 threads in lock step.
__global__ __launch_bounds__(256) void k_wy_tw(const double *Wp, int64_t part_stride, int nparts, const double *G,
                                               const double *tau, int kb, double *W2, int64_t nc) {
    __shared__ double sG[kNb][kNb + 1];   // sG[q][i] = G(i, q), rows padded against bank conflicts
    __shared__ double sW[8][kNb];
    for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) sG[e / kNb][e % kNb] = G[e];
    const int q = threadIdx.x & (kNb - 1), cl = threadIdx.x / kNb;
    const int64_t c = (int64_t)blockIdx.x * 8 + cl;
    double w0 = 0.0, w1 = 0.0;
    if (c < nc && q < kb) {
        int b = 0;
        for (; b + 2 <= nparts; b += 2) {
            w0 += Wp[(int64_t)b * part_stride + c * kNb + q];
            w1 += Wp[(int64_t)(b + 1) * part_stride + c * kNb + q];
        }
        if (b < nparts) w0 += Wp[(int64_t)b * part_stride + c * kNb + q];
    }
    const double w = w0 + w1;
    const double tq = q < kb ? tau[q] : 0.0;
    __syncthreads();
    // step i: thread q == i finishes W2_i (the sum over j < i is complete)
    double acc = 0.0;
    for (int i = 0; i < kb; ++i) {
        if (q == i) sW[cl][i] = tq * (w - acc);
        __syncthreads();
        if (q > i) acc += sG[q][i] * sW[cl][i];   // G(i, q) W2_i
    }
    if (c < nc && q < kb) W2[c * kNb + q] = sW[cl][q];
}

// The whole trailing update of a triangular-pentagonal panel whose tail
// has few rows (g <= kTpSmall), in one launch: for trailing column c,
//   W = C_top[:, c] + V_S^T C_S[:, c],  W2 = T^T W,
//   C_top[:, c] -= W2,  C_S[:, c] -= V_S W2,
// with V = [I; V_S] (the panel's own rows of V are the identity) and
// G = I + V_S^T V_S.  C_top: the panel's rows of the triangular block;
// C_S: the g tail rows.  32 lanes per column (lane q: panel row q, so the
// column's panel rows are one contiguous load), 8 columns per workgroup;
// T^T is applied by forward substitution through its inverse, one row per
// step, W2_i going from lane i to the other lanes by a shuffle:
//   W2_i = tau_i (W_i - sum_{j < i} G(j, i) W2_j).
constexpr int kTpCols = 8;   // columns per workgroup of k_tp_update
__global__ __launch_bounds__(256) void k_tp_update(const double *V, int64_t ldv, const double *tau, int kb, int g,
                                                   double *Ctop, double *CS, int64_t lda, int64_t nc) {
    __shared__ double sVS[kTpSmall][kNb];
    __shared__ double sG[kNb][kNb + 1];
    __shared__ double stau[kNb];
    __shared__ double sW[kTpCols][kNb];
    for (int e = threadIdx.x; e < kTpSmall * kNb; e += blockDim.x) {
        const int r = e / kNb, q = e % kNb;
        sVS[r][q] = (r < g && q < kb) ? V[(int64_t)q * ldv + kb + r] : 0.0;
    }
    if (threadIdx.x < kNb) stau[threadIdx.x] = threadIdx.x < kb ? tau[threadIdx.x] : 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
        const int i = e / kNb, j = e % kNb;
        double s = (i == j) ? 1.0 : 0.0;
#pragma unroll 1
        for (int r = 0; r < g; ++r) s += sVS[r][i] * sVS[r][j];
        sG[i][j] = s;
    }
    __syncthreads();
    const int q = threadIdx.x & (kNb - 1), cl = threadIdx.x / kNb;
    const int64_t c = (int64_t)blockIdx.x * kTpCols + cl;
    const bool live = c < nc;
    double *top = Ctop + (live ? c : 0) * lda;
    double *cs = CS + (live ? c : 0) * lda;
    const double t0 = (live && q < kb) ? top[q] : 0.0;
    double w = t0;
#pragma unroll 1
    for (int r = 0; r < g; ++r) w += sVS[r][q] * (live ? cs[r] : 0.0);
    const double tq = stau[q];   // 0 beyond kb: those lanes keep W2 = 0
    double acc = 0.0, w2 = 0.0;
#pragma unroll 1
    for (int i = 0; i < kb; ++i) {
        const double b = __shfl(tq * (w - acc), i, kNb);   // W2_i, final on lane i
        if (q == i) w2 = b;
        if (q > i) acc += sG[i][q] * b;
    }
    if (live && q < kb) top[q] = t0 - w2;
    sW[cl][q] = w2;
    __syncthreads();
    // C_S[r] -= sum_q V_S[r][q] W2_q, lane r of the column's 32
#pragma unroll 1
    for (int r = q; r < g; r += kNb) {
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < kNb; ++k) d += sVS[r][k] * sW[cl][k];
        if (live) cs[r] -= d;
    }
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

// Rows of one slice of the split products V^T X: the long dimension is cut
// into slices of kSplitRows rows, each a GEMM of its own (one strided
// batch), and the partial products are summed by the kernel that reads them.
constexpr int64_t kSplitRows = 512;

int64_t split_parts(int64_t rows) { return std::max<int64_t>(1, (rows + kSplitRows - 1) / kSplitRows); }

// Partial products P_b = V_b^T X_b (kNb x nc each, leading dimension kNb,
// part b at P + b * part_stride) over the row slices of V (rows x kb, ldv)
// and X (rows x nc, ldx), from part `first` on.  Returns the parts written.
// (With only kb = 32 output rows, rocBLAS reaches the FP64 peak on these
// slices; the products' own long dimension would give it a handful of
// workgroups.)
bool split_vt_x(rocblas_handle h, int kb, int64_t nc, int64_t rows, const double *V, int64_t ldv, const double *X,
                int64_t ldx, double *P, int64_t part_stride, int64_t first, int64_t &parts) {
    parts = 0;
    if (rows <= 0 || nc <= 0) return true;
    const int64_t full = rows / kSplitRows, rem = rows - full * kSplitRows;
    const double one = 1.0, zero = 0.0;
    const double *A = V, *B = X;
    const int64_t lda = ldv, ldb = ldx;
    const int64_t m = kb, n = nc, ldc = kNb;
    if (full > 0) {
        if (rocblas_dgemm_strided_batched(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)m,
                                          (rocblas_int)n, (rocblas_int)kSplitRows, &one, A, (rocblas_int)lda,
                                          kSplitRows, B, (rocblas_int)ldb, kSplitRows, &zero,
                                          P + first * part_stride, (rocblas_int)ldc, part_stride,
                                          (rocblas_int)full) != rocblas_status_success)
            return false;
        parts += full;
    }
    if (rem > 0) {
        if (!gemm(h, true, m, n, rem, 1.0, A + full * kSplitRows, lda, B + full * kSplitRows, ldb, 0.0,
                  P + (first + parts) * part_stride, ldc))
            return false;
        parts += 1;
    }
    return true;
}

}  // namespace

int64_t wide_qr_panel_rows(int64_t h, int32_t n, bool tp) {
    return tp ? kNb + std::max<int64_t>(0, h - n) : std::max<int64_t>(h, kNb);
}

int64_t wide_qr_workspace_doubles(int64_t max_nv, int32_t n) {
    const int64_t parts = split_parts(max_nv) + 1;
    return (int64_t)kNb * max_nv                          // V
           + n                                            // tau
           + kNb * kNb                                    // T
           + gram_parts(max_nv) * kNb * kNb               // partial V^T V
           + (int64_t)kNb * n                             // W2
           + parts * kNb * std::max<int64_t>(n, kNb)      // partial V^T C
           + 2 * kMaxPassWgs * kPartStride + 2 * kPartStride;
}

figaro_status wide_qr_init(WideQr &w, double *ws, int64_t max_nv, int32_t n, void *blas, std::string &err) {
    w.ldv = std::max<int64_t>(max_nv, 1);
    const int64_t parts = split_parts(w.ldv) + 1;
    w.V = ws;
    w.tau = w.V + kNb * w.ldv;
    w.T = w.tau + n;
    w.G = w.T + kNb * kNb;
    w.W = w.G + gram_parts(w.ldv) * kNb * kNb;
    w.Wp = w.W + (int64_t)kNb * n;
    w.wp_stride = kNb * std::max<int64_t>(n, kNb);
    w.part = w.Wp + parts * w.wp_stride;
    w.head = w.part + 2 * kMaxPassWgs * kPartStride;
    if (blas) {   // a handle shared with another workspace of the plan
        w.blas = blas;
        return FIGARO_OK;
    }
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

namespace {

// The panel of job J at column k (false once the job has no panel there).
bool panel_args(const WideQrJob &J, int64_t k, PanelArgs &a) {
    const int64_t kend = J.tp ? J.n : std::min<int64_t>(J.n, J.h);
    if (k >= kend) return false;
    a = PanelArgs{};
    a.A = J.A;
    a.lda = J.lda;
    a.k = k;
    a.kb = (int32_t)std::min<int64_t>(kNb, kend - k);
    a.s0 = J.tp ? J.n : k + a.kb;
    a.tp = J.tp ? 1 : 0;
    a.nv = a.kb + (J.h - a.s0);
    a.V = J.w->V;
    a.ldv = J.w->ldv;
    a.tau = J.w->tau + k;
    a.part = J.w->part;
    a.head = J.w->head;
    if (a.nv <= kSmallRows) {
        a.wgs = 1;
        a.rows_per_wg = a.nv;
    } else {
        a.wgs = (int32_t)std::min<int64_t>(kMaxPassWgs, (a.nv + kPassThreads - 1) / kPassThreads);
        a.rows_per_wg = (a.nv + a.wgs - 1) / a.wgs;
    }
    return true;
}

// One-workgroup panels: one launch per register shape, one workgroup per job.
hipError_t launch_small_panels(const std::vector<PanelArgs> &pa, hipStream_t s) {
    for (int shape = 0; shape < 7; ++shape) {
        PanelBatch b{};
        for (const PanelArgs &a : pa) {
            const int64_t g = a.nv - a.kb;
            const int sh = (a.tp && g <= 4) ? 4 : (a.tp && g <= 16) ? 5 : (a.tp && g <= kTpSmall) ? 6
                           : a.nv <= 64 ? 0 : a.nv <= kPassThreads ? 1 : a.nv <= 2 * kPassThreads ? 2 : 3;
            if (sh == shape) b.a[b.count++] = a;
        }
        if (b.count == 0) continue;
        switch (shape) {
            case 4: hipLaunchKernelGGL((k_panel_tp<4>), dim3(b.count), dim3(64), 0, s, b); break;
            case 5: hipLaunchKernelGGL((k_panel_tp<16>), dim3(b.count), dim3(64), 0, s, b); break;
            case 6: hipLaunchKernelGGL((k_panel_tp<kTpSmall>), dim3(b.count), dim3(64), 0, s, b); break;
            case 0: hipLaunchKernelGGL((k_panel_one<1, 64>), dim3(b.count), dim3(64), 0, s, b); break;
            case 1: hipLaunchKernelGGL((k_panel_one<1, kPassThreads>), dim3(b.count), dim3(kPassThreads), 0, s, b); break;
            case 2: hipLaunchKernelGGL((k_panel_one<2, kPassThreads>), dim3(b.count), dim3(kPassThreads), 0, s, b); break;
            default: hipLaunchKernelGGL((k_panel_one<4, kPassThreads>), dim3(b.count), dim3(kPassThreads), 0, s, b);
        }
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    return hipSuccess;
}

// Tall panels: one launch per column over the workgroups of every job.
hipError_t launch_tall_panels(const std::vector<PanelArgs> &pa, hipStream_t s) {
    if (pa.empty()) return hipSuccess;
    PanelBatch b{};
    int kbmax = 0;
    for (const PanelArgs &a : pa) {
        b.a[b.count] = a;
        b.wg0[b.count + 1] = b.wg0[b.count] + a.wgs;
        ++b.count;
        kbmax = std::max(kbmax, (int)a.kb);
    }
    for (int p = 0; p <= kbmax; ++p) {
        hipLaunchKernelGGL(k_panel_pass, dim3(b.wg0[b.count]), dim3(kPassThreads), 0, s, b, p);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    return hipSuccess;
}

}  // namespace

figaro_status wide_qr_many(const std::vector<WideQrJob> &jobs, hipStream_t s, std::string &err) {
    if (jobs.empty()) return FIGARO_OK;
    if (jobs.size() > (size_t)kMaxJobs) {
        for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxJobs) {
            std::vector<WideQrJob> part(jobs.begin() + j0, jobs.begin() + std::min(jobs.size(), j0 + kMaxJobs));
            if (figaro_status st = wide_qr_many(part, s, err); st != FIGARO_OK) return st;
        }
        return FIGARO_OK;
    }
    rocblas_handle bh = (rocblas_handle)jobs[0].w->blas;
    int64_t kmax = 0;
    for (const WideQrJob &J : jobs) {
        if (!J.w->blas || J.h < (J.tp ? J.n : 1) || wide_qr_panel_rows(J.h, J.n, J.tp) > J.w->ldv) {
            err = "blocked QR: bad shape";
            return FIGARO_EINVAL;
        }
        if (J.lda > INT32_MAX || J.w->ldv > INT32_MAX) {   // rocBLAS takes 32-bit leading dimensions
            err = "blocked QR: more than 2^31 rows";
            return FIGARO_EUNSUPPORTED;
        }
        kmax = std::max<int64_t>(kmax, J.tp ? J.n : std::min<int64_t>(J.n, J.h));
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
    for (int64_t k = 0; k < kmax; k += kNb) {
        std::vector<PanelArgs> small, tall;
        std::vector<std::pair<const WideQrJob *, PanelArgs>> active;
        for (const WideQrJob &J : jobs) {
            PanelArgs a;
            if (!panel_args(J, k, a)) continue;
            (a.nv <= kSmallRows ? small : tall).push_back(a);
            active.push_back({&J, a});
        }
        if (launch_small_panels(small, s) != hipSuccess) return hip_fail("panel");
        if (launch_tall_panels(tall, s) != hipSuccess) return hip_fail("panel pass");
        for (auto &[Jp, a] : active) {
            const WideQrJob &J = *Jp;
            const WideQr &w = *J.w;
            const int64_t n = J.n, h = J.h, lda = J.lda;
            const bool tp = J.tp;
            const int64_t nc = n - k - a.kb;
            if (nc <= 0) continue;
            double *C = J.A + (k + a.kb) * lda;   // trailing columns, row 0
            if (tp && h - n <= kTpSmall) {
                hipLaunchKernelGGL(k_tp_update, dim3((unsigned)((nc + kTpCols - 1) / kTpCols)), dim3(256), 0, s, w.V, w.ldv,
                                   a.tau, a.kb, (int)(h - n), C + k, C + n, lda, nc);
                if (hipGetLastError() != hipSuccess) return hip_fail("tp update");
                continue;
            }
            // V^T V (split over the rows and summed)
            const int64_t gparts = gram_parts(a.nv);
            hipLaunchKernelGGL(k_vtv_parts, dim3((unsigned)gparts), dim3(256), 0, s, w.V, w.ldv, (int)a.kb, a.nv,
                               w.G);
            if (hipGetLastError() != hipSuccess) return hip_fail("V^T V");
            hipLaunchKernelGGL(k_wy_g, dim3(kNb * kNb / 256), dim3(256), 0, s, w.G, (int)gparts, w.T);
            if (hipGetLastError() != hipSuccess) return hip_fail("wy G");
            // W2 = T^T V^T C over the panel's rows and the tail rows (split
            // products, summed with the T^T product)
            int64_t wparts = 0, more = 0;
            if (!tp) {
                if (!split_vt_x(bh, a.kb, nc, a.nv, w.V, w.ldv, C + k, lda, w.Wp, w.wp_stride, 0, wparts))
                    return blas_fail();
            } else {
                if (!split_vt_x(bh, a.kb, nc, a.kb, w.V, w.ldv, C + k, lda, w.Wp, w.wp_stride, 0, wparts))
                    return blas_fail();
                if (!split_vt_x(bh, a.kb, nc, h - n, w.V + a.kb, w.ldv, C + n, lda, w.Wp, w.wp_stride, wparts, more))
                    return blas_fail();
                wparts += more;
            }
            hipLaunchKernelGGL(k_wy_tw, dim3((unsigned)((nc + 7) / 8)), dim3(256), 0, s, w.Wp, w.wp_stride,
                               (int)wparts, w.T, a.tau, a.kb, w.W, nc);
            if (hipGetLastError() != hipSuccess) return hip_fail("wy T^T W");
            // C -= V W2
            if (!tp) {
                if (!gemm(bh, false, a.nv, nc, a.kb, -1.0, w.V, w.ldv, w.W, kNb, 1.0, C + k, lda))
                    return blas_fail();
            } else {
                if (!gemm(bh, false, a.kb, nc, a.kb, -1.0, w.V, w.ldv, w.W, kNb, 1.0, C + k, lda))
                    return blas_fail();
                if (!gemm(bh, false, h - n, nc, a.kb, -1.0, w.V + a.kb, w.ldv, w.W, kNb, 1.0, C + n, lda))
                    return blas_fail();
            }
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
