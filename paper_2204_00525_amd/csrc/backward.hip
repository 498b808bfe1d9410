// Backward (adjoint) kernels for gfx950.
//
// R depends on the values only through R0 (Theorem 6: R0^T R0 = A^T A), and
// R0 is a linear function of the values once the keys are fixed.  With
// K = R^{-1} copyltu(R triu(dR)^T) R^{-T} (the adjoint of the R factor of a
// QR decomposition: dA = A K for any A with R^T R = A^T A), the gradient of
// every R0 row r is r K, restricted to the columns the row can be non-zero in.
// The kernels below push r K back through the head/tail recurrences, the
// join of the children's heads and the root heads to the relation values.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "bwd_batch.hpp"
#include "device_common.hpp"
#include "tails.hpp"

namespace figaro {
namespace {

// K = R^{-1} Phi R^{-T} with Phi = tril(M) + tril(M,-1)^T, M = R triu(dR)^T.
// n <= 64: everything in LDS.  R and triu(dR) are staged; the n^2 entries of
// Phi are spread over the 256 threads; then thread t < n solves R Y[:, t] =
// Phi[:, t] in place and R K[:, t] = Y[t, :]^T (back substitutions, the
// operands in LDS, so only the FMA chain is sequential).
constexpr int kAdjSmall = 64;
__global__ __launch_bounds__(256) void k_qr_adjoint_small(const double *R, const double *dR, int n, double *K,
                                                          int32_t *status) {
    __shared__ double sR[kAdjSmall][kAdjSmall + 1];
    __shared__ double sD[kAdjSmall][kAdjSmall + 1];
    __shared__ double sW[kAdjSmall][kAdjSmall + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        sR[r][c] = (c >= r) ? R[e] : 0.0;
        sD[r][c] = (c >= r) ? dR[e] : 0.0;
    }
    __syncthreads();
    // Phi[i][t] = M[a][b], a = max(i, t), b = min(i, t), M[a][b] = sum_{k >= a} R[a][k] dR[b][k]
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e % n, t = e / n;
        const int a = (i >= t) ? i : t, b = (i >= t) ? t : i;
        double m = 0.0;
        for (int k = a; k < n; ++k) m = fma(sR[a][k], sD[b][k], m);
        sW[i][t] = m;
    }
    __syncthreads();
    if (tid < n) {
        // Y[:, t] = R^{-1} Phi[:, t]
        const int t = tid;
        for (int i = n - 1; i >= 0; --i) {
            double y = sW[i][t];
            for (int k = i + 1; k < n; ++k) y = fma(-sR[i][k], sW[k][t], y);
            sW[i][t] = y / sR[i][i];
        }
    }
    __syncthreads();
    if (tid < n) {
        // K[:, t] = R^{-1} Y[t, :]^T, built in row t of sD (dR is no longer needed)
        const int t = tid;
        for (int i = n - 1; i >= 0; --i) {
            double y = sW[t][i];
            for (int k = i + 1; k < n; ++k) y = fma(-sR[i][k], sD[t][k], y);
            sD[t][i] = y / sR[i][i];
        }
        for (int i = 0; i < n; ++i) K[(int64_t)t * n + i] = sD[t][i];
    }
    if (tid == 0) {
        int32_t singular = 0;
        for (int i = 0; i < n; ++i) singular |= (sR[i][i] == 0.0) ? 1 : 0;
        status[0] = singular;
    }
}

// The same for n <= 128: R and triu(dR) staged in LDS as packed upper
// triangles (row r from column r on, 2 x 66 KB at n = 128), the n^2 entries
// of Phi over 256 threads into W (global, n x n), then thread t < n solves
// R Y[:, t] = Phi[:, t] in W and R K[:, t] = Y[t, :]^T.
constexpr int kAdjPack = kMaxCols * (kMaxCols + 1) / 2;
__device__ __forceinline__ int packed_row(int r, int n) { return r * n - r * (r - 1) / 2 - r; }
__global__ __launch_bounds__(256) void k_qr_adjoint(const double *R, const double *dR, int n, double *K,
                                                    double *W, int32_t *status) {
    __shared__ double sR[kAdjPack];
    __shared__ double sD[kAdjPack];
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        if (c >= r) {
            sR[packed_row(r, n) + c] = R[e];
            sD[packed_row(r, n) + c] = dR[e];
        }
    }
    __syncthreads();
    // Phi[i][t] = M[a][b], a = max(i, t), b = min(i, t), M[a][b] = sum_{k >= a} R[a][k] dR[b][k]
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e % n, t = e / n;
        const int a = (i >= t) ? i : t, b = (i >= t) ? t : i;
        const double *ra = sR + packed_row(a, n), *db = sD + packed_row(b, n);
        double m0 = 0.0, m1 = 0.0;
        int k = a;
        for (; k + 1 < n; k += 2) {
            m0 = fma(ra[k], db[k], m0);
            m1 = fma(ra[k + 1], db[k + 1], m1);
        }
        if (k < n) m0 = fma(ra[k], db[k], m0);
        W[(int64_t)t * n + i] = m0 + m1;
    }
    __syncthreads();
    if (tid < n) {
        // Y[:, t] = R^{-1} Phi[:, t]
        const int t = tid;
        double *w = W + (int64_t)t * n;
        for (int i = n - 1; i >= 0; --i) {
            const double *ri = sR + packed_row(i, n);
            double y = w[i];
            for (int k = i + 1; k < n; ++k) y = fma(-ri[k], w[k], y);
            w[i] = y / ri[i];
        }
    }
    __syncthreads();
    if (tid < n) {
        // K[:, t] = R^{-1} (row t of Y)
        const int t = tid;
        double *kt = K + (int64_t)t * n;
        for (int i = n - 1; i >= 0; --i) {
            const double *ri = sR + packed_row(i, n);
            double y = W[(int64_t)i * n + t];
            for (int k = i + 1; k < n; ++k) y = fma(-ri[k], kt[k], y);
            kt[i] = y / ri[i];
        }
    }
    if (tid == 0) {
        int32_t singular = 0;
        for (int i = 0; i < n; ++i) singular |= (sR[packed_row(i, n) + i] == 0.0) ? 1 : 0;
        status[0] = singular;
    }
}

// Second half of the backward of a head/tail tile: g holds dT (the
// gradient of the tail rows) on the output columns oc0 .. oc0 + nout - 1 of
// the level.  w = beta dT; the suffix sums over each piece run as a forward
// segmented scan over the lanes in reverse order; the item gradients
//   ds_t = alpha_t dT_t - sum_{u > t in its piece} w_u + dsigma[piece of t]
// are written to gout (column-major through the wave's LDS staging slice, or
// row-major directly).
template <int NB, int RPL>
__device__ __forceinline__ void bwd_finish(const HelmertBwdArgs &a, double (&x)[RPL][NB], const TileItems<RPL> &ti,
                                           int64_t cs, int64_t ce, int lane, int oc0, int nout, double *st,
                                           double *rs = nullptr) {
    double agg[NB];
    bool lane_last = false;
#pragma unroll
    for (int c = 0; c < NB; ++c) agg[c] = 0.0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        // lane aggregate for the lanes below: items up to and including the
        // lane's first piece end
        const double wk = lane_last ? 0.0 : ti.be[k];
#pragma unroll
        for (int c = 0; c < NB; ++c) agg[c] = fma(wk, x[k][c], agg[c]);
        lane_last = lane_last || ti.last[k];
    }
    const int rev = 63 - lane;
#pragma unroll
    for (int c = 0; c < NB; ++c) agg[c] = __shfl(agg[c], rev, 64);
    segmented_carry<NB>(agg, __builtin_bitreverse64(__ballot(lane_last)), lane);
    double run[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) run[c] = __shfl(agg[c], rev, 64);
#pragma unroll
    for (int k = RPL - 1; k >= 0; --k) {
        const double lm = ti.last[k] ? 0.0 : 1.0;
        const int32_t pk = ti.valid[k] ? ti.pid[k] : 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double E = run[c] * lm;
            const double gp = (c < nout) ? a.gpieces[(int64_t)(oc0 + c) * a.ld_gp + pk] : 0.0;
            const double out = fma(ti.al[k], x[k][c], -E) + gp;
            run[c] = fma(ti.be[k], x[k][c], E);
            x[k][c] = out;
        }
    }
    const int64_t nitems = ce - cs;
    if (a.gout_rowmajor && rs && oc0 == 0 && nout == NB && a.ld_gout == NB) {
        // the tile's rows are one contiguous block of the row-major output:
        // build it in the wave's LDS slice (each lane's RPL rows, lanes
        // padded by one double against bank conflicts), then store it
        // linearly, 64 consecutive doubles per store instruction (same wave:
        // LDS accesses complete in order, no barrier needed)
        constexpr int LR = RPL * NB, LS = LR + 1;
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) rs[lane * LS + k * NB + c] = x[k][c];
        const int total = (int)nitems * NB;
        double *dst = a.gout + cs * a.ld_gout;
        for (int e = lane; e < total; e += 64) {
            const int l = e / LR;
            dst[e] = rs[l * LS + (e - l * LR)];
        }
        return;
    }
    if (a.gout_rowmajor) {
        // rows of the lane's items are contiguous in a row-major output
        const int64_t base = cs + (int64_t)lane * RPL;
#pragma unroll
        for (int k = 0; k < RPL; ++k)
            if (ti.valid[k]) {
                double *row = a.gout + (base + k) * a.ld_gout + oc0;
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < nout) row[c] = x[k][c];
            }
        return;
    }
    // coalesced stores: per column, the lane-contiguous items go through the
    // wave's LDS slice and come back lane-strided (same wave: LDS accesses
    // complete in order, no barrier needed)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        // (a guard, not a break: a break would stop the unrolling and send x
        // to scratch memory)
        if (c < nout) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) st[lane * RPL + k] = x[k][c];
            double v[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) v[k] = st[k * 64 + lane];
            double *dst = a.gout + (int64_t)(oc0 + c) * a.ld_gout + cs;
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (k * 64 + lane < nitems) dst[k * 64 + lane] = v[k];
        }
    }
}

// g[k][c] += sum_e x[k][e] * sK[koff + e * NB + c], two rows at a time (each
// K row read serves both).
template <int NB, int RPL>
__device__ __forceinline__ void tile_times_k(const double (&x)[RPL][NB], const double *sK, int koff,
                                             double (&g)[RPL][NB]) {
    constexpr int KB = (RPL % 2 == 0) ? 2 : 1;
#pragma unroll
    for (int k0 = 0; k0 < RPL; k0 += KB) {
#pragma unroll
        for (int e = 0; e < NB; ++e) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double kv = sK[koff + e * NB + c];
#pragma unroll
                for (int q = 0; q < KB; ++q) g[k0 + q][c] = fma(x[k0 + q][e], kv, g[k0 + q][c]);
            }
        }
    }
}

// Backward of one head/tail level; see HelmertBwdArgs.  Chunks are
// independent here (no accumulation), one or more per wave.  The block of K
// that the level's rows touch is staged in LDS; the tails are recomputed
// (tile_tails) and dT = T K_blk goes through bwd_finish.
// ROWS: the output is row-major with exactly NB columns (the gradient of
// joined heads), written through a row-major tile in LDS.
// bx0: the first workgroup of this task in the launch (batched launches).
template <int NB, int RPL, int MODE, bool ROWS>
__device__ __forceinline__ void helmert_bwd_body(const HelmertBwdArgs &a, int bx0) {
    __shared__ double sK[NB * NB];   // sK[e * NB + c] = K[colmap[e]][colmap[c]], zero outside ncols
    __shared__ double stage[kWavesPerBlock * 64 * RPL];   // per-wave store staging
    __shared__ double rstage[ROWS ? kWavesPerBlock * 64 * (RPL * NB + 1) : 1];   // per-wave row-major tile
    for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) {
        const int e = i / NB, c = i % NB;
        sK[i] = (e < a.ncols && c < a.ncols) ? a.K[(int64_t)a.colmap[c] * a.n_total + a.colmap[e]] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = ((int)blockIdx.x - bx0) * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;
    const int64_t c_begin = a.nchunks * wave / a.waves;
    const int64_t c_end = a.nchunks * (wave + 1) / a.waves;
    double *st = stage + (threadIdx.x >> 6) * (64 * RPL);
    for (int64_t ch = c_begin; ch < c_end; ++ch) {
        const int64_t cs = a.chunk_start[ch], ce = a.chunk_start[ch + 1];
        double x[RPL][NB];
        TileItems<RPL> ti;
        tile_tails<NB, RPL, MODE, false>(tail_src(a), cs, ce, lane, x, ti);
        // The LDS offset is opaque to the compiler, so the reads of K are not
        // hoisted out of the chunk loop (all of K would not fit in registers).
        int koff = 0;
        asm volatile("" : "+v"(koff));
        double g[RPL][NB];
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) g[k][c] = 0.0;
        tile_times_k<NB, RPL>(x, sK, koff, g);
        bwd_finish<NB, RPL>(a, g, ti, cs, ce, lane, 0, a.ncols, st,
                            ROWS ? rstage + (threadIdx.x >> 6) * (64 * (RPL * NB + 1)) : nullptr);
    }
}

template <int NB, int RPL, int MODE, bool ROWS>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_helmert_bwd(HelmertBwdArgs a) {
    helmert_bwd_body<NB, RPL, MODE, ROWS>(a, 0);
}

// The same level of independent tasks in one launch: task t owns
// workgroups [wg0[t], wg0[t + 1]).
template <int NB, int RPL, int MODE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_helmert_bwd_multi(HelmertBwdBatch b) {
    int t = 0;
    while (t + 1 < b.count && (int)blockIdx.x >= b.wg0[t + 1]) ++t;
    helmert_bwd_body<NB, RPL, MODE, false>(b.a[t], b.wg0[t]);
}

// The same for wide levels (ncols > kChunkCols), in column chunks of
// kChunkCols: workgroup column blockIdx.y produces the gradient on output
// columns oc0 .. oc0 + 31; for every input chunk the tails are recomputed
// and multiplied by the matching block of K (all of K[:, oc0..] is staged).
template <int MODE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_helmert_bwd_wide(HelmertBwdArgs a) {
    constexpr int NB = kChunkCols, RPL = 2;
    __shared__ double sK[kMaxCols * NB];   // sK[e * NB + c] = K[colmap[e]][colmap[oc0 + c]]
    __shared__ double stage[kWavesPerBlock * 64 * RPL];
    const int oc0 = blockIdx.y * NB;
    const int nout = min(NB, a.ncols - oc0);
    for (int i = threadIdx.x; i < kMaxCols * NB; i += blockDim.x) {
        const int e = i / NB, c = i % NB;
        sK[i] = (e < a.ncols && c < nout) ? a.K[(int64_t)a.colmap[oc0 + c] * a.n_total + a.colmap[e]] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;
    const int64_t c_begin = a.nchunks * wave / a.waves;
    const int64_t c_end = a.nchunks * (wave + 1) / a.waves;
    double *st = stage + (threadIdx.x >> 6) * (64 * RPL);
    for (int64_t ch = c_begin; ch < c_end; ++ch) {
        const int64_t cs = a.chunk_start[ch], ce = a.chunk_start[ch + 1];
        double g[RPL][NB];
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) g[k][c] = 0.0;
        TileItems<RPL> ti;
        for (int ic0 = 0; ic0 < a.ncols; ic0 += NB) {
            TailSrc src = tail_src(a);
            src.in = a.in + (int64_t)ic0 * a.ld_in;
            src.ncols = min(NB, a.ncols - ic0);
            double x[RPL][NB];
            tile_tails<NB, RPL, MODE, false>(src, cs, ce, lane, x, ti);
            int koff = ic0 * NB;
            asm volatile("" : "+v"(koff));
            tile_times_k<NB, RPL>(x, sK, koff, g);
        }
        bwd_finish<NB, RPL>(a, g, ti, cs, ce, lane, oc0, nout, st);
    }
}

// Backward of process_and_join_children.  Part 0: one thread per (key
// group g, own column c), c fastest, so a wave reads whole row segments of
// the row-major ds: dOwn[c][g] = ds[g][own_pos + c] * own_mult[g].
// Part 1 + j: one thread per (group q of child j, column c): the sum over
// the parent key groups g with cidx_j[g] = q (the plan's inverse index, a
// fixed order, so the result is deterministic) of ds[g][colpos_j[c]] *
// mult_j[g].  ds is row-major, so the threads of one q read one row.  The
// parts are consecutive ranges of blocks (a one-dimensional grid).
__global__ void k_join_bwd(JoinBwdArgs a) {
    int part = 0;
    while (part <= a.nchildren && (int64_t)blockIdx.x >= a.part_block0[part + 1]) ++part;
    const int64_t idx = ((int64_t)blockIdx.x - a.part_block0[part]) * blockDim.x + threadIdx.x;
    if (part == 0) {
        if (a.own_cols <= 0) return;
        const int64_t g = idx / a.own_cols;
        const int c = (int)(idx - g * a.own_cols);
        if (g >= a.groups) return;
        a.dOwn[(int64_t)c * a.ld_own + g] = a.ds[g * a.ld_ds + a.own_pos + c] * a.own_mult[g];
        return;
    }
    const int j = part - 1;
    const int cc = a.child_cols[j];
    const int64_t q = idx / cc;
    const int c = (int)(idx - q * cc);
    if (q >= a.child_groups[j]) return;
    double sum = 0.0;
    if (a.nchunks[j] > 0) {
        // long lists: the chunks' partial sums, in chunk order
        for (int64_t k = a.chunk_off[j][q]; k < a.chunk_off[j][q + 1]; ++k) sum += a.part[j][k * cc + c];
    } else {
        const int64_t lo = a.inv_off[j][q], hi = a.inv_off[j][q + 1];
        const int col = a.colpos[j][c];
        const int32_t *inv = a.inv_idx[j];
        const double *mult = a.mult[j];
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t g = inv[i];
            sum = fma(a.ds[g * a.ld_ds + col], mult[g], sum);
        }
    }
    if (a.dsigma_rowmajor[j]) a.dsigma[j][q * a.ld_dsigma[j] + c] = sum;
    else a.dsigma[j][(int64_t)c * a.ld_dsigma[j] + q] = sum;
}

// Partial sums of child j's long inverse lists: one thread per (chunk,
// column), the chunk's kJoinChunk entries (or fewer at the end of a list)
// in list order.
__global__ void k_join_bwd_chunks(JoinBwdArgs a, int j) {
    const int cc = a.child_cols[j];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = idx / cc;
    const int c = (int)(idx - k * cc);
    if (k >= a.nchunks[j]) return;
    const int64_t q = a.chunk_q[j][k];
    const int64_t lo = a.inv_off[j][q] + (k - a.chunk_off[j][q]) * kJoinChunk;
    const int64_t hi = std::min<int64_t>(a.inv_off[j][q + 1], lo + kJoinChunk);
    const int col = a.colpos[j][c];
    const int32_t *inv = a.inv_idx[j];
    const double *mult = a.mult[j];
    double sum = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t g = inv[i];
        sum = fma(a.ds[g * a.ld_ds + col], mult[g], sum);
    }
    a.part[j][k * cc + c] = sum;
}

// Root rows h_g = s_g / sqrt(c_g): dh_g = h_g K, so ds_g[c] = (s_g . K[:, c]) / c_g.
// One thread per (root group, column c); column c of K is staged in LDS.
__global__ void k_root_bwd(RootBwdArgs a) {
    __shared__ double kc[kMaxCols];
    const int c = blockIdx.y;
    for (int e = threadIdx.x; e < a.n; e += blockDim.x) kc[e] = a.K[(int64_t)c * a.n + e];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.groups) return;
    const double f = a.inv_sqrt_c ? a.inv_sqrt_c[g] : 1.0;
    double d = 0.0;
    for (int e = 0; e < a.n; ++e) d = fma(a.s[(int64_t)e * a.ld_s + g], kc[e], d);
    if (a.ds_rowmajor) a.ds[g * a.ld_ds + c] = d * f * f;
    else a.ds[(int64_t)c * a.ld_ds + g] = d * f * f;
}

__global__ void k_copy_cols(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t rows,
                            int32_t ncols) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows) return;
    for (int c = 0; c < ncols; ++c) dst[(int64_t)c * ld_dst + t] = src[(int64_t)c * ld_src + t];
}

int nb_bwd(int ncols) {
    if (ncols <= 8) return 8;
    if (ncols <= 16) return 16;
    return 32;
}

template <int NB>
hipError_t helmert_bwd_nb(const HelmertBwdArgs &a, bool unit, hipStream_t s) {
    constexpr int RPL = (NB == 8) ? 8 : (NB == 16 ? 4 : 2);
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock), block(64 * kWavesPerBlock);
    const bool rows = a.gout_rowmajor && a.ncols == NB && a.ld_gout == NB;
    if (rows) {
        if (unit) hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 0, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 1, true>), grid, block, 0, s, a);
    } else {
        if (unit) hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 0, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 1, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t helmert_bwd_wide(const HelmertBwdArgs &a, bool unit, hipStream_t s) {
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock, (a.ncols + kChunkCols - 1) / kChunkCols);
    dim3 block(64 * kWavesPerBlock);
    if (unit) hipLaunchKernelGGL((k_helmert_bwd_wide<0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_helmert_bwd_wide<1>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_qr_adjoint(const double *R, const double *dR, int32_t n, double *K, double *W, int32_t *status,
                             hipStream_t s) {
    if (n <= kAdjSmall) hipLaunchKernelGGL(k_qr_adjoint_small, dim3(1), dim3(256), 0, s, R, dR, (int)n, K, status);
    else hipLaunchKernelGGL(k_qr_adjoint, dim3(1), dim3(256), 0, s, R, dR, (int)n, K, W, status);
    return hipGetLastError();
}

hipError_t launch_helmert_bwd(const HelmertBwdArgs &a, bool unit, hipStream_t s) {
    if (a.waves <= 0 || a.nchunks <= 0) return hipSuccess;
    if (a.ncols > kChunkCols) return helmert_bwd_wide(a, unit, s);
    switch (nb_bwd(a.ncols)) {
        case 8: return helmert_bwd_nb<8>(a, unit, s);
        case 16: return helmert_bwd_nb<16>(a, unit, s);
        default: return helmert_bwd_nb<32>(a, unit, s);
    }
}

int helmert_bwd_shape_class(int ncols) { return ncols > kChunkCols ? 0 : nb_bwd(ncols); }

template <int NB>
void helmert_bwd_batch_nb(const HelmertBwdBatch &b, bool unit, hipStream_t s) {
    constexpr int RPL = (NB == 8) ? 8 : (NB == 16 ? 4 : 2);
    const dim3 grid(b.wg0[b.count]), block(64 * kWavesPerBlock);
    if (unit) hipLaunchKernelGGL((k_helmert_bwd_multi<NB, RPL, 0>), grid, block, 0, s, b);
    else hipLaunchKernelGGL((k_helmert_bwd_multi<NB, RPL, 1>), grid, block, 0, s, b);
}

hipError_t launch_helmert_bwd_batch(const HelmertBwdBatch &b, bool unit, hipStream_t s) {
    if (b.count <= 0 || b.count > kHelmertBwdBatch || b.wg0[b.count] <= 0) return hipErrorInvalidValue;
    const int nb = helmert_bwd_shape_class(b.a[0].ncols);
    for (int t = 0; t < b.count; ++t)
        if (nb == 0 || helmert_bwd_shape_class(b.a[t].ncols) != nb || b.a[t].gout_rowmajor) return hipErrorInvalidValue;
    switch (nb) {
        case 8: helmert_bwd_batch_nb<8>(b, unit, s); break;
        case 16: helmert_bwd_batch_nb<16>(b, unit, s); break;
        default: helmert_bwd_batch_nb<32>(b, unit, s);
    }
    return hipGetLastError();
}

hipError_t launch_join_bwd(const JoinBwdArgs &a_in, hipStream_t s) {
    JoinBwdArgs a = a_in;
    const int bs = 256;
    // part p covers blocks part_block0[p] .. part_block0[p + 1] - 1
    a.part_block0[0] = 0;
    a.part_block0[1] = (a.groups * std::max(a.own_cols, 0) + bs - 1) / bs;
    for (int j = 0; j < a.nchildren; ++j)
        a.part_block0[j + 2] = a.part_block0[j + 1] + (a.child_groups[j] * a.child_cols[j] + bs - 1) / bs;
    const int64_t blocks = a.part_block0[a.nchildren + 1];
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    for (int j = 0; j < a.nchildren; ++j) {
        if (a.nchunks[j] <= 0) continue;
        const int64_t cb = (a.nchunks[j] * a.child_cols[j] + bs - 1) / bs;
        if (cb > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_join_bwd_chunks, dim3((unsigned)cb), dim3(bs), 0, s, a, j);
    }
    hipLaunchKernelGGL(k_join_bwd, dim3((unsigned)blocks), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_root_bwd(const RootBwdArgs &a, hipStream_t s) {
    if (a.groups <= 0 || a.n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_root_bwd, dim3((unsigned)((a.groups + bs - 1) / bs), (unsigned)a.n), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy_cols(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t rows,
                            int32_t ncols, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((rows + bs - 1) / bs)), dim3(bs), 0, s, src, ld_src, dst,
                       ld_dst, rows, ncols);
    return hipGetLastError();
}

}  // namespace figaro
