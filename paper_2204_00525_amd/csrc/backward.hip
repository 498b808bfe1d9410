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
#include "device_common.hpp"

namespace figaro {
namespace {

// K = R^{-1} Phi R^{-T} with Phi = tril(M) + tril(M,-1)^T, M = R triu(dR)^T.
// One workgroup of 64 threads, n <= 64.  Thread t owns column t.
__global__ __launch_bounds__(64) void k_qr_adjoint(const double *R, const double *dR, int n, double *K,
                                                   int32_t *status) {
    __shared__ double sR[64][65];
    __shared__ double sW[64][65];
    const int t = threadIdx.x;
    if (t < n)
        for (int c = 0; c < n; ++c) sR[t][c] = (c >= t) ? R[(int64_t)c * n + t] : 0.0;
    __syncthreads();
    // M[i][t] = sum_{k >= max(i, t)} R[i][k] dR[t][k]
    if (t < n)
        for (int i = 0; i < n; ++i) {
            double m = 0.0;
            for (int k = (i > t ? i : t); k < n; ++k) m = fma(sR[i][k], dR[(int64_t)k * n + t], m);
            sW[i][t] = m;
        }
    __syncthreads();
    // symmetrise from the lower triangle: Phi[i][t] = M[t][i] for i < t
    if (t < n)
        for (int i = 0; i < t; ++i) sW[i][t] = sW[t][i];
    __syncthreads();
    // Y = R^{-1} Phi, column t in place
    if (t < n)
        for (int i = n - 1; i >= 0; --i) {
            double y = sW[i][t];
            for (int k = i + 1; k < n; ++k) y = fma(-sR[i][k], sW[k][t], y);
            sW[i][t] = y / sR[i][i];
        }
    __syncthreads();
    // K = R^{-1} Y^T: column t solves R k = (row t of Y)
    if (t < n)
        for (int i = n - 1; i >= 0; --i) {
            double y = sW[t][i];
            for (int k = i + 1; k < n; ++k) y = fma(-sR[i][k], K[(int64_t)t * n + k], y);
            K[(int64_t)t * n + i] = y / sR[i][i];
        }
    if (t == 0) {
        int32_t singular = 0;
        for (int i = 0; i < n; ++i) singular |= (sR[i][i] == 0.0) ? 1 : 0;
        status[0] = singular;
    }
}

// Backward of one head/tail level; see HelmertBwdArgs.  Chunks are
// independent here (no accumulation), one or more per wave.
template <int NB, int RPL, int MODE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_helmert_bwd(HelmertBwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;
    const int64_t c_begin = a.nchunks * wave / a.waves;
    const int64_t c_end = a.nchunks * (wave + 1) / a.waves;
    for (int64_t ch = c_begin; ch < c_end; ++ch) {
        const int64_t cs = a.chunk_start[ch], ce = a.chunk_start[ch + 1];
        const int64_t base = cs + (int64_t)lane * RPL;
        double x[RPL][NB];
        int32_t pid[RPL];
        bool valid[RPL], first[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            valid[k] = base + k < ce;
            pid[k] = valid[k] ? a.pid[base + k] : -1;
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const bool live = c < a.ncols;
            const double *col = a.in + (int64_t)(live ? c : 0) * a.ld_in;
#pragma unroll
            for (int k = 0; k < RPL; ++k) x[k][c] = (live && valid[k]) ? col[base + k] : 0.0;
        }
        const int32_t prev_last = __shfl_up(pid[RPL - 1], 1, 64);
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t prev = (k == 0) ? prev_last : pid[k - 1];
            first[k] = !valid[k] || (k == 0 && lane == 0) || pid[k] != prev;
        }
        bool lane_flag = false;
#pragma unroll
        for (int k = 0; k < RPL; ++k) lane_flag = lane_flag || first[k];
        double acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) sum = (first[k] ? 0.0 : sum) + x[k][c];
            acc[c] = sum;
        }
        const uint64_t mask = __ballot(lane_flag);
        segmented_carry<NB>(acc, mask, lane);
        const int nf0 = __shfl_down((int)first[0], 1, 64);
        const bool next_first0 = (lane == 63) || (nf0 != 0);
        // recompute the tails (as in the forward pass)
        double al[RPL], be[RPL];
        bool last[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int64_t t = base + k;
            al[k] = 0.0;
            be[k] = 0.0;
            if (valid[k] && !first[k]) {
                if constexpr (MODE == 0) {
                    const double j = (double)(t - a.piece_start[pid[k]]);
                    const double q = 1.0 / sqrt(j * (j + 1.0));
                    const double phi = a.phi_piece[pid[k]];
                    al[k] = phi * j * q;
                    be[k] = phi * q;
                } else {
                    al[k] = a.alpha[t];
                    be[k] = a.beta[t];
                }
            }
            last[k] = valid[k] && ((k + 1 < RPL) ? first[k + 1] : next_first0);
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double xv = x[k][c];
                const double run = first[k] ? 0.0 : acc[c];
                x[k][c] = first[k] ? 0.0 : (al[k] * xv - be[k] * run);
                acc[c] = run + xv;
            }
        }
        // dT = T K_blk (the tail rows' gradient on the block's columns)
        double g[RPL][NB];
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) g[k][c] = 0.0;
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            if (e >= a.ncols) break;
            const double *Ke = a.K + (int64_t)a.colmap[e];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c >= a.ncols) break;
                const double kv = Ke[(int64_t)a.colmap[c] * a.n_total];
#pragma unroll
                for (int k = 0; k < RPL; ++k) g[k][c] = fma(x[k][e], kv, g[k][c]);
            }
        }
        // w = beta dT; reverse segmented scan: E_t = sum_{u > t in its piece} w_u
        bool stop = false, lane_last = false;
        double A[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) A[c] = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            if (!stop) {
#pragma unroll
                for (int c = 0; c < NB; ++c) A[c] = fma(be[k], g[k][c], A[c]);
            }
            stop = stop || last[k];
            lane_last = lane_last || last[k];
        }
        bool f = lane_last;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const bool pf = __shfl_down((int)f, off, 64) != 0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double pa = __shfl_down(A[c], off, 64);
                if (lane + off < 64 && !f) A[c] += pa;
            }
            if (lane + off < 64) f = f || pf;
        }
        double run[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double v = __shfl_down(A[c], 1, 64);
            run[c] = (lane == 63) ? 0.0 : v;
        }
#pragma unroll
        for (int k = RPL - 1; k >= 0; --k) {
            const int64_t t = base + k;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double E = last[k] ? 0.0 : run[c];
                const double w = be[k] * g[k][c];
                if (valid[k] && c < a.ncols)
                    a.gout[(int64_t)c * a.ld_gout + t] =
                        fma(al[k], g[k][c], -E) + a.gpieces[(int64_t)c * a.ld_gp + pid[k]];
                run[c] = w + E;
            }
        }
    }
}

__global__ void k_join_bwd(JoinBwdArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int part = blockIdx.y;
    if (part == 0) {
        if (i >= a.groups) return;
        const double om = a.own_mult[i];
        for (int c = 0; c < a.own_cols; ++c)
            a.dOwn[(int64_t)c * a.ld_own + i] = a.ds[(int64_t)(a.own_pos + c) * a.ld_ds + i] * om;
        return;
    }
    const int j = part - 1;
    if (i >= a.child_groups[j]) return;
    const int64_t lo = a.inv_off[j][i], hi = a.inv_off[j][i + 1];
    const int32_t *pos = a.colpos[j];
    for (int c = 0; c < a.child_cols[j]; ++c) {
        const double *src = a.ds + (int64_t)pos[c] * a.ld_ds;
        double sum = 0.0;
        for (int64_t q = lo; q < hi; ++q) {
            const int32_t g = a.inv_idx[j][q];
            sum = fma(src[g], a.mult[j][g], sum);
        }
        a.dsigma[j][(int64_t)c * a.ld_dsigma[j] + i] = sum;
    }
}

__global__ void k_root_bwd(RootBwdArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.groups) return;
    const double f = a.inv_sqrt_c ? a.inv_sqrt_c[g] : 1.0;
    double row[kMaxCols];
#pragma unroll
    for (int e = 0; e < kMaxCols; ++e) row[e] = (e < a.n) ? a.s[(int64_t)e * a.ld_s + g] * f : 0.0;
    for (int c = 0; c < a.n; ++c) {
        const double *Kc = a.K + (int64_t)c * a.n;
        double d = 0.0;
#pragma unroll
        for (int e = 0; e < kMaxCols; ++e)
            if (e < a.n) d = fma(row[e], Kc[e], d);
        a.ds[(int64_t)c * a.ld_ds + g] = d * f;
    }
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
    if (ncols <= 32) return 32;
    return 64;
}

template <int NB>
hipError_t helmert_bwd_nb(const HelmertBwdArgs &a, bool unit, hipStream_t s) {
    constexpr int RPL = (NB == 8) ? 8 : (NB == 16 ? 4 : (NB == 32 ? 2 : 1));
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock), block(64 * kWavesPerBlock);
    if (unit) hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_helmert_bwd<NB, RPL, 1>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_qr_adjoint(const double *R, const double *dR, int32_t n, double *K, int32_t *status,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_qr_adjoint, dim3(1), dim3(64), 0, s, R, dR, (int)n, K, status);
    return hipGetLastError();
}

hipError_t launch_helmert_bwd(const HelmertBwdArgs &a, bool unit, hipStream_t s) {
    if (a.waves <= 0 || a.nchunks <= 0) return hipSuccess;
    switch (nb_bwd(a.ncols)) {
        case 8: return helmert_bwd_nb<8>(a, unit, s);
        case 16: return helmert_bwd_nb<16>(a, unit, s);
        case 32: return helmert_bwd_nb<32>(a, unit, s);
        default: return helmert_bwd_nb<64>(a, unit, s);
    }
}

hipError_t launch_join_bwd(const JoinBwdArgs &a, hipStream_t s) {
    int64_t mx = a.groups;
    for (int j = 0; j < a.nchildren; ++j) mx = std::max(mx, a.child_groups[j]);
    if (mx <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_join_bwd, dim3((unsigned)((mx + bs - 1) / bs), 1 + a.nchildren), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_root_bwd(const RootBwdArgs &a, hipStream_t s) {
    if (a.groups <= 0) return hipSuccess;
    const int bs = 128;
    hipLaunchKernelGGL(k_root_bwd, dim3((unsigned)((a.groups + bs - 1) / bs)), dim3(bs), 0, s, a);
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
