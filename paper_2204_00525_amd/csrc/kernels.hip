// HIP kernels for gfx950 (CDNA4, wave64).
//
//  k_helmert : segmented (generalized) head/tail of a tile of items, fused
//              with a wave-level Householder QR that accumulates the tail rows
//              into a per-wave upper-triangular R  (heads_and_tails and
//              project_away_join_attributes of Algorithm 3, and the leaf of
//              the post-processing TSQR of the section "Post-processing")
//  k_dense   : wave-level Householder TSQR step over a dense stack of rows
//              (the second post-processing step), final step sign-normalises
//  k_join    : process_and_join_children of Algorithm 3 (gather + exact
//              integer scale products)
//  k_root    : the root's Data rows (heads) appended to the stack
//  k_permute : caller order <-> plan order
//
// Storage: all matrices column-major FP64; a wave owns a tile of 64*RPL items,
// lane l holding items l*RPL .. l*RPL+RPL-1 (contiguous per lane, so a column
// load of the tile is one contiguous 64*RPL*8-byte span), and one row of the
// running R (lane l holds row l).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace figaro {
namespace {

constexpr int kWavesPerBlock = 4;

// Butterfly all-reduce: partners add the same two operands (in either order,
// which is exact), so every lane ends with the same bits; read lane 0 into
// scalar registers to make that uniformity visible to the compiler.
__device__ __forceinline__ double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return uniform(v);
}

// One Householder step per column j of the stacked matrix [R; X], where R is
// held one row per lane (lane l holds row l, lanes >= NB hold zero rows) and X
// holds RPL rows per lane.  The reflector of column j acts on the pivot row
// (row j of R, lane j), the rows of R below it and every row of X.  It is
// generated as in LAPACK's dlarfg: with p the pivot row, x the column below
// the pivot and D_k = x . B_k over the non-pivot rows,
//   beta = -sign(p_j) sqrt(p_j^2 + ||x||^2),  tau = (beta - p_j) / beta,
//   v = [1; x / (p_j - beta)],                w_k = p_k + D_k / (p_j - beta),
//   pivot row: B_jk -= tau w_k;  other rows: B_ik -= tau w_k x_i / (p_j - beta),
// and the step is skipped (H = I) when ||x|| = 0.  No quantity here can
// overflow when the column below the pivot is tiny (rank-deficient tiles).
template <int NB, int RPL>
__device__ __forceinline__ void qr_accumulate(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double d[NB];
        const bool below = lane > j;
#pragma unroll
        for (int k = j; k < NB; ++k) {
            double acc = below ? rs[j] * rs[k] : 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc = fma(x[r][j], x[r][k], acc);
            d[k] = acc;
        }
#pragma unroll
        for (int k = j; k < NB; ++k) d[k] = wave_sum(d[k]);
        double p[NB];
#pragma unroll
        for (int k = j; k < NB; ++k) p[k] = lane_value(rs[k], j);
        const double xn2 = d[j];
        if (xn2 > 0.0) {
            const double pj = p[j];
            const double nrm = sqrt(fma(pj, pj, xn2));
            const double beta = (pj >= 0.0) ? -nrm : nrm;
            const double tau = (beta - pj) / beta;
            const double scale = 1.0 / (pj - beta);
            const double ts = tau * scale;
            const double vo = below ? rs[j] : 0.0;
#pragma unroll
            for (int k = j + 1; k < NB; ++k) {
                const double w = fma(scale, d[k], p[k]);
                const double g = ts * w;
#pragma unroll
                for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, x[r][j], x[r][k]);
                rs[k] = (lane == j) ? fma(-tau, w, rs[k]) : fma(-g, vo, rs[k]);
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][j] = 0.0;
            if (lane == j) rs[j] = beta;
            else if (below) rs[j] = 0.0;
        }
    }
}

// Same step for wide tiles with a runtime column loop: the pivot column is
// always register column 0 and every step rotates the columns left by one, so
// after NB steps every column is back in place.  Columns already eliminated
// are zero on the rows the later reflectors act on and are left unchanged.
template <int NB, int RPL>
__device__ __forceinline__ void qr_accumulate_rot(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
    for (int j = 0; j < NB; ++j) {
        const bool below = lane > j;
        double d[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            double acc = below ? rs[0] * rs[k] : 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc = fma(x[r][0], x[r][k], acc);
            d[k] = wave_sum(acc);
        }
        double p[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) p[k] = lane_value(rs[k], j);
        const double xn2 = d[0];
        if (xn2 > 0.0) {
            const double pj = p[0];
            const double nrm = sqrt(fma(pj, pj, xn2));
            const double beta = (pj >= 0.0) ? -nrm : nrm;
            const double tau = (beta - pj) / beta;
            const double scale = 1.0 / (pj - beta);
            const double ts = tau * scale;
            const double vo = below ? rs[0] : 0.0;
#pragma unroll
            for (int k = 1; k < NB; ++k) {
                const double w = fma(scale, d[k], p[k]);
                const double g = ts * w;
#pragma unroll
                for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, x[r][0], x[r][k]);
                rs[k] = (lane == j) ? fma(-tau, w, rs[k]) : fma(-g, vo, rs[k]);
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][0] = 0.0;
            if (lane == j) rs[0] = beta;
            else if (below) rs[0] = 0.0;
        }
        // rotate columns left by one
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double t = x[r][0];
#pragma unroll
            for (int k = 0; k < NB - 1; ++k) x[r][k] = x[r][k + 1];
            x[r][NB - 1] = t;
        }
        const double t = rs[0];
#pragma unroll
        for (int k = 0; k < NB - 1; ++k) rs[k] = rs[k + 1];
        rs[NB - 1] = t;
    }
}

template <int NB, int RPL>
__device__ __forceinline__ void qr_step(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
    if constexpr (NB <= 32) qr_accumulate<NB, RPL>(x, rs, lane);
    else qr_accumulate_rot<NB, RPL>(x, rs, lane);
}

// Write this wave's R (rows 0..ncols-1 of the running R) into the stack,
// spreading local column c to global column colmap[c]; other columns get 0.
template <int NB>
__device__ __forceinline__ void store_r(const HelmertArgs &a, const double (&rs)[NB], int lane, int wave) {
    if (lane >= a.ncols) return;
    const int64_t row = a.stack_row0 + (int64_t)wave * a.ncols + lane;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c < a.ncols) a.stack[(int64_t)a.colmap[c] * a.ld_stack + row] = rs[c];
    for (int gc = 0; gc < a.n_total; ++gc)
        if (a.inv_colmap[gc] < 0) a.stack[(int64_t)gc * a.ld_stack + row] = 0.0;
}

// MODE 0: items count 1 each (tail coefficients from the position in the
// piece); MODE 1: explicit per-item coefficients.
template <int NB, int RPL, int MODE, bool FUSE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_helmert(HelmertArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;
    const int64_t c_begin = a.nchunks * wave / a.waves;
    const int64_t c_end = a.nchunks * (wave + 1) / a.waves;
    double rs[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rs[c] = 0.0;

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
        // piece starts: the chunk's first item, and every change of piece id
        const int32_t prev_last = __shfl_up(pid[RPL - 1], 1, 64);
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t prev = (k == 0) ? prev_last : pid[k - 1];
            first[k] = !valid[k] || (k == 0 && lane == 0) || pid[k] != prev;
        }
        bool lane_flag = false;
#pragma unroll
        for (int k = 0; k < RPL; ++k) lane_flag = lane_flag || first[k];
        // per-lane aggregate since the lane's last piece start
        double acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) s = (first[k] ? 0.0 : s) + x[k][c];
            acc[c] = s;
        }
        // segmented inclusive scan of the lane aggregates across the wave
        bool f = lane_flag;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const bool pf = __shfl_up((int)f, off, 64) != 0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double pa = __shfl_up(acc[c], off, 64);
                if (lane >= off && !f) acc[c] += pa;
            }
            if (lane >= off) f = f || pf;
        }
        // carry into this lane = inclusive value of the previous lane
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double v = __shfl_up(acc[c], 1, 64);
            acc[c] = (lane == 0) ? 0.0 : v;
        }
        // (shuffle unconditionally: a shuffle under a divergent mask would read
        // an inactive lane)
        const int nf0 = __shfl_down((int)first[0], 1, 64);
        const bool next_first0 = (lane == 63) || (nf0 != 0);
        // tails, piece sums
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int64_t t = base + k;
            double al = 0.0, be = 0.0;
            if (valid[k] && !first[k]) {
                if constexpr (MODE == 0) {
                    const double j = (double)(t - a.piece_start[pid[k]]);
                    const double q = 1.0 / sqrt(j * (j + 1.0));
                    const double phi = a.phi_piece[pid[k]];
                    al = phi * j * q;
                    be = phi * q;
                } else {
                    al = a.alpha[t];
                    be = a.beta[t];
                }
            }
            const bool last = valid[k] && ((k + 1 < RPL) ? first[k + 1] : next_first0);
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double xv = x[k][c];
                const double run = first[k] ? 0.0 : acc[c];
                x[k][c] = first[k] ? 0.0 : (al * xv - be * run);
                acc[c] = run + xv;
            }
            if (last && a.pieces_out) {
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < a.ncols) a.pieces_out[(int64_t)c * a.ld_pieces + pid[k]] = acc[c];
            }
        }
        if constexpr (FUSE) {
            qr_step<NB, RPL>(x, rs, lane);
        } else {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                if (!valid[k]) continue;
                const int64_t row = a.r0_row0 + base + k;
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < a.ncols) a.r0[(int64_t)a.colmap[c] * a.ld_r0 + row] = x[k][c];
                if (a.block_of_row) a.block_of_row[row] = a.block_id;
            }
        }
    }
    if constexpr (FUSE) store_r<NB>(a, rs, lane, wave);
}

template <int NB, int RPL>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_dense(DenseArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;
    constexpr int T = 64 * RPL;
    double rs[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rs[c] = 0.0;
    for (int64_t tile = 0; tile < a.tiles_per_wave; ++tile) {
        const int64_t base = ((int64_t)wave * a.tiles_per_wave + tile) * T + (int64_t)lane * RPL;
        double x[RPL][NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const bool live = c < a.n;
            const double *col = a.in + (int64_t)(live ? c : 0) * a.ld_in;
#pragma unroll
            for (int k = 0; k < RPL; ++k) x[k][c] = (live && base + k < a.rows) ? col[base + k] : 0.0;
        }
        qr_step<NB, RPL>(x, rs, lane);
    }
    if (lane >= a.n) return;
    if (a.waves == 1 && a.final_r) {
        double diag = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c == lane) diag = rs[c];
        const double sg = (diag < 0.0) ? -1.0 : 1.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < a.n) a.final_r[(int64_t)c * a.n + lane] = (c >= lane) ? sg * rs[c] : 0.0;
    } else {
        const int64_t row = (int64_t)wave * a.n + lane;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < a.n) a.out[(int64_t)c * a.ld_out + row] = rs[c];
    }
}

__global__ void k_join(JoinArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.groups) return;
    const double om = a.own_mult[g];
    for (int c = 0; c < a.own_cols; ++c)
        a.s[(int64_t)(a.own_pos + c) * a.ld_s + g] = a.own[(int64_t)c * a.ld_own + g] * om;
    for (int j = 0; j < a.nchildren; ++j) {
        const int64_t q = a.cidx[j][g];
        const double m = a.mult[j][g];
        const double *sg = a.sigma[j];
        const int64_t ld = a.ld_sigma[j];
        const int32_t *pos = a.colpos[j];
        for (int c = 0; c < a.child_cols[j]; ++c) a.s[(int64_t)pos[c] * a.ld_s + g] = sg[(int64_t)c * ld + q] * m;
    }
}

__global__ void k_root(RootArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.groups) return;
    const double f = a.inv_sqrt_c ? a.inv_sqrt_c[g] : 1.0;
    const int64_t row = a.row0 + g;
    for (int c = 0; c < a.n; ++c) a.dst[(int64_t)c * a.ld_dst + row] = a.s[(int64_t)c * a.ld_s + g] * f;
    if (a.block_of_row) a.block_of_row[row] = a.block_id;
}

__global__ void k_permute(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, const int64_t *perm,
                          int64_t rows, int32_t ncols, int inverse, int64_t total_rows) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!inverse) {
        if (p >= rows) return;
        const int64_t q = perm[p];
        for (int c = 0; c < ncols; ++c) dst[(int64_t)c * ld_dst + p] = src[(int64_t)c * ld_src + q];
    } else {
        if (p >= total_rows) return;
        const int64_t q = perm[p];
        for (int c = 0; c < ncols; ++c) dst[(int64_t)c * ld_dst + q] = (p < rows) ? src[(int64_t)c * ld_src + p] : 0.0;
    }
}

__global__ void k_fill(double *p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int nb_for(int ncols) {
    if (ncols <= 8) return 8;
    if (ncols <= 16) return 16;
    if (ncols <= 32) return 32;
    return 64;
}

template <int NB>
constexpr int rpl_for() {
    return NB == 8 ? 8 : (NB == 16 ? 4 : (NB == 32 ? 2 : 1));
}

template <int NB>
hipError_t helmert_nb(const HelmertArgs &a, bool unit, bool fuse, hipStream_t s) {
    constexpr int RPL = rpl_for<NB>();
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock), block(64 * kWavesPerBlock);
    if (unit) {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 0, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 0, false>), grid, block, 0, s, a);
    } else {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 1, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 1, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int NB>
hipError_t dense_nb(const DenseArgs &a, hipStream_t s) {
    constexpr int RPL = rpl_for<NB>();
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock), block(64 * kWavesPerBlock);
    hipLaunchKernelGGL((k_dense<NB, RPL>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

int tile_items_for(int ncols) {
    switch (nb_for(ncols)) {
        case 8: return 64 * rpl_for<8>();
        case 16: return 64 * rpl_for<16>();
        case 32: return 64 * rpl_for<32>();
        default: return 64 * rpl_for<64>();
    }
}

int dense_tile_rows_for(int ncols) { return tile_items_for(ncols); }

hipError_t launch_helmert(const HelmertArgs &a, bool unit, bool fuse, hipStream_t s) {
    if (a.waves <= 0 || a.nchunks <= 0) return hipSuccess;
    switch (nb_for(a.ncols)) {
        case 8: return helmert_nb<8>(a, unit, fuse, s);
        case 16: return helmert_nb<16>(a, unit, fuse, s);
        case 32: return helmert_nb<32>(a, unit, fuse, s);
        default: return helmert_nb<64>(a, unit, fuse, s);
    }
}

hipError_t launch_dense(const DenseArgs &a, hipStream_t s) {
    if (a.waves <= 0) return hipSuccess;
    switch (nb_for(a.n)) {
        case 8: return dense_nb<8>(a, s);
        case 16: return dense_nb<16>(a, s);
        case 32: return dense_nb<32>(a, s);
        default: return dense_nb<64>(a, s);
    }
}

hipError_t launch_join(const JoinArgs &a, hipStream_t s) {
    if (a.groups <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_join, dim3((unsigned)((a.groups + bs - 1) / bs)), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_root(const RootArgs &a, bool, hipStream_t s) {
    if (a.groups <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_root, dim3((unsigned)((a.groups + bs - 1) / bs)), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_permute(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, const int64_t *perm,
                          int64_t rows, int32_t ncols, bool inverse, int64_t total_rows, hipStream_t s) {
    const int64_t n = inverse ? total_rows : rows;
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, src, ld_src, dst, ld_dst,
                       perm, rows, ncols, inverse ? 1 : 0, total_rows);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int bs = 256;
    int64_t blocks = std::min<int64_t>((count + bs - 1) / bs, 8192);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(bs), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int bs = 256;
    int64_t blocks = std::min<int64_t>((count + bs - 1) / bs, 8192);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(bs), 0, s, p, count, v);
    return hipGetLastError();
}

}  // namespace figaro
