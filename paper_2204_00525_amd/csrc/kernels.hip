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

#include <utility>

#include "internal.hpp"
#include "device_common.hpp"

namespace figaro {
namespace {

// Sum each of C per-lane values over the 64 lanes, leaving the totals in
// scalar registers.  Recursive halving: v_permlane32_swap pairs two values so
// that lanes 0-31 carry the half sums of one and lanes 32-63 of the other;
// v_permlane16_swap does the same across rows, so one register then carries
// four values, one per 16-lane row; four DPP steps finish each row, and one
// lane per row is read out.  About 7 instructions per value instead of 20.
__device__ __forceinline__ double swap32_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b),
                                                     false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ double swap16_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b),
                                                     false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ double row_sum16(double v) {
    v += dpp<0xB1>(v, 0.0);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v, 0.0);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v, 0.0);   // row_half_mirror
    v += dpp<0x140>(v, 0.0);   // row_mirror
    return v;
}

template <int C>
__device__ __forceinline__ void wave_sum_batch(double *v) {
    if constexpr (C == 1) {
        v[0] = wave_sum(v[0]);
    } else {
        constexpr int C2 = (C + 1) / 2;
        constexpr int C4 = (C2 + 1) / 2;
        double h[C2];
#pragma unroll
        for (int i = 0; i < C2; ++i) h[i] = swap32_add(v[2 * i], (2 * i + 1 < C) ? v[2 * i + 1] : 0.0);
        double q[C4];
#pragma unroll
        for (int i = 0; i < C4; ++i) q[i] = row_sum16(swap16_add(h[2 * i], (2 * i + 1 < C2) ? h[2 * i + 1] : 0.0));
        // row 0 of q[i] holds value 4i, row 1 value 4i+2, row 2 value 4i+1, row 3 value 4i+3
#pragma unroll
        for (int i = 0; i < C4; ++i) {
            v[4 * i] = lane_value(q[i], 0);
            if (4 * i + 1 < C) v[4 * i + 1] = lane_value(q[i], 32);
            if (4 * i + 2 < C) v[4 * i + 2] = lane_value(q[i], 16);
            if (4 * i + 3 < C) v[4 * i + 3] = lane_value(q[i], 48);
        }
    }
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
template <int NB, int RPL, int J>
__device__ __forceinline__ void qr_column(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
    constexpr int C = NB - J;
    double d[C];
    const bool below = lane > J;
#pragma unroll
    for (int k = J; k < NB; ++k) {
        double acc = below ? rs[J] * rs[k] : 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc = fma(x[r][J], x[r][k], acc);
        d[k - J] = acc;
    }
    wave_sum_batch<C>(d);
    double p[C];
#pragma unroll
    for (int k = J; k < NB; ++k) p[k - J] = lane_value(rs[k], J);
    const double xn2 = d[0];
    if (xn2 > 0.0) {
        const double pj = p[0];
        const double nrm = sqrt(fma(pj, pj, xn2));
        const double beta = (pj >= 0.0) ? -nrm : nrm;
        const double tau = (beta - pj) / beta;
        const double scale = 1.0 / (pj - beta);
        const double ts = tau * scale;
        const double vo = below ? rs[J] : 0.0;
#pragma unroll
        for (int k = J + 1; k < NB; ++k) {
            const double w = fma(scale, d[k - J], p[k - J]);
            const double g = ts * w;
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, x[r][J], x[r][k]);
            rs[k] = (lane == J) ? fma(-tau, w, rs[k]) : fma(-g, vo, rs[k]);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) x[r][J] = 0.0;
        if (lane == J) rs[J] = beta;
        else if (below) rs[J] = 0.0;
    }
}

template <int NB, int RPL, int... Js>
__device__ __forceinline__ void qr_columns(double (&x)[RPL][NB], double (&rs)[NB], int lane,
                                           std::integer_sequence<int, Js...>) {
    (qr_column<NB, RPL, Js>(x, rs, lane), ...);
}

template <int NB, int RPL>
__device__ __forceinline__ void qr_accumulate(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
    qr_columns<NB, RPL>(x, rs, lane, std::make_integer_sequence<int, NB>{});
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
            d[k] = acc;
        }
        wave_sum_batch<NB>(d);
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

// ROT selects the compact runtime-loop form (code size O(NB) instead of
// O(NB^2), at twice the arithmetic); wide tiles always use it.
template <int NB, int RPL, bool ROT = false>
__device__ __forceinline__ void qr_step(double (&x)[RPL][NB], double (&rs)[NB], int lane) {
    if constexpr (NB <= 32 && !ROT) qr_accumulate<NB, RPL>(x, rs, lane);
    else qr_accumulate_rot<NB, RPL>(x, rs, lane);
}

// Merging the running R factors of the waves of a workgroup into wave 0:
// the other waves write their R rows to LDS (rows padded to NB+1 doubles to
// spread LDS banks) and wave 0 folds them in as extra tiles through the same
// QR call site as the data tiles (one copy of the QR code per kernel).
template <int NB>
__device__ __forceinline__ void merge_publish(const double (&rs)[NB], int lane, int wib, double *lds) {
    if (wib > 0 && lane < NB) {
#pragma unroll
        for (int c = 0; c < NB; ++c) lds[((wib - 1) * NB + lane) * (NB + 1) + c] = rs[c];
    }
}

template <int NB, int RPL>
__device__ __forceinline__ void merge_load(double (&x)[RPL][NB], int lane, int t0, const double *lds) {
    constexpr int ROWS = (kWavesPerBlock - 1) * NB;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int r = t0 + lane * RPL + k;
#pragma unroll
        for (int c = 0; c < NB; ++c) x[k][c] = (r < ROWS) ? lds[r * (NB + 1) + c] : 0.0;
    }
}

template <int NB, int RPL>
constexpr int merge_tiles() {
    return ((kWavesPerBlock - 1) * NB + 64 * RPL - 1) / (64 * RPL);
}

template <int NB>
constexpr int merge_lds_doubles() {
    return (kWavesPerBlock - 1) * NB * (NB + 1);
}

// Write the running R (rows 0..ncols-1) of a workgroup into the stack,
// spreading local column c to global column colmap[c]; other columns get 0.
template <int NB>
__device__ __forceinline__ void store_r(const HelmertArgs &a, const double (&rs)[NB], int lane, int64_t slot) {
    if (lane >= a.ncols) return;
    const int64_t row = a.stack_row0 + slot * a.ncols + lane;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c < a.ncols) a.stack[(int64_t)a.colmap[c] * a.ld_stack + row] = rs[c];
    for (uint64_t m = a.other_cols; m; m &= m - 1)
        a.stack[(int64_t)__builtin_ctzll(m) * a.ld_stack + row] = 0.0;
}

// MODE 0: items count 1 each (tail coefficients from the position in the
// piece); MODE 1: explicit per-item coefficients.  FUSE: fold the tails into
// the running R of the wave, merge the waves of the workgroup and write one R
// per workgroup; otherwise write the tail rows to the R0 buffer.
//
// Merge protocol (FUSE): waves 1..3 publish their R to LDS after their data
// chunks and wait at the barrier; wave 0 waits at the same barrier once its
// data chunks are done and then folds the published factors in as extra
// tiles through the same QR call site.  Every wave executes exactly one
// barrier and all branches around it are uniform within a wave.
template <int NB, int RPL, int MODE, bool FUSE, int OCC, bool ROT>
__global__ __launch_bounds__(64 * kWavesPerBlock, OCC) void k_helmert(HelmertArgs a) {
    __shared__ double lds[FUSE ? merge_lds_doubles<NB>() : 1];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wave = blockIdx.x * kWavesPerBlock + wib;
    const bool active = wave < a.waves;
    if (!FUSE && !active) return;
    const int64_t c_begin = active ? a.nchunks * wave / a.waves : 0;
    const int64_t c_end = active ? a.nchunks * (wave + 1) / a.waves : 0;
    double rs[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rs[c] = 0.0;
    const int64_t n_data = c_end - c_begin;
    const int64_t n_iter = n_data + ((FUSE && wib == 0) ? merge_tiles<NB, RPL>() : 0);

    for (int64_t it = 0; it < n_iter; ++it) {
        double x[RPL][NB];
        if (FUSE && it >= n_data) {
            if (it == n_data) __syncthreads();
            merge_load<NB, RPL>(x, lane, (int)(it - n_data) * 64 * RPL, lds);
        } else {
            const int64_t ch = c_begin + it;
            const int64_t cs = a.chunk_start[ch], ce = a.chunk_start[ch + 1];
            const int64_t base = cs + (int64_t)lane * RPL;
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
                double sum = 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) sum = (first[k] ? 0.0 : sum) + x[k][c];
                acc[c] = sum;
            }
            const uint64_t mask = __ballot(lane_flag);
            segmented_carry<NB>(acc, mask, lane);
            // (shuffle unconditionally: a shuffle under a divergent mask would
            // read an inactive lane)
            const int nf0 = __shfl_down((int)first[0], 1, 64);
            const bool next_first0 = (lane == 63) || (nf0 != 0);
            // tails, piece sums
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int64_t t = base + k;
                double al = 0.0, be = 0.0;
                if constexpr (MODE == 0) {
                    if (valid[k] && !first[k]) {
                        const double j = (double)(t - a.piece_start[pid[k]]);
                        const double q = 1.0 / sqrt(j * (j + 1.0));
                        const double phi = a.phi_piece[pid[k]];
                        al = phi * j * q;
                        be = phi * q;
                    }
                } else {
                    // branch-free: every lane loads (a clamped index for
                    // items past the end), the piece start selects zero
                    const int64_t tc = valid[k] ? t : cs;
                    const double a0 = a.alpha[tc], b0 = a.beta[tc];
                    const bool use = valid[k] && !first[k];
                    al = use ? a0 : 0.0;
                    be = use ? b0 : 0.0;
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
            if constexpr (!FUSE) {
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    if (!valid[k] || !a.r0) continue;
                    const int64_t row = a.r0_row0 + base + k;
#pragma unroll
                    for (int c = 0; c < NB; ++c)
                        if (c < a.ncols) a.r0[(int64_t)a.colmap[c] * a.ld_r0 + row] = x[k][c];
                    for (uint64_t m = a.other_cols; m; m &= m - 1)
                        a.r0[(int64_t)__builtin_ctzll(m) * a.ld_r0 + row] = 0.0;
                    if (a.block_of_row) a.block_of_row[row] = a.block_id;
                }
                continue;
            }
        }
        if constexpr (FUSE) qr_step<NB, RPL, ROT>(x, rs, lane);
    }
    if constexpr (FUSE) {
        if (wib > 0) {
            merge_publish<NB>(rs, lane, wib, lds);
            __syncthreads();
        } else {
            store_r<NB>(a, rs, lane, blockIdx.x);
        }
    }
}

// Dense TSQR step: workgroup b folds rows [b*4*tpw*T, (b+1)*4*tpw*T) (T rows
// per tile, tpw tiles per wave) into one R and writes it to rows b*n..b*n+n-1
// of `out`; with a single workgroup, the sign-normalised R goes to final_r.
// Same merge protocol as k_helmert.
template <int NB, int RPL, bool ROT>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_dense(DenseArgs a) {
    __shared__ double lds[merge_lds_doubles<NB>()];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    constexpr int T = 64 * RPL;
    double rs[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rs[c] = 0.0;
    const int64_t n_data = a.tiles_per_wave;
    const int64_t n_iter = n_data + ((wib == 0) ? merge_tiles<NB, RPL>() : 0);
    for (int64_t it = 0; it < n_iter; ++it) {
        double x[RPL][NB];
        if (it >= n_data) {
            if (it == n_data) __syncthreads();
            merge_load<NB, RPL>(x, lane, (int)(it - n_data) * T, lds);
        } else {
            const int64_t base = (wave * a.tiles_per_wave + it) * T + (int64_t)lane * RPL;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool live = c < a.n;
                const double *col = a.in + (int64_t)(live ? c : 0) * a.ld_in;
#pragma unroll
                for (int k = 0; k < RPL; ++k) x[k][c] = (live && base + k < a.rows) ? col[base + k] : 0.0;
            }
        }
        qr_step<NB, RPL, ROT>(x, rs, lane);
    }
    if (wib > 0) {
        merge_publish<NB>(rs, lane, wib, lds);
        __syncthreads();
        return;
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
        const int64_t row = (int64_t)blockIdx.x * a.n + lane;
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

// Tile shapes of the head/tail + QR kernel: rows per lane (RPL), minimum
// resident waves per SIMD the register budget is built for, and the QR form
// (ROT: compact runtime column loop; otherwise fully unrolled triangular).
// variant 0: unrolled; variant 1: compact.
template <int NB, int V>
struct Shape;
template <> struct Shape<8, 0> { static constexpr int RPL = 8, OCC = 1; static constexpr bool ROT = false; };
template <> struct Shape<8, 1> { static constexpr int RPL = 8, OCC = 1; static constexpr bool ROT = true; };
template <> struct Shape<16, 0> { static constexpr int RPL = 4, OCC = 1; static constexpr bool ROT = false; };
template <> struct Shape<16, 1> { static constexpr int RPL = 4, OCC = 1; static constexpr bool ROT = true; };
template <> struct Shape<32, 0> { static constexpr int RPL = 2, OCC = 1; static constexpr bool ROT = false; };
template <> struct Shape<32, 1> { static constexpr int RPL = 2, OCC = 1; static constexpr bool ROT = true; };
template <> struct Shape<64, 0> { static constexpr int RPL = 1, OCC = 1; static constexpr bool ROT = true; };
template <> struct Shape<64, 1> { static constexpr int RPL = 1, OCC = 1; static constexpr bool ROT = true; };

template <int NB>
constexpr int rpl_for() { return Shape<NB, 0>::RPL; }

template <int NB, int V>
hipError_t helmert_nb(const HelmertArgs &a, bool unit, bool fuse, hipStream_t s) {
    constexpr int RPL = Shape<NB, V>::RPL, OCC = Shape<NB, V>::OCC;
    constexpr bool ROT = Shape<NB, V>::ROT;
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock), block(64 * kWavesPerBlock);
    if (unit) {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 0, true, OCC, ROT>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 0, false, OCC, ROT>), grid, block, 0, s, a);
    } else {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 1, true, OCC, ROT>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 1, false, OCC, ROT>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int NB, int V>
hipError_t dense_nb(const DenseArgs &a, hipStream_t s) {
    constexpr int RPL = Shape<NB, V>::RPL;
    dim3 grid(a.waves), block(64 * kWavesPerBlock);
    hipLaunchKernelGGL((k_dense<NB, RPL, Shape<NB, V>::ROT>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

int tile_items_for(int ncols, int variant) {
    const bool v1 = variant == 1;
    switch (nb_for(ncols)) {
        case 8: return 64 * (v1 ? Shape<8, 1>::RPL : Shape<8, 0>::RPL);
        case 16: return 64 * (v1 ? Shape<16, 1>::RPL : Shape<16, 0>::RPL);
        case 32: return 64 * (v1 ? Shape<32, 1>::RPL : Shape<32, 0>::RPL);
        default: return 64 * (v1 ? Shape<64, 1>::RPL : Shape<64, 0>::RPL);
    }
}

int dense_tile_rows_for(int ncols) { return tile_items_for(ncols, 0); }
int waves_per_block() { return kWavesPerBlock; }

hipError_t launch_helmert(const HelmertArgs &a, bool unit, bool fuse, int variant, hipStream_t s) {
    if (a.waves <= 0 || a.nchunks <= 0) return hipSuccess;
    const bool v1 = variant == 1;
    switch (nb_for(a.ncols)) {
        case 8: return v1 ? helmert_nb<8, 1>(a, unit, fuse, s) : helmert_nb<8, 0>(a, unit, fuse, s);
        case 16: return v1 ? helmert_nb<16, 1>(a, unit, fuse, s) : helmert_nb<16, 0>(a, unit, fuse, s);
        case 32: return v1 ? helmert_nb<32, 1>(a, unit, fuse, s) : helmert_nb<32, 0>(a, unit, fuse, s);
        default: return helmert_nb<64, 0>(a, unit, fuse, s);
    }
}

hipError_t launch_dense(const DenseArgs &a, int variant, hipStream_t s) {
    if (a.waves <= 0) return hipSuccess;
    const bool v1 = variant == 1;
    switch (nb_for(a.n)) {
        case 8: return v1 ? dense_nb<8, 1>(a, s) : dense_nb<8, 0>(a, s);
        case 16: return v1 ? dense_nb<16, 1>(a, s) : dense_nb<16, 0>(a, s);
        case 32: return v1 ? dense_nb<32, 1>(a, s) : dense_nb<32, 0>(a, s);
        default: return dense_nb<64, 0>(a, s);
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
