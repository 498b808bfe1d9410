// HIP kernels for gfx950 (CDNA4, wave64).
//
//  k_helmert : segmented (generalized) head/tail of a tile of items, fused
//              with a wave-level Householder QR that accumulates the tail rows
//              into a per-wave upper-triangular R  (heads_and_tails and
//              project_away_join_attributes of Algorithm 3, and the leaf of
//              the post-processing TSQR of the section "Post-processing")
//  k_dense   : wave-level Householder TSQR step over a dense stack of rows
//              (the second post-processing step, n <= 16), final step
//              sign-normalises
//  k_dense_coop : the same step for n > 16, the waves of a workgroup sharing
//              each tile by column blocks
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
#include "tails.hpp"

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

// Same reduction, leaving every total in every lane (vector registers):
// after the row sums, register q holds the four totals of a group in its four
// 16-lane rows; a permlane16 swap of q with itself spreads them to lane
// halves, and a permlane32 swap of each half with itself to the whole wave.
__device__ __forceinline__ void spread4(double q, double &a, double &b, double &c, double &d) {
    // rows of q: [a, c, b, d]
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(q), (unsigned)__double2loint(q),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(q), (unsigned)__double2hiint(q),
                                                     false, false);
    // lo[0]/hi[0] rows: [a, a, b, b]; lo[1]/hi[1] rows: [c, c, d, d]
    const auto l0 = __builtin_amdgcn_permlane32_swap(lo[0], lo[0], false, false);
    const auto h0 = __builtin_amdgcn_permlane32_swap(hi[0], hi[0], false, false);
    const auto l1 = __builtin_amdgcn_permlane32_swap(lo[1], lo[1], false, false);
    const auto h1 = __builtin_amdgcn_permlane32_swap(hi[1], hi[1], false, false);
    // permlane32 swap of r with itself: [0] = its lower half everywhere, [1] = its upper half
    a = __hiloint2double((int)h0[0], (int)l0[0]);
    b = __hiloint2double((int)h0[1], (int)l0[1]);
    c = __hiloint2double((int)h1[0], (int)l1[0]);
    d = __hiloint2double((int)h1[1], (int)l1[1]);
}

template <int C>
__device__ __forceinline__ void wave_sum_batch(double *v) {
    constexpr int C2 = (C + 1) / 2;
    constexpr int C4 = (C2 + 1) / 2;
    double h[C2];
#pragma unroll
    for (int i = 0; i < C2; ++i) h[i] = swap32_add(v[2 * i], (2 * i + 1 < C) ? v[2 * i + 1] : 0.0);
#pragma unroll
    for (int i = 0; i < C4; ++i) {
        const double q = row_sum16(swap16_add(h[2 * i], (2 * i + 1 < C2) ? h[2 * i + 1] : 0.0));
        double t0, t1, t2, t3;
        spread4(q, t0, t1, t2, t3);
        v[4 * i] = t0;
        if (4 * i + 1 < C) v[4 * i + 1] = t1;
        if (4 * i + 2 < C) v[4 * i + 2] = t2;
        if (4 * i + 3 < C) v[4 * i + 3] = t3;
    }
}

// Reciprocal by the hardware estimate refined with two Newton iterations
// (r <- r + r (1 - x r)); x is a normal number here.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Reciprocal square root by the hardware estimate refined with two Newton
// iterations (y <- y + y (1/2 - (s/2) y^2)); s is a positive normal number.
__device__ __forceinline__ double rsqrt_refined(double s) {
    double y = __builtin_amdgcn_rsq(s);
    const double h = 0.5 * s;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

// Householder reflector of one column of [R; X] (LAPACK dlarfg form): with p
// the pivot R_jj and x2 = ||X_j||^2 > 0,
//   beta = -sign(p) sqrt(p^2 + x2),  tau = (beta - p) / beta,  scale = 1 / (p - beta),
// so that v = [1; X_j * scale] and H = I - tau v v^T.  For x2 = 0 the
// reflector is the identity (tau = 0) and R_jj stays p.  Branch-free.  One
// reciprocal square root gives both |beta| = s / sqrt(s) and 1 / beta.
struct Reflector {
    double tau, scale, ts, rjj;
};

__device__ __forceinline__ Reflector reflector(double p, double x2) {
    // act = 1 for x2 > 0, else 0; every quantity it multiplies is finite, so
    // multiplying by it replaces the selects
    const double act = (x2 > 0.0) ? 1.0 : 0.0;
    // (exact: one of the two terms of each sum is zero)
    const double off = 1.0 - act;
    const double s = fma(act, fma(p, p, x2), off);   // p^2 + x2, or 1
    const double r = rsqrt_refined(s);
    const double nrm = s * r;
    const double beta = (p >= 0.0) ? -nrm : nrm;
    const double inv_b = (p >= 0.0) ? -r : r;        // 1 / beta
    const double den = fma(act, p - beta, off);      // p - beta (|p - beta| >= nrm), or 1
    Reflector h;
    h.scale = recip(den);
    h.tau = -act * den * inv_b;                      // (beta - p) / beta, or 0
    h.ts = -act * inv_b;                             // tau * scale, or 0
    h.rjj = fma(act, beta, off * p);                 // beta, or p
    return h;
}

// One Householder step per column J of the stacked matrix [R; X]: R (NB x NB
// upper triangular, row-major in the wave's LDS slice) on top of the tile X
// (RPL rows per lane).  Because R is triangular, the reflector of column J
// touches only row J of R and the rows of X: with D_k = X_J . X_k and p the
// old row J,
//   w_k = p_k + scale D_k,   X_k -= tau scale w_k X_J,   R_Jk = p_k - tau w_k,
// and R_JJ = beta.  Row J is read once and written once per tile; every lane
// reads and writes the same LDS words (broadcast).
template <int NB, int RPL, int J>
__device__ __forceinline__ void qr_column(double (&x)[RPL][NB], double *rw) {
    constexpr int C = NB - J;
    double d[C];
#pragma unroll
    for (int k = J; k < NB; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc = fma(x[r][J], x[r][k], acc);
        d[k - J] = acc;
    }
    double p[C];
#pragma unroll
    for (int k = J; k < NB; ++k) p[k - J] = rw[J * NB + k];
    wave_sum_batch<C>(d);
    const Reflector h = reflector(p[0], d[0]);
#pragma unroll
    for (int k = J + 1; k < NB; ++k) {
        const double w = fma(h.scale, d[k - J], p[k - J]);
        const double g = h.ts * w;
#pragma unroll
        for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, x[r][J], x[r][k]);
        rw[J * NB + k] = fma(-h.tau, w, p[k - J]);
    }
    rw[J * NB + J] = h.rjj;
#pragma unroll
    for (int r = 0; r < RPL; ++r) x[r][J] = 0.0;
}

template <int NB, int RPL, int... Js>
__device__ __forceinline__ void qr_columns(double (&x)[RPL][NB], double *rw, std::integer_sequence<int, Js...>) {
    (qr_column<NB, RPL, Js>(x, rw), ...);
}

// Same step for wide tiles with a runtime column loop over the `ncols` live
// columns: the pivot column is always register column 0 and every step
// rotates the register columns left by one, so at step j register column k
// holds column j + k.  Register columns that wrap around hold eliminated
// (zero) columns, and their updates are the identity; their R entries go to
// a spare row at the end of the slice, which keeps the step branch-free.
// The columns of the tile end up rotated, which is harmless: the tile is
// discarded and R lives in LDS in its own column order.
template <int NB, int RPL>
__device__ __forceinline__ void qr_accumulate_rot(double (&x)[RPL][NB], double *rw, int ncols) {
    for (int j = 0; j < ncols; ++j) {
        double d[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc = fma(x[r][0], x[r][k], acc);
            d[k] = acc;
        }
        double p[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const bool live = k < NB - j;
            const double v = rw[live ? j * NB + j + k : NB * NB + k];
            p[k] = live ? v : 0.0;
        }
        wave_sum_batch<NB>(d);
        const Reflector h = reflector(p[0], d[0]);
#pragma unroll
        for (int k = 1; k < NB; ++k) {
            const double w = fma(h.scale, d[k], p[k]);
            const double g = h.ts * w;
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, x[r][0], x[r][k]);
            rw[(k < NB - j) ? j * NB + j + k : NB * NB + k] = fma(-h.tau, w, p[k]);
        }
        rw[j * NB + j] = h.rjj;
        // rotate columns left by one (column j is zero now)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
#pragma unroll
            for (int k = 0; k < NB - 1; ++k) x[r][k] = x[r][k + 1];
            x[r][NB - 1] = 0.0;
        }
    }
}

// ROT selects the compact runtime-loop form (code size O(NB) instead of
// O(NB^2)); the widest tiles always use it.
template <int NB, int RPL, bool ROT = false>
__device__ __forceinline__ void qr_step(double (&x)[RPL][NB], double *rw, int ncols) {
    if constexpr (NB <= 40 && !ROT) qr_columns<NB, RPL>(x, rw, std::make_integer_sequence<int, NB>{});
    else qr_accumulate_rot<NB, RPL>(x, rw, ncols);
}

// Blocked step for tiles of 32 columns (compact WY form): the first 16
// columns of [R; X] are factored column by column as above, keeping the tile
// part y_J = scale * X_J of every Householder vector v_J = [e_J; y_J] in
// place of the eliminated column; the 16 reflectors then reach the trailing
// 16 columns at once, and the last 16 columns are factored column by column.
// With Y the 16 vectors' tile parts, X the trailing tile columns and R' the
// trailing part of R's first 16 rows, the products G = Y^T Y and W = Y^T X
// are sums over the tile's rows, which the matrix cores form with
// v_mfma_f64_16x16x4f64 instead of one cross-lane reduction per entry.
// Applying H_0, ..., H_15 in turn then needs, for the reflector J,
//   z_J = R'_J + W_J - sum_{i<J} G_Ji zh_i,   zh_J = tau_J z_J,
// (v_J^T of the trailing columns after H_0..H_{J-1}; v_i^T v_J = G_iJ for
// i != J), after which R'_J -= zh_J and X -= Y Zh.  This is the forward
// compact WY update Q^T C = C - V T^T V^T C with the triangular factor T
// applied by substitution.
//
// Operand layouts of v_mfma_f64_16x16x4f64 (D = A B + C; lane l, register r):
// A[l % 16][l / 16], B[l / 16][l % 16], D[4 r + l / 16][l % 16].  Both
// products take A[m][k] = Y[row k][m]; B[k][n] = Y[row k][n] or X[row k][n],
// so a lane needs column l % 16 of rows that depend on l / 16 only.  The
// tile's rows are moved there through the wave's LDS area, 64 rows (one per
// lane) at a time: row k of lane L's registers is written as row L of a
// column-major 64-row block, and lane (g, c) reads rows 16 g .. 16 g + 15 of
// column c (the sums run over all rows, so any row order will do).
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));
constexpr int kPanelCols = 16;
constexpr int kWyLd = 66;                                  // padded column stride of the 64-row block
constexpr int kWyScratch = 2 * kPanelCols * kWyLd + kPanelCols;   // block (reused for G, W, Zh) + tau

template <int RPL, int J>
__device__ __forceinline__ void wy_panel_column(double (&x)[RPL][32], double *rw, double *tau, int lane) {
    constexpr int NB = 32, C = kPanelCols - J;
    double d[C], p[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc = fma(x[r][J], x[r][J + k], acc);
        d[k] = acc;
        p[k] = rw[J * NB + J + k];
    }
    wave_sum_batch<C>(d);
    const Reflector h = reflector(p[0], d[0]);
#pragma unroll
    for (int k = 1; k < C; ++k) {
        const double w = fma(h.scale, d[k], p[k]);
        const double g = h.ts * w;
#pragma unroll
        for (int r = 0; r < RPL; ++r) x[r][J + k] = fma(-g, x[r][J], x[r][J + k]);
        rw[J * NB + J + k] = fma(-h.tau, w, p[k]);
    }
    rw[J * NB + J] = h.rjj;
#pragma unroll
    for (int r = 0; r < RPL; ++r) x[r][J] *= h.scale;
    if (lane == 0) tau[J] = h.tau;
}

template <int RPL, int... Js>
__device__ __forceinline__ void wy_panel(double (&x)[RPL][32], double *rw, double *tau, int lane,
                                         std::integer_sequence<int, Js...>) {
    (wy_panel_column<RPL, Js>(x, rw, tau, lane), ...);
}

template <int RPL, int... Js>
__device__ __forceinline__ void wy_tail_columns(double (&x)[RPL][32], double *rw, std::integer_sequence<int, Js...>) {
    (qr_column<32, RPL, kPanelCols + Js>(x, rw), ...);
}

template <int RPL>
__device__ __forceinline__ void qr_step_wy32(double (&x)[RPL][32], double *rw, double *sc, int lane) {
    constexpr int NB = 32, P = kPanelCols, LD = kWyLd;
    double *tb = sc;                       // [32][LD]: the 64-row block
    double *tau = sc + 2 * P * LD;         // [16]
    wy_panel<RPL>(x, rw, tau, lane, std::make_integer_sequence<int, P>{});
    // G = Y^T Y and W = Y^T X on the matrix cores
    const int g = lane >> 4, c = lane & 15;
    mfma_f64x4 accG = {0.0, 0.0, 0.0, 0.0}, accW = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
#pragma unroll
        for (int col = 0; col < NB; ++col) tb[col * LD + lane] = x[k][col];
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
            const double2 y2 = *reinterpret_cast<const double2 *>(tb + c * LD + 16 * g + q);
            const double2 x2 = *reinterpret_cast<const double2 *>(tb + (P + c) * LD + 16 * g + q);
            accG = __builtin_amdgcn_mfma_f64_16x16x4f64(y2.x, y2.x, accG, 0, 0, 0);
            accW = __builtin_amdgcn_mfma_f64_16x16x4f64(y2.x, x2.x, accW, 0, 0, 0);
            accG = __builtin_amdgcn_mfma_f64_16x16x4f64(y2.y, y2.y, accG, 0, 0, 0);
            accW = __builtin_amdgcn_mfma_f64_16x16x4f64(y2.y, x2.y, accW, 0, 0, 0);
        }
    }
    // G and W row-major [16][16] (over the block, whose reads are done)
    double *G = tb, *W = tb + P * P, *Zh = tb + 2 * P * P;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        G[(4 * r + g) * P + c] = accG[r];
        W[(4 * r + g) * P + c] = accW[r];
    }
    // the reflectors in turn on column c of the trailing block (the four
    // lanes of a column compute the same values; one of them stores)
    double zh[P];
#pragma unroll
    for (int J = 0; J < P; ++J) {
        const double rjc = rw[J * NB + P + c];
        double z = rjc + W[J * P + c];
#pragma unroll
        for (int i = 0; i < J; ++i) z = fma(-G[J * P + i], zh[i], z);
        zh[J] = tau[J] * z;
        if (lane < P) {
            rw[J * NB + P + c] = rjc - zh[J];
            Zh[J * P + c] = zh[J];
        }
    }
    // X -= Y Zh on the tile's rows
#pragma unroll
    for (int J = 0; J < P; ++J) {
#pragma unroll
        for (int n = 0; n < P; ++n) {
            const double zv = Zh[J * P + n];
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][P + n] = fma(-x[r][J], zv, x[r][P + n]);
        }
    }
    wy_tail_columns<RPL>(x, rw, std::make_integer_sequence<int, NB - P>{});
}

// Whether the head/tail kernel of this shape uses the blocked step (32
// columns, fully unrolled, one wave per SIMD: the LDS then holds the 64-row
// blocks of all four waves).
template <int NB, bool ROT, int OCC>
constexpr bool use_wy() {
    return NB == 32 && !ROT && OCC == 1;
}

// Each wave keeps its running R in its own LDS slice (NB x NB doubles,
// row-major, zero below the diagonal; the compact form adds a spare row).
// Merging the waves of a workgroup: after a barrier, wave 0 folds the R
// factors of waves 1..3 in as extra tiles through the same QR call site as
// the data tiles.
template <int NB, bool ROT>
constexpr int r_slice_doubles() {
    return NB * NB + (ROT ? NB : 0);
}

template <int NB, bool ROT>
__device__ __forceinline__ void r_zero(double *rw, int lane) {
    for (int i = lane; i < r_slice_doubles<NB, ROT>(); i += 64) rw[i] = 0.0;
}

template <int NB, int RPL, bool ROT>
__device__ __forceinline__ void merge_load(double (&x)[RPL][NB], int lane, int t0, const double *lds) {
    constexpr int ROWS = (kWavesPerBlock - 1) * NB;
    constexpr int SL = r_slice_doubles<NB, ROT>();
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int r = t0 + lane * RPL + k;
        // row r of the merge block: row r % NB of wave 1 + r / NB
        const int src = (r < ROWS) ? ((1 + r / NB) * SL + (r % NB) * NB) : 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) x[k][c] = (r < ROWS) ? lds[src + c] : 0.0;
    }
}

template <int NB, int RPL>
constexpr int merge_tiles() {
    return ((kWavesPerBlock - 1) * NB + 64 * RPL - 1) / (64 * RPL);
}

// Write the R (rows 0..ncols-1) of a workgroup into the stack, spreading
// local column c to global column colmap[c]; other columns get 0.
template <int NB>
__device__ __forceinline__ void store_r(const HelmertArgs &a, const double *rw, int lane, int64_t slot) {
    if (lane >= a.ncols) return;
    const int64_t row = a.stack_row0 + slot * a.ncols + lane;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c < a.ncols) a.stack[(int64_t)a.colmap[c] * a.ld_stack + row] = rw[lane * NB + c];
    for (int h = 0; h < 2; ++h)
        for (uint64_t m = a.other_cols[h]; m; m &= m - 1)
            a.stack[(int64_t)(64 * h + __builtin_ctzll(m)) * a.ld_stack + row] = 0.0;
}

// Whether the fused kernel of this shape stages its next tile in LDS: the
// staging areas and R slices of the OCC workgroups a CU is meant to hold
// must fit its 160 KiB of LDS.
template <int NB, int RPL, bool ROT, int OCC>
constexpr bool stage_fits() {
    return OCC * kWavesPerBlock * 8 * (Stage<NB, RPL>::doubles + r_slice_doubles<NB, ROT>()) <= 160 * 1024;
}

// MODE 0: items count 1 each (tail coefficients from the position in the
// piece); MODE 1: explicit per-item coefficients.  JOIN: the items are the
// joined heads, read in place through a.js (the first level of
// project_away_join_attributes fused with process_and_join_children).  FUSE: fold the tails into
// the running R of the wave, merge the waves of the workgroup and write one R
// per workgroup; otherwise write the tail rows to the R0 buffer.
//
// Merge protocol (FUSE): each wave accumulates into its own LDS slice; waves
// 1..3 wait at the barrier after their data chunks; wave 0 waits at the same
// barrier once its data chunks are done and then folds the other slices in
// as extra tiles through the same QR call site.  Every wave executes exactly
// one barrier and all branches around it are uniform within a wave.
//
// Staging (FUSE, where it fits): the asynchronous copies of the next chunk
// are issued after the current chunk has been read from the staging area and
// before its tails and QR are computed; they land while the QR runs.
// bx0: the first workgroup of this task in the launch (batched launches).
template <int NB, int RPL, int MODE, bool FUSE, int OCC, bool ROT, bool JOIN>
__device__ __forceinline__ void helmert_body(const HelmertArgs &a, int bx0) {
    // the compact QR's column loop reads R through loop-carried LDS addresses
    // the compiler cannot tell apart from the staging area, so it would wait
    // for the copies at its first column: no staging there
    constexpr bool STAGE = FUSE && !ROT && !JOIN && stage_fits<NB, RPL, ROT, OCC>();
    using S = Stage<NB, RPL>;
    __shared__ double lds[FUSE ? kWavesPerBlock * r_slice_doubles<NB, ROT>() : 1];
    __shared__ double stage_lds[STAGE ? kWavesPerBlock * S::doubles : 1];
    __shared__ int32_t prefetch_sink[JOIN ? 64 : 1];
    constexpr bool WY = FUSE && use_wy<NB, ROT, OCC>();
    __shared__ double wy_lds[WY ? kWavesPerBlock * kWyScratch : 1];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int wave = ((int)blockIdx.x - bx0) * kWavesPerBlock + wib;
    const bool active = wave < a.waves;
    if (!FUSE && !active) return;
    const int64_t c_begin = active ? a.nchunks * wave / a.waves : 0;
    const int64_t c_end = active ? a.nchunks * (wave + 1) / a.waves : 0;
    double *rw = lds + (FUSE ? wib * r_slice_doubles<NB, ROT>() : 0);
    if constexpr (FUSE) r_zero<NB, ROT>(rw, lane);
    const int64_t n_data = c_end - c_begin;
    const int64_t n_iter = n_data + ((FUSE && wib == 0) ? merge_tiles<NB, RPL>() : 0);
    TailSrc src = tail_src(a);
    src.pieces_out = a.pieces_out;
    src.ld_pieces = a.ld_pieces;
    // column chunk of a wide task: task columns c0 .. c0 + NB - 1
    int c0 = 0, join_col0 = a.join_col0;
    if constexpr (!FUSE) {
        if (a.wide_cols > 0) {
            c0 = (int)blockIdx.y * NB;
            src.ncols = min(NB, a.wide_cols - c0);
            if (src.in) src.in += (int64_t)c0 * a.ld_in;
            if (src.pieces_out) src.pieces_out += (int64_t)c0 * a.ld_pieces;
            join_col0 += c0;
        }
    }

    // chunk boundaries (and first pieces) of chunks wbase .. wbase + 63, one
    // per lane, read out with readlane: no wait on a global load between
    // tiles except when the window moves on
    int64_t wbase = c_begin, w_cs = 0;
    int32_t w_p0 = 0;
    auto window = [&](int64_t first) {
        wbase = first;
        const int64_t i = (first + lane < a.nchunks) ? first + lane : a.nchunks;
        w_cs = a.chunk_start[i];
        w_p0 = a.chunk_piece0[i];
    };
    auto bounds = [&](int64_t ch, int64_t &cs, int64_t &ce) {
        if (ch + 2 - wbase > 63) window(ch);
        const int i = (int)(ch - wbase);
        cs = readlane64(w_cs, i);
        ce = readlane64(w_cs, i + 1);
    };
    window(c_begin);

    // staging: chunk c_begin + it + 1 is copied while chunk c_begin + it is
    // worked on (full chunks with 16-byte aligned columns only).  The first
    // chunk is read directly: a copy issued before the loop makes the
    // compiler wait for it before every LDS read of the loop.
    double *st = stage_lds + (STAGE ? wib * S::doubles : 0);
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.in) & 15) == 0) && ((a.ld_in & 1) == 0);
    bool staged = false;
    int32_t staged_p0 = 0;
    auto issue = [&](int64_t ch) {
        int64_t cs, ce;
        bounds(ch, cs, ce);
        staged = aligned && ce - cs == S::T && (cs & 1) == 0;
        if (staged) {
            const int i = (int)(ch - wbase);
            staged_p0 = MODE == 0 ? (__builtin_amdgcn_readlane(w_p0, i) & ~1) : 0;
            const int32_t p1 = MODE == 0 ? __builtin_amdgcn_readlane(w_p0, i + 1) : 0;
            stage_issue<NB, RPL, MODE>(src, cs, staged_p0, p1, st, lane);
        }
    };
    for (int64_t it = 0; it < n_iter; ++it) {
        double x[RPL][NB];
        if (FUSE && it >= n_data) {
            if (it == n_data) __syncthreads();
            merge_load<NB, RPL, ROT>(x, lane, (int)(it - n_data) * 64 * RPL, lds);
        } else {
            const int64_t ch = c_begin + it;
            int64_t cs, ce;
            bounds(ch, cs, ce);
            TileItems<RPL> ti;
            TileCoef<RPL> cf;
            if (STAGE && staged) {
                // the copies have landed; read them, and finish reading
                // before the area is refilled
                __builtin_amdgcn_s_waitcnt(kWaitVm0);
                stage_read<NB, RPL, MODE>(src, cs, staged_p0, st, lane, x, ti, cf);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            } else {
                if constexpr (FUSE) tile_load<NB, RPL, MODE, JOIN>(src, cs, ce, lane, x, ti, cf, &a.js, a.join_col0);
                else tile_load<NB, RPL, MODE, JOIN>(src, cs, ce, lane, x, ti, cf, &a.js, join_col0);
                if constexpr (JOIN && FUSE) {
                    if (it + 1 < n_data) {
                        int64_t ncs, nce;
                        bounds(ch + 1, ncs, nce);
                        join_prefetch<RPL>(a.js, ncs, nce, lane, prefetch_sink);
                    }
                }
                // nothing of this chunk may stay in flight past the next
                // chunk's copies (the compiler would then wait for those too)
                if constexpr (STAGE) __builtin_amdgcn_s_waitcnt(kWaitVm0);
            }
            if constexpr (STAGE) {
                staged = false;
                if (it + 1 < n_data) issue(ch + 1);
            }
            tile_finish<NB, RPL, MODE, true>(src, cs, lane, x, ti, cf);
            if constexpr (!FUSE) {
                const int64_t base = cs + (int64_t)lane * RPL;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    if (!ti.valid[k] || !a.r0) continue;
                    const int64_t row = a.r0_row0 + base + k;
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        if (c >= src.ncols) continue;
                        const int oc = a.wide_cols == 0 ? a.colmap[c]
                                       : a.cols_ident ? c0 + c : a.wide_colmap[c0 + c];
                        a.r0[(int64_t)oc * a.ld_r0 + row] = x[k][c];
                    }
                    // the columns outside the task: zeros, written by the
                    // first chunk
                    if (c0 == 0)
                        for (int h = 0; h < 2; ++h)
                            for (uint64_t m = a.other_cols[h]; m; m &= m - 1)
                                a.r0[(int64_t)(64 * h + __builtin_ctzll(m)) * a.ld_r0 + row] = 0.0;
                    if (a.block_of_row) a.block_of_row[row] = a.block_id;
                }
                continue;
            }
        }
        if constexpr (WY) {
            if constexpr (NB == 32) qr_step_wy32<RPL>(x, rw, wy_lds + wib * kWyScratch, lane);
        } else if constexpr (FUSE) {
            qr_step<NB, RPL, ROT>(x, rw, a.ncols);
        }
    }
    if constexpr (FUSE) {
        if (wib > 0) __syncthreads();
        else store_r<NB>(a, rw, lane, (int)blockIdx.x - bx0);
    }
}

template <int NB, int RPL, int MODE, bool FUSE, int OCC, bool ROT, bool JOIN>
__global__ __launch_bounds__(64 * kWavesPerBlock, OCC) void k_helmert(HelmertArgs a) {
    helmert_body<NB, RPL, MODE, FUSE, OCC, ROT, JOIN>(a, 0);
}

// The same level of independent tasks in one launch: task t owns
// workgroups [wg0[t], wg0[t + 1]).  Upper levels are small and bound by
// latency, so tasks side by side share it; first levels that each fill the
// chip overlap one task's last tiles with the next one's first.
template <int NB, int RPL, int MODE, bool FUSE, int OCC, bool ROT>
__global__ __launch_bounds__(64 * kWavesPerBlock, OCC) void k_helmert_multi(HelmertBatch b) {
    int t = 0;
    while (t + 1 < b.count && (int)blockIdx.x >= b.wg0[t + 1]) ++t;
    helmert_body<NB, RPL, MODE, FUSE, OCC, ROT, false>(b.a[t], b.wg0[t]);
}

// Dense TSQR step: workgroup b folds rows [b*4*tpw*T, (b+1)*4*tpw*T) (T rows
// per tile, tpw tiles per wave) into one R and writes it to rows b*n..b*n+n-1
// of `out`; with a single workgroup, the sign-normalised R goes to final_r.
// Same merge protocol as k_helmert.
template <int NB, int RPL, bool ROT, int OCC>
__global__ __launch_bounds__(64 * kWavesPerBlock, OCC) void k_dense(DenseArgs a) {
    __shared__ double lds[kWavesPerBlock * r_slice_doubles<NB, ROT>()];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wib;
    constexpr int T = 64 * RPL;
    double *rw = lds + wib * r_slice_doubles<NB, ROT>();
    r_zero<NB, ROT>(rw, lane);
    const int64_t n_data = a.tiles_per_wave;
    // only wave 0 of the workgroup has rows: nothing to merge (it still
    // meets the others at the one barrier, after its tiles)
    const bool merge = a.rows - (int64_t)blockIdx.x * kWavesPerBlock * a.tiles_per_wave * T > a.tiles_per_wave * T;
    const int64_t n_iter = n_data + ((wib == 0 && merge) ? merge_tiles<NB, RPL>() : 0);
    for (int64_t it = 0; it < n_iter; ++it) {
        double x[RPL][NB];
        if (it >= n_data) {
            if (it == n_data) __syncthreads();
            merge_load<NB, RPL, ROT>(x, lane, (int)(it - n_data) * T, lds);
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
        qr_step<NB, RPL, ROT>(x, rw, a.n);
    }
    if (wib > 0 || !merge) __syncthreads();
    if (wib > 0) return;
    if (lane >= a.n) return;
    if (a.waves == 1 && a.final_r) {
        const double sg = (rw[lane * NB + lane] < 0.0) ? -1.0 : 1.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < a.n) a.final_r[(int64_t)c * a.n + lane] = (c >= lane) ? sg * rw[lane * NB + c] : 0.0;
    } else {
        const int64_t row = (int64_t)blockIdx.x * a.n + lane;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < a.n) a.out[(int64_t)c * a.ld_out + row] = rw[lane * NB + c];
    }
}

// Cooperative dense TSQR step (n > 16): the W waves of a workgroup share
// each tile of 64 coop_rpl(CW) rows; wave w holds columns [CW w, CW w + CW)
// of the tile (coop_rpl(CW) rows per lane) and the same columns of the workgroup's R
// (all n rows, row-major, in its LDS slice).  CW is 4 for n <= 32 (W = 6 or
// 8), 8 for n <= 64 (W = 5 up to 40 columns, 8 above) and 16 up to 128
// (W = 8).  At the step of column j the wave that owns j forms the
// reflector from its own column (the column loop is unrolled within the
// block, so the owner works on the columns it still holds in place) and
// publishes the column and the reflector's scalars through LDS; after one
// barrier the waves to its right apply the reflector to their
// columns (and their part of row j of R).  The scalars and the column are
// double-buffered by the parity of a column step count that runs on across
// tiles, so one barrier per column suffices.  Sharing the tile
// spreads each column's cross-lane reductions over the waves, so a tile
// step takes the latency of one column's reflector per column instead of
// that of all its reductions.  Every wave runs the same number of steps and
// barriers.  Workgroup b folds rows [b W', (b+1) W'), W' = tiles_per_wave *
// 64 coop_rpl(CW) rows, into one R; the single workgroup of the last level
// sign-normalises it.
constexpr int kNarrowCols = 8;
constexpr int kMidCols = 16;
// rows per lane of a shared tile: blocks of at most 8 columns per wave hold
// 8 rows of each column per lane (512-row tiles, so a level divides the
// rows by 16 at n = 32), blocks of 16 columns 4 (256-row tiles).  Eight
// waves of 16 columns cover 128: two waves per SIMD, 64 tile doubles per
// lane.
constexpr int coop_rpl(int cw) { return cw <= kNarrowCols ? 8 : 4; }

// One column step of the shared-tile kernel with the column's place in its
// block (JL) known at compile time (narrow blocks): the owner reduces only
// the JL..CW-1 columns it still holds and reads its registers in place, with
// no rotation.  j = o CW + JL >= n is skipped by every wave alike.
// Dot products over a lane's rows of a shared tile, in two interleaved
// partial sums (even and odd rows) to halve the dependent chain.
template <int RPL, int CW>
__device__ __forceinline__ double dot_rows(const double (&x)[RPL][CW], int a, int b) {
    double e = 0.0, o = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; r += 2) {
        e = fma(x[r][a], x[r][b], e);
        if (r + 1 < RPL) o = fma(x[r + 1][a], x[r + 1][b], o);
    }
    return e + o;
}

template <int RPL, int CW>
__device__ __forceinline__ double dot_rows(const double (&v)[RPL], const double (&x)[RPL][CW], int b) {
    double e = 0.0, o = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; r += 2) {
        e = fma(v[r], x[r][b], e);
        if (r + 1 < RPL) o = fma(v[r + 1], x[r + 1][b], o);
    }
    return e + o;
}

template <int W, int CW, int RPL, int JL>
__device__ __forceinline__ void coop_column(double (&x)[RPL][CW], double *rw, double (*xb)[64 * RPL],
                                            double (*sc)[4], int wib, int o, int n, int lane, int par) {
    const int j = o * CW + JL;
    if (j >= n) return;
    // buffer parity from a step count that runs on across tiles, so the
    // next tile's first column never reuses the buffer of this tile's last
    const int slot = (par + j) & 1;
    if (wib == o) {
        constexpr int C = CW - JL;
        double d[C], p[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            d[k] = dot_rows<RPL>(x, JL, JL + k);
            p[k] = rw[j * CW + JL + k];
        }
        wave_sum_batch<C>(d);
        const Reflector h = reflector(p[0], d[0]);
#pragma unroll
        for (int r = 0; r < RPL; ++r) xb[slot][lane * RPL + r] = x[r][JL];
        sc[slot][0] = h.scale;
        sc[slot][1] = h.ts;
        sc[slot][2] = h.tau;
#pragma unroll
        for (int k = 1; k < C; ++k) {
            const double w = fma(h.scale, d[k], p[k]);
            const double g = h.ts * w;
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][JL + k] = fma(-g, x[r][JL], x[r][JL + k]);
            rw[j * CW + JL + k] = fma(-h.tau, w, p[k]);
        }
        rw[j * CW + JL] = h.rjj;
    }
    __syncthreads();
    if (wib > o) {
        double xj[RPL], d[CW], p[CW];
#pragma unroll
        for (int r = 0; r < RPL; ++r) xj[r] = xb[slot][lane * RPL + r];
        const double scale = sc[slot][0], ts = sc[slot][1], tau = sc[slot][2];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            d[k] = dot_rows<RPL>(xj, x, k);
            p[k] = rw[j * CW + k];
        }
        wave_sum_batch<CW>(d);
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            const double w = fma(scale, d[k], p[k]);
            const double g = ts * w;
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r][k] = fma(-g, xj[r], x[r][k]);
            rw[j * CW + k] = fma(-tau, w, p[k]);
        }
    }
}

template <int W, int CW, int RPL, int... JLs>
__device__ __forceinline__ void coop_block(double (&x)[RPL][CW], double *rw, double (*xb)[64 * RPL],
                                           double (*sc)[4], int wib, int o, int n, int lane, int par,
                                           std::integer_sequence<int, JLs...>) {
    (coop_column<W, CW, RPL, JLs>(x, rw, xb, sc, wib, o, n, lane, par), ...);
}

template <int W, int CW>
__global__ __launch_bounds__(64 * W) void k_dense_coop(DenseArgs a) {
    constexpr int RPL = coop_rpl(CW), T = 64 * RPL;
    constexpr int NW = CW * W;                   // rows of an R slice
    constexpr int SL = (NW + 1) * CW;            // slice: NW rows + a spare row
    __shared__ double rsl[W * SL];
    __shared__ double xb[2][T];
    __shared__ double sc[2][4];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    double *rw = rsl + wib * SL;
    for (int i = lane; i < SL; i += 64) rw[i] = 0.0;
    const int n = a.n;
    for (int64_t it = 0; it < a.tiles_per_wave; ++it) {
        double x[RPL][CW];
        const int64_t base = ((int64_t)blockIdx.x * a.tiles_per_wave + it) * T + (int64_t)lane * RPL;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int col = CW * wib + c;
            const bool live = col < n;
            const double *src = a.in + (int64_t)(live ? col : 0) * a.ld_in;
#pragma unroll
            for (int k = 0; k < RPL; ++k) x[k][c] = (live && base + k < a.rows) ? src[base + k] : 0.0;
        }
        const int par = (int)((it * n) & 1);
        static_assert(CW <= kMidCols, "column blocks of at most 16 columns per wave");
        for (int o = 0; o < W; ++o)
            coop_block<W, CW, RPL>(x, rw, xb, sc, wib, o, n, lane, par, std::make_integer_sequence<int, CW>{});
    }
    __syncthreads();   // every slice complete (the diagonal is read across slices)
    const bool fin = gridDim.x == 1 && a.final_r;
    for (int j = lane; j < n; j += 64) {
        const double dg = rsl[(j / CW) * SL + j * CW + (j % CW)];
        const double sg = (fin && dg < 0.0) ? -1.0 : 1.0;
#pragma unroll 4
        for (int c = 0; c < CW; ++c) {
            const int col = CW * wib + c;
            if (col >= n) break;
            const double v = (col >= j) ? sg * rw[j * CW + c] : 0.0;
            if (fin) a.final_r[(int64_t)col * n + j] = v;
            else a.out[(int64_t)col * a.ld_out + (int64_t)blockIdx.x * n + j] = v;
        }
    }
}

// One thread per (key group, output column): the column's source (own sums
// or a child's sums gathered through the child index) times the exact
// integer multiplier of the group.
__global__ void k_join(JoinArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int oc = blockIdx.y;
    if (g >= a.groups) return;
    const int src = a.col_src[oc], c = a.col_idx[oc];
    double v;
    if (src < 0) {
        v = a.own[(int64_t)c * a.ld_own + g] * a.own_mult[g];
    } else {
        const int64_t q = a.cidx[src][g];
        v = a.sigma[src][(int64_t)c * a.ld_sigma[src] + q] * a.mult[src][g];
    }
    a.s[(int64_t)oc * a.ld_s + g] = v;
}

// One thread per (root key group, column).
// Column-major [ncols][ld_src] -> row-major [rows][ncols] (one thread per row).
__global__ void k_rowmajor(const double *src, int64_t ld_src, int64_t rows, int32_t ncols, double *dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows) return;
    for (int c = 0; c < ncols; ++c) dst[t * ncols + c] = src[(int64_t)c * ld_src + t];
}

__global__ void k_root(RootArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (g >= a.groups) return;
    const double f = a.inv_sqrt_c ? a.inv_sqrt_c[g] : 1.0;
    const int64_t row = a.row0 + g;
    a.dst[(int64_t)c * a.ld_dst + row] = a.s[(int64_t)c * a.ld_s + g] * f;
    if (c == 0 && a.block_of_row) a.block_of_row[row] = a.block_id;
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
    return 40;
}

// Tile shapes of the head/tail + QR kernel: rows per lane (RPL), minimum
// resident waves per SIMD the register budget is built for (OCC), and the QR
// form (ROT: compact runtime column loop; otherwise fully unrolled
// triangular).  variant 0: unrolled, one wave per SIMD; 1: compact; 2:
// unrolled, two waves per SIMD.
template <int NB, int V>
struct Shape {
    static constexpr bool ROT = V == 1;
    static constexpr int RPL = V == 2 ? (NB <= 8 ? 6 : NB <= 16 ? 2 : 1)
                                      : (NB <= 8 ? 8 : NB <= 16 ? 4 : !ROT ? 2 : 1);
    static constexpr int OCC = (V == 2 && NB <= 32) ? 2 : 1;
};

constexpr int kVariants = 3;

template <int NB, int V>
hipError_t helmert_nb(const HelmertArgs &a, bool unit, bool fuse, hipStream_t s) {
    constexpr int RPL = Shape<NB, V>::RPL, OCC = Shape<NB, V>::OCC;
    constexpr bool ROT = Shape<NB, V>::ROT;
    // a wide task's column chunks side by side (never fused)
    if (a.wide_cols > 0 && (fuse || a.ncols != NB)) return hipErrorInvalidValue;
    const unsigned chunks = a.wide_cols > 0 ? (unsigned)((a.wide_cols + NB - 1) / NB) : 1u;
    dim3 grid((a.waves + kWavesPerBlock - 1) / kWavesPerBlock, chunks), block(64 * kWavesPerBlock);
    if (a.join) {
        // joined heads are key groups with counts: weighted tails only
        if (unit) return hipErrorInvalidValue;
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 1, true, OCC, ROT, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 1, false, OCC, ROT, true>), grid, block, 0, s, a);
    } else if (unit) {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 0, true, OCC, ROT, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 0, false, OCC, ROT, false>), grid, block, 0, s, a);
    } else {
        if (fuse) hipLaunchKernelGGL((k_helmert<NB, RPL, 1, true, OCC, ROT, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_helmert<NB, RPL, 1, false, OCC, ROT, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int NB, int V>
hipError_t dense_nb(const DenseArgs &a, hipStream_t s) {
    constexpr int RPL = Shape<NB, V>::RPL, OCC = Shape<NB, V>::OCC;
    dim3 grid(a.waves), block(64 * kWavesPerBlock);
    hipLaunchKernelGGL((k_dense<NB, RPL, Shape<NB, V>::ROT, OCC>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int NB>
hipError_t helmert_v(const HelmertArgs &a, bool unit, bool fuse, int variant, hipStream_t s) {
    switch (variant) {
        case 1: return helmert_nb<NB, 1>(a, unit, fuse, s);
        case 2: return helmert_nb<NB, 2>(a, unit, fuse, s);
        default: return helmert_nb<NB, 0>(a, unit, fuse, s);
    }
}

template <int NB>
hipError_t dense_v(const DenseArgs &a, int variant, hipStream_t s) {
    switch (variant) {
        case 1: return dense_nb<NB, 1>(a, s);
        case 2: return dense_nb<NB, 2>(a, s);
        default: return dense_nb<NB, 0>(a, s);
    }
}

}  // namespace

template <int V>
int tile_items_v(int ncols) {
    switch (nb_for(ncols)) {
        case 8: return 64 * Shape<8, V>::RPL;
        case 16: return 64 * Shape<16, V>::RPL;
        case 32: return 64 * Shape<32, V>::RPL;
        case 40: return 64 * (V == 1 ? Shape<40, 1>::RPL : Shape<40, 0>::RPL);
        default: return 64 * Shape<64, 0>::RPL;
    }
}

int tile_items_for(int ncols, int variant) {
    // wide tasks run in column chunks of kChunkCols
    if (ncols > kFusedMaxCols) ncols = kChunkCols;
    switch (variant) {
        case 1: return tile_items_v<1>(ncols);
        case 2: return tile_items_v<2>(ncols);
        default: return tile_items_v<0>(ncols);
    }
}

bool dense_coop(int ncols) { return ncols > 16; }

int dense_tile_rows_for(int ncols, int variant) {
    if (!dense_coop(ncols)) return tile_items_for(ncols, variant);
    return 64 * coop_rpl(ncols <= 64 ? kNarrowCols : kMidCols);
}

int dense_waves_per_block(int ncols) {
    return dense_coop(ncols) ? 1 : kWavesPerBlock;
}
int waves_per_block() { return kWavesPerBlock; }
int num_variants() { return kVariants; }

hipError_t launch_helmert(const HelmertArgs &a, bool unit, bool fuse, int variant, hipStream_t s) {
    if (a.waves <= 0 || a.nchunks <= 0) return hipSuccess;
    switch (nb_for(a.ncols)) {
        case 8: return helmert_v<8>(a, unit, fuse, variant, s);
        case 16: return helmert_v<16>(a, unit, fuse, variant, s);
        case 32: return helmert_v<32>(a, unit, fuse, variant, s);
        case 40:
            if (a.ncols > kFusedMaxCols) return hipErrorInvalidValue;   // wide tasks run in column chunks
            return variant == 1 ? helmert_nb<40, 1>(a, unit, fuse, s) : helmert_nb<40, 0>(a, unit, fuse, s);
        default: return hipErrorInvalidValue;
    }
}

int helmert_shape_class(int ncols) { return nb_for(ncols); }

template <int NB, int V>
hipError_t helmert_batch_nb(const HelmertBatch &b, bool unit, bool fuse, hipStream_t s) {
    constexpr int RPL = Shape<NB, V>::RPL, OCC = Shape<NB, V>::OCC;
    constexpr bool ROT = Shape<NB, V>::ROT;
    const dim3 grid(b.wg0[b.count]), block(64 * kWavesPerBlock);
    if (unit) {
        if (fuse) hipLaunchKernelGGL((k_helmert_multi<NB, RPL, 0, true, OCC, ROT>), grid, block, 0, s, b);
        else hipLaunchKernelGGL((k_helmert_multi<NB, RPL, 0, false, OCC, ROT>), grid, block, 0, s, b);
    } else {
        if (fuse) hipLaunchKernelGGL((k_helmert_multi<NB, RPL, 1, true, OCC, ROT>), grid, block, 0, s, b);
        else hipLaunchKernelGGL((k_helmert_multi<NB, RPL, 1, false, OCC, ROT>), grid, block, 0, s, b);
    }
    return hipGetLastError();
}

template <int NB>
hipError_t helmert_batch_v(const HelmertBatch &b, bool unit, bool fuse, int variant, hipStream_t s) {
    switch (variant) {
        case 1: return helmert_batch_nb<NB, 1>(b, unit, fuse, s);
        case 2: return helmert_batch_nb<NB, 2>(b, unit, fuse, s);
        default: return helmert_batch_nb<NB, 0>(b, unit, fuse, s);
    }
}

hipError_t launch_helmert_batch(const HelmertBatch &b, bool unit, bool fuse, int variant, hipStream_t s) {
    if (b.count <= 0 || b.count > kHelmertBatch || b.wg0[b.count] <= 0) return hipErrorInvalidValue;
    const int nb = nb_for(b.a[0].ncols);
    for (int t = 0; t < b.count; ++t)
        if (b.a[t].ncols > kFusedMaxCols || nb_for(b.a[t].ncols) != nb || b.a[t].wide_cols != 0 || b.a[t].join)
            return hipErrorInvalidValue;
    switch (nb) {
        case 8: return helmert_batch_v<8>(b, unit, fuse, variant, s);
        case 16: return helmert_batch_v<16>(b, unit, fuse, variant, s);
        case 32: return helmert_batch_v<32>(b, unit, fuse, variant, s);
        case 40:
            return variant == 1 ? helmert_batch_nb<40, 1>(b, unit, fuse, s) : helmert_batch_nb<40, 0>(b, unit, fuse, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense(const DenseArgs &a, int variant, hipStream_t s) {
    if (a.waves <= 0) return hipSuccess;
    if (a.n > kMaxCols) return hipErrorInvalidValue;
    if (!dense_coop(a.n)) {
        switch (nb_for(a.n)) {
            case 8: return dense_v<8>(a, variant, s);
            default: return dense_v<16>(a, variant, s);
        }
    }
    const dim3 grid(a.waves);
    if (a.n <= kFusedMaxCols) {
        static_assert(kFusedMaxCols <= 5 * kNarrowCols, "five column blocks cover a narrow stack");
        // up to 32 columns: 4 per wave (6 or 8 waves); above: 8 per wave
        if (a.n <= 24) hipLaunchKernelGGL((k_dense_coop<6, 4>), grid, dim3(384), 0, s, a);
        else if (a.n <= 32) hipLaunchKernelGGL((k_dense_coop<8, 4>), grid, dim3(512), 0, s, a);
        else hipLaunchKernelGGL((k_dense_coop<5, kNarrowCols>), grid, dim3(320), 0, s, a);
    } else if (a.n <= 64) {
        // 8 columns per wave on 512-row tiles
        hipLaunchKernelGGL((k_dense_coop<8, kNarrowCols>), grid, dim3(512), 0, s, a);
    } else {
        // 16 columns per wave on 256-row tiles
        hipLaunchKernelGGL((k_dense_coop<8, kMidCols>), grid, dim3(512), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_join(const JoinArgs &a, hipStream_t s) {
    if (a.groups <= 0 || a.nsub <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_join, dim3((unsigned)((a.groups + bs - 1) / bs), (unsigned)a.nsub), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rowmajor(const double *src, int64_t ld_src, int64_t rows, int32_t ncols, double *dst, hipStream_t s) {
    if (rows <= 0 || ncols <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_rowmajor, dim3((unsigned)((rows + bs - 1) / bs)), dim3(bs), 0, s, src, ld_src, rows, ncols,
                       dst);
    return hipGetLastError();
}

hipError_t launch_root(const RootArgs &a, bool, hipStream_t s) {
    if (a.groups <= 0 || a.n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_root, dim3((unsigned)((a.groups + bs - 1) / bs), (unsigned)a.n), dim3(bs), 0, s, a);
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
