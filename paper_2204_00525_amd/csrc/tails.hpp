// Segmented (generalized) heads and tails of one tile of items, shared by the
// forward and backward head/tail kernels.  Internal.
//
// A tile is one chunk of at most 64*RPL consecutive items; lane l holds items
// l*RPL .. l*RPL+RPL-1.  Items are grouped into pieces (a key group, or the
// part of a key group inside the chunk); within a piece with running sum
// P_j of the first j items, the tail row of item j+1 (j >= 1) is
//   T = alpha * a_{j+1} - beta * P_j
// (section "Heads and Tails", Definition "Head and Tail" for unit weights,
// Definition 2 for weighted items; alpha, beta carry the scale factor of
// Algorithm 3), and the first item of a piece has no tail.  For unit weights
// alpha = phi j / sqrt(j (j+1)), beta = phi / sqrt(j (j+1)); weighted items
// bring alpha, beta from the plan.
#pragma once

#include "device_common.hpp"

namespace figaro {
namespace {

// Where the items of a head/tail level come from (a block of columns of
// `in`), their piece ids and tail coefficients, and where piece sums go.
struct TailSrc {
    const double *in;
    int64_t ld_in;
    int32_t ncols;
    const int32_t *pid;
    const int64_t *piece_start;
    const double *phi_piece;
    const double *alpha;
    const double *beta;
    double *pieces_out;          // may be null
    int64_t ld_pieces;
};

template <class Args>
__device__ __forceinline__ TailSrc tail_src(const Args &a) {
    TailSrc t;
    t.in = a.in;
    t.ld_in = a.ld_in;
    t.ncols = a.ncols;
    t.pid = a.pid;
    t.piece_start = a.piece_start;
    t.phi_piece = a.phi_piece;
    t.alpha = a.alpha;
    t.beta = a.beta;
    t.pieces_out = nullptr;
    t.ld_pieces = 0;
    return t;
}

template <int RPL>
struct TileItems {
    int32_t pid[RPL];
    bool valid[RPL];
    bool first[RPL];     // first item of its piece within the chunk (or invalid)
    bool last[RPL];      // valid and last item of its piece within the chunk
    double al[RPL], be[RPL];
};

// Loads the tile's columns into x (zero for invalid items and columns >=
// ncols) and replaces them by the tail rows (zero for the first item of
// every piece).  With PIECES, the sum of every piece is written to
// pieces_out[c * ld_pieces + piece id] (if pieces_out is not null).
//
// Running sums are reset at piece starts by multiplying with a 0/1 factor
// rather than by selects; a non-finite value therefore spreads into the
// following pieces of the tile, which only matters for inputs that make R
// non-finite anyway.
template <int NB, int RPL, int MODE, bool PIECES>
__device__ __forceinline__ void tile_tails(const TailSrc &a, int64_t cs, int64_t ce, int lane,
                                           double (&x)[RPL][NB], TileItems<RPL> &ti) {
    const int64_t base = cs + (int64_t)lane * RPL;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        ti.valid[k] = base + k < ce;
        ti.pid[k] = ti.valid[k] ? a.pid[base + k] : -1;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const bool live = c < a.ncols;
        const double *col = a.in + (int64_t)(live ? c : 0) * a.ld_in;
#pragma unroll
        for (int k = 0; k < RPL; ++k) x[k][c] = (live && ti.valid[k]) ? col[base + k] : 0.0;
    }
    // piece starts: the chunk's first item, and every change of piece id
    // (shuffle unconditionally: under a divergent mask it would read an
    // inactive lane)
    const int32_t prev_last = __shfl_up(ti.pid[RPL - 1], 1, 64);
    double keep[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int32_t prev = (k == 0) ? prev_last : ti.pid[k - 1];
        ti.first[k] = !ti.valid[k] || (k == 0 && lane == 0) || ti.pid[k] != prev;
        keep[k] = ti.first[k] ? 0.0 : 1.0;
    }
    bool lane_flag = false;
#pragma unroll
    for (int k = 0; k < RPL; ++k) lane_flag = lane_flag || ti.first[k];
    // per-lane aggregate since the lane's last piece start, then the carry
    // from the lanes below
    double acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) sum = fma(sum, keep[k], x[k][c]);
        acc[c] = sum;
    }
    segmented_carry<NB>(acc, __ballot(lane_flag), lane);
    const int nf0 = __shfl_down((int)ti.first[0], 1, 64);
    const bool next_first0 = (lane == 63) || (nf0 != 0);
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int64_t t = base + k;
        const bool use = ti.valid[k] && !ti.first[k];
        double al = 0.0, be = 0.0;
        if constexpr (MODE == 0) {
            if (use) {
                const double j = (double)(t - a.piece_start[ti.pid[k]]);
                const double q = 1.0 / sqrt(j * (j + 1.0));
                const double phi = a.phi_piece[ti.pid[k]];
                al = phi * j * q;
                be = phi * q;
            }
        } else {
            // branch-free: every lane loads (a clamped index for items past
            // the end), the piece start selects zero
            const int64_t tc = ti.valid[k] ? t : cs;
            const double a0 = a.alpha[tc], b0 = a.beta[tc];
            al = use ? a0 : 0.0;
            be = use ? b0 : 0.0;
        }
        ti.al[k] = al;
        ti.be[k] = be;
        ti.last[k] = ti.valid[k] && ((k + 1 < RPL) ? ti.first[k + 1] : next_first0);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double xv = x[k][c];
            const double run = acc[c] * keep[k];
            x[k][c] = fma(al, xv, -be * run);
            acc[c] = run + xv;
        }
        if constexpr (PIECES) {
            if (ti.last[k] && a.pieces_out) {
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < a.ncols) a.pieces_out[(int64_t)c * a.ld_pieces + ti.pid[k]] = acc[c];
            }
        }
    }
}

}  // namespace
}  // namespace figaro
