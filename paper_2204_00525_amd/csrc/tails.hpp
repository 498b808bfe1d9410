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

// Per-item inputs of the tail coefficients: MODE 0 the position j of the
// item in its piece and the piece's scale phi; MODE 1 alpha and beta.
template <int RPL>
struct TileCoef {
    double c0[RPL], c1[RPL];
};

// Columns col0 .. col0 + NB - 1 of the joined heads of items
// base .. base + RPL - 1 read in place (JoinSrc): own sums times own_mult,
// or a child's sums at the child group of the item times that child's mult.
// The source of a column is uniform over the wave; its base address, stride
// and factor are picked with selects, so the loads of all columns are
// branch-free and in flight together.  The products are rounded as such
// (never contracted into a later addition), exactly as the stored joined
// heads would be.
template <int NB, int RPL>
__device__ __forceinline__ void join_load(const JoinSrc &js, int col0, int ncols, int64_t base, const bool (&valid)[RPL],
                                          int64_t tclamp, double (&x)[RPL][NB]) {
    int64_t t[RPL];
    double om[RPL];
    int32_t ci[kFuseMaxChildren][RPL];
    double mu[kFuseMaxChildren][RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        t[k] = valid[k] ? base + k : tclamp;
        om[k] = js.own_mult[t[k]];
#pragma unroll
        for (int j = 0; j < kFuseMaxChildren; ++j) {
            const bool has = j < js.nchildren;
            ci[j][k] = has ? js.cidx[j][t[k]] : 0;
            mu[j][k] = has ? js.mult[j][t[k]] : 0.0;
        }
    }
    // all loads first (nothing waits on them inside the column loop), then
    // the products
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const bool live = c < ncols;
        const int code = js.code[live ? col0 + c : col0];
        const int src = (code >> 8) - 1, q = code & 0xff;
        const bool own = src < 0;
        const int sj = own ? 0 : src;
        const double *colp = own ? js.own + (int64_t)q * js.ld_own : js.sigma[sj] + q;
        const int64_t ld = own ? 1 : js.ld_sigma[sj];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            int32_t g = ci[0][k];
#pragma unroll
            for (int j = 1; j < kFuseMaxChildren; ++j) g = (sj == j) ? ci[j][k] : g;
            x[k][c] = colp[own ? t[k] : (int64_t)g * ld];
        }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const bool live = c < ncols;
        const int src = (js.code[live ? col0 + c : col0] >> 8) - 1;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            double m = om[k];
#pragma unroll
            for (int j = 0; j < kFuseMaxChildren; ++j) m = (src == j) ? mu[j][k] : m;
            x[k][c] = (live && valid[k]) ? __dmul_rn(x[k][c], m) : 0.0;
        }
    }
}

// Loads the tile's columns into x (zero for invalid items and columns >=
// ncols), the piece ids and the coefficient inputs.  Every lane loads its
// coefficients (clamped indices for items past the end or the first item of
// a piece), so no load sits under a divergent branch.  JOIN: the columns are
// those of the joined heads, read through js from column col0 on.
template <int NB, int RPL, int MODE, bool JOIN = false>
__device__ __forceinline__ void tile_load(const TailSrc &a, int64_t cs, int64_t ce, int lane,
                                          double (&x)[RPL][NB], TileItems<RPL> &ti, TileCoef<RPL> &cf,
                                          const JoinSrc *js = nullptr, int col0 = 0) {
    const int64_t base = cs + (int64_t)lane * RPL;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        ti.valid[k] = base + k < ce;
        ti.pid[k] = ti.valid[k] ? a.pid[base + k] : -1;
    }
    if constexpr (JOIN) {
        join_load<NB, RPL>(*js, col0, a.ncols, base, ti.valid, cs, x);
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const bool live = c < a.ncols;
            const double *col = a.in + (int64_t)(live ? c : 0) * a.ld_in;
#pragma unroll
            for (int k = 0; k < RPL; ++k) x[k][c] = (live && ti.valid[k]) ? col[base + k] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        if constexpr (MODE == 0) {
            const int32_t p = ti.valid[k] ? ti.pid[k] : a.pid[cs];
            cf.c0[k] = (double)(base + k - a.piece_start[p]);
            cf.c1[k] = a.phi_piece[p];
        } else {
            const int64_t tc = ti.valid[k] ? base + k : cs;
            cf.c0[k] = a.alpha[tc];
            cf.c1[k] = a.beta[tc];
        }
    }
}

// Replaces the loaded columns by the tail rows (zero for the first item of
// every piece).  With PIECES, the sum of every piece is written to
// pieces_out[c * ld_pieces + piece id] (if pieces_out is not null).
//
// Running sums are reset at piece starts by multiplying with a 0/1 factor
// rather than by selects; a non-finite value therefore spreads into the
// following pieces of the tile, which only matters for inputs that make R
// non-finite anyway.
template <int NB, int RPL, int MODE, bool PIECES>
__device__ __forceinline__ void tile_finish(const TailSrc &a, int64_t cs, int lane, double (&x)[RPL][NB],
                                            TileItems<RPL> &ti, const TileCoef<RPL> &cf) {
    // piece starts: the chunk's first item, and every change of piece id
    // (the lane shifts run unconditionally: under a divergent mask they
    // would read an inactive lane)
    const int32_t prev_last = wave_shr1(ti.pid[RPL - 1]);
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
    const int nf0 = wave_shl1((int)ti.first[0]);
    const bool next_first0 = (lane == 63) || (nf0 != 0);
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const bool use = ti.valid[k] && !ti.first[k];
        double al = 0.0, be = 0.0;
        if constexpr (MODE == 0) {
            if (use) {
                const double j = cf.c0[k];
                const double q = 1.0 / sqrt(j * (j + 1.0));
                al = cf.c1[k] * j * q;
                be = cf.c1[k] * q;
            }
        } else {
            al = use ? cf.c0[k] : 0.0;
            be = use ? cf.c1[k] : 0.0;
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

template <int NB, int RPL, int MODE, bool PIECES, bool JOIN = false>
__device__ __forceinline__ void tile_tails(const TailSrc &a, int64_t cs, int64_t ce, int lane,
                                           double (&x)[RPL][NB], TileItems<RPL> &ti,
                                           const JoinSrc *js = nullptr, int col0 = 0) {
    TileCoef<RPL> cf;
    tile_load<NB, RPL, MODE, JOIN>(a, cs, ce, lane, x, ti, cf, js, col0);
    tile_finish<NB, RPL, MODE, PIECES>(a, cs, lane, x, ti, cf);
}

// Early fetch of the children's rows of the items cs .. ce - 1 (the next
// chunk) into the caches: a 4-byte asynchronous copy of each row start into
// a scratch LDS word that nobody reads.  The wave does not wait for these;
// by the time it gathers the rows they are close.
template <int RPL>
__device__ __forceinline__ void join_prefetch(const JoinSrc &js, int64_t cs, int64_t ce, int lane, void *sink);

// ---------------------------------------------------------------------------
// Staging of the next tile in LDS.  A wave that processes consecutive chunks
// copies the next full chunk (64*RPL items) from global memory into its own
// LDS area with asynchronous global-to-LDS loads (16 bytes per lane, no
// registers held while they fly) and works on the current tile meanwhile.
// Layout of a wave's area, T = 64*RPL: the NB columns of the tile ([NB][T]
// doubles), the two coefficient inputs ([T] doubles each: alpha and beta, or
// for MODE 0 the window of phi and of the piece starts of the chunk's
// pieces), the piece ids ([T] int32).
template <int NB, int RPL>
struct Stage {
    static constexpr int T = 64 * RPL;
    static constexpr int W = T + 2;             // window entries (even start)
    static constexpr int C0 = NB * T;
    static constexpr int C1 = C0 + W;
    static constexpr int PID = C1 + W;          // in doubles; T int32 follow
    static constexpr int doubles = PID + T / 2;
};

__device__ __forceinline__ void lds_copy16(const void *src, void *dst) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                     (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

__device__ __forceinline__ void lds_copy4(const void *src, void *dst) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                     (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
}

template <int RPL>
__device__ __forceinline__ void join_prefetch(const JoinSrc &js, int64_t cs, int64_t ce, int lane, void *sink) {
    const int64_t base = cs + (int64_t)lane * RPL;
#pragma unroll
    for (int j = 0; j < kFuseMaxChildren; ++j) {
        if (j < js.nchildren) {
            int32_t g[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) g[k] = js.cidx[j][base + k < ce ? base + k : cs];
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (base + k < ce) lds_copy4(js.sigma[j] + (int64_t)g[k] * js.ld_sigma[j], sink);
        }
    }
}

// n (<= N) 8-byte entries from src to dst (both 16-byte aligned); lane l
// copies entries 128 q + 2 l and 128 q + 2 l + 1.  Reads entry n when n is
// odd (the caller guarantees it exists).
template <int N>
__device__ __forceinline__ void stage_span(const void *src, void *dst, int n, int lane) {
    const char *s = (const char *)src;
    char *d = (char *)dst;
#pragma unroll
    for (int q = 0; q < (N + 127) / 128; ++q) {
        const int e = 128 * q + 2 * lane;
        if (e < n) lds_copy16(s + 8 * (int64_t)e, d + 8 * 128 * q);
    }
}

// Issue the copies of chunk [cs, cs + T) (a full chunk; the columns start
// 16-byte aligned).  MODE 0 copies the window of the chunk's pieces from the
// even id p0 to p1 - 1.
template <int NB, int RPL, int MODE>
__device__ __forceinline__ void stage_issue(const TailSrc &a, int64_t cs, int32_t p0, int32_t p1, double *st,
                                            int lane) {
    using S = Stage<NB, RPL>;
    constexpr int T = S::T;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c < a.ncols) stage_span<T>(a.in + (int64_t)c * a.ld_in + cs, st + c * T, T, lane);
    if constexpr (MODE == 0) {
        stage_span<S::W>(a.phi_piece + p0, st + S::C0, p1 - p0, lane);
        stage_span<S::W>(a.piece_start + p0, st + S::C1, p1 - p0, lane);
    } else {
        stage_span<T>(a.alpha + cs, st + S::C0, T, lane);
        stage_span<T>(a.beta + cs, st + S::C1, T, lane);
    }
    int32_t *pid = (int32_t *)(st + S::PID);
#pragma unroll
    for (int q = 0; q < RPL; ++q) lds_copy4(a.pid + cs + 64 * q + lane, pid + 64 * q);
}

// The staged chunk into registers (all items valid).
template <int NB, int RPL, int MODE>
__device__ __forceinline__ void stage_read(const TailSrc &a, int64_t cs, int32_t p0, const double *st, int lane,
                                           double (&x)[RPL][NB], TileItems<RPL> &ti, TileCoef<RPL> &cf) {
    using S = Stage<NB, RPL>;
    constexpr int T = S::T;
    const int r0 = lane * RPL;
    const int32_t *pid = (const int32_t *)(st + S::PID);
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        ti.valid[k] = true;
        ti.pid[k] = pid[r0 + k];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
#pragma unroll
        for (int k = 0; k < RPL; ++k) x[k][c] = (c < a.ncols) ? st[c * T + r0 + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        if constexpr (MODE == 0) {
            const int w = ti.pid[k] - p0;
            const int64_t *ps = (const int64_t *)(st + S::C1);
            cf.c0[k] = (double)(cs + r0 + k - ps[w]);
            cf.c1[k] = st[S::C0 + w];
        } else {
            cf.c0[k] = st[S::C0 + r0 + k];
            cf.c1[k] = st[S::C1 + r0 + k];
        }
    }
}

}  // namespace
}  // namespace figaro
