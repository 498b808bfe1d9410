// The plan on the device: key segmentation (the sort order the paper's
// algorithms assume), the semi-join reduction of dangling tuples, the count
// queries of Algorithm 2 (section "Scaling Factors as Count Queries") and the
// first level of every head/tail task, from device key columns.  The result
// equals the host builder's plan exactly: the same dense ids, the same stable
// order, the same integer counts and the same correctly rounded scale
// factors.
//
// Building blocks (all stable, all exact):
//  * an exclusive scan of int64 values (per-tile sums, a scan of those, and
//    the tiles scanned with their offsets);
//  * an LSD radix sort of keys of up to 128 bits with a 64-bit payload, in
//    8-bit digits: per-tile digit histograms, a scan of them in digit-major
//    order, and a scatter in which every element's rank among the equal
//    digits before it in its tile comes from eight wave ballots (one per
//    digit bit), the per-wave counts of earlier waves and the running counts
//    of earlier rounds, so equal keys keep their order;
//  * compaction of flagged positions (scan of the flags);
//  * lookup of packed keys in a sorted list of distinct keys (binary search).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

namespace figaro {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;
constexpr uint64_t kExact = uint64_t(1) << 53;   // counts must stay below 2^53

// status bits raised on the device
constexpr int kStOverflow = 1;     // a count reaches 2^53
constexpr int kStInexact = 2;      // an up-count division leaves a remainder
constexpr int kStUnmatched = 4;    // a key group finds no child group

int64_t tiles(int64_t n) { return (n + kTile - 1) / kTile; }
unsigned grid_for(int64_t n, int bs = kBlock) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Temporary device buffers of one plan build (freed when it ends).
struct Temp {
    std::vector<void *> ptrs;
    ~Temp() {
        for (void *q : ptrs) (void)hipFree(q);
    }
    template <class T>
    T *get(int64_t n) {
        void *q = nullptr;
        if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) throw std::bad_alloc();
        ptrs.push_back(q);
        return static_cast<T *>(q);
    }
};

// ---------------------------------------------------------------------------
// Scan, compaction
// ---------------------------------------------------------------------------

__global__ void k_tile_sums(const int64_t *in, int64_t n, int64_t *sums) {
    __shared__ int64_t sh[kBlock];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t acc = 0;
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + t;
        if (i < n) acc += in[i];
    }
    sh[t] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    if (t == 0) sums[blockIdx.x] = sh[0];
}

// out[i] = off[tile of i] + sum of in[j] for the j < i of the same tile
// (thread t of a tile scans its 8 consecutive elements)
__global__ void k_tile_scan(const int64_t *in, int64_t n, const int64_t *off, int64_t *out) {
    __shared__ int64_t sh[kBlock];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)t * kItems;
    int64_t v[kItems], loc = 0;
    for (int k = 0; k < kItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        loc += v[k];
    }
    sh[t] = loc;
    __syncthreads();
    for (int s = 1; s < kBlock; s <<= 1) {
        const int64_t add = t >= s ? sh[t - s] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t run = (off ? off[blockIdx.x] : 0) + sh[t] - loc;
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// exclusive scan; in and out may not alias
void scan_excl(const int64_t *in, int64_t *out, int64_t n, Temp &T, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nt = tiles(n);
    if (nt == 1) {
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kBlock), 0, s, in, n, nullptr, out);
        return;
    }
    int64_t *sums = T.get<int64_t>(nt), *off = T.get<int64_t>(nt);
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nt), dim3(kBlock), 0, s, in, n, sums);
    scan_excl(sums, off, nt, T, s);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nt), dim3(kBlock), 0, s, in, n, off, out);
}

int64_t read_i64(const int64_t *p, hipStream_t s) {
    int64_t v = 0;
    if (hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        throw std::runtime_error("device read failed");
    return v;
}

// flagged positions (flags 0/1, n of them) in increasing order into pos_out;
// returns their number (synchronises)
__global__ void k_compact(const int64_t *flags, const int64_t *at, int64_t n, int64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) out[at[i]] = i;
}

int64_t compact(const int64_t *flags, int64_t n, int64_t *out, Temp &T, hipStream_t s) {
    if (n <= 0) return 0;
    int64_t *at = T.get<int64_t>(n);
    scan_excl(flags, at, n, T, s);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(n)), dim3(kBlock), 0, s, flags, at, n, out);
    return read_i64(at + n - 1, s) + read_i64(flags + n - 1, s);
}

// ---------------------------------------------------------------------------
// Radix sort of 128-bit keys (lo, hi) with a 64-bit payload
// ---------------------------------------------------------------------------

__device__ __forceinline__ int key_digit(uint64_t lo, uint64_t hi, int shift) {
    uint64_t v;
    if (shift >= 64) v = hi >> (shift - 64);
    else if (shift == 0) v = lo;
    else v = (lo >> shift) | (hi << (64 - shift));
    return (int)(v & 255);
}

__global__ void k_digit_hist(const uint64_t *lo, const uint64_t *hi, int64_t n, int shift, int64_t *hist, int64_t nt) {
    __shared__ int cnt[256];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + t;
        if (i < n) atomicAdd(&cnt[key_digit(lo[i], hi ? hi[i] : 0, shift)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nt + blockIdx.x] = cnt[t];
}

// Round k of a tile handles its elements k*256 .. k*256+255 (thread t takes
// element k*256 + t): the element's rank among the equal digits before it is
// the running count of its digit over earlier rounds, the counts of earlier
// waves of this round, and the equal-digit lanes below it in its wave.
__global__ void k_digit_scatter(const uint64_t *lo, const uint64_t *hi, const int64_t *pay, int64_t n, int shift,
                                const int64_t *off, int64_t nt, uint64_t *lo_o, uint64_t *hi_o, int64_t *pay_o) {
    __shared__ int wcnt[kBlock / 64][256];
    __shared__ int64_t run[256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    run[t] = off[(int64_t)t * nt + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int k = 0; k < kItems; ++k) {
        for (int q = 0; q < kBlock / 64; ++q) wcnt[q][t] = 0;
        const int64_t i = base + (int64_t)k * kBlock + t;
        const bool valid = i < n;
        const uint64_t klo = valid ? lo[i] : 0, khi = (valid && hi) ? hi[i] : 0;
        const int d = valid ? key_digit(klo, khi, shift) : 0;
        uint64_t same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t set = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? set : ~set;
        }
        const int rank = __popcll(same & below);
        __syncthreads();
        if (valid && rank == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int64_t pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            lo_o[pos] = klo;
            if (hi) hi_o[pos] = khi;
            pay_o[pos] = pay[i];
        }
        __syncthreads();
        int add = 0;
        for (int q = 0; q < kBlock / 64; ++q) add += wcnt[q][t];
        run[t] += add;
        __syncthreads();
    }
}

// Sorts (lo, hi, pay) by the low `bits` bits of the key, stably; hi may be
// null (keys of at most 64 bits).  The sorted arrays may end up in the
// scratch buffers: the pointers are updated.
void radix_sort(uint64_t *&lo, uint64_t *&hi, int64_t *&pay, int64_t n, int bits, Temp &T, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t nt = tiles(n);
    int64_t *hist = T.get<int64_t>(256 * nt), *off = T.get<int64_t>(256 * nt);
    uint64_t *lo2 = T.get<uint64_t>(n), *hi2 = hi ? T.get<uint64_t>(n) : nullptr;
    int64_t *pay2 = T.get<int64_t>(n);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)nt), dim3(kBlock), 0, s, lo, hi, n, shift, hist, nt);
        scan_excl(hist, off, 256 * nt, T, s);
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nt), dim3(kBlock), 0, s, lo, hi, pay, n, shift, off, nt,
                           lo2, hi2, pay2);
        std::swap(lo, lo2);
        std::swap(hi, hi2);
        std::swap(pay, pay2);
    }
}

__device__ __forceinline__ bool key_less(uint64_t alo, uint64_t ahi, uint64_t blo, uint64_t bhi) {
    return ahi < bhi || (ahi == bhi && alo < blo);
}

// index of each query key among `cnt` sorted distinct keys, -1 if absent
__device__ __forceinline__ int64_t find_key(const uint64_t *slo, const uint64_t *shi, int64_t cnt, uint64_t qlo,
                                            uint64_t qhi) {
    int64_t a = 0, b = cnt;
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (key_less(slo[m], shi ? shi[m] : 0, qlo, qhi)) a = m + 1;
        else b = m;
    }
    return (a < cnt && slo[a] == qlo && (shi ? shi[a] : 0) == qhi) ? a : -1;
}

// ---------------------------------------------------------------------------
// Keys
// ---------------------------------------------------------------------------

// Dense ids of some attributes of one relation packed into up to 128 bits
// (first attribute highest).
constexpr int kMaxPack = 32;
struct PackCols {
    const int32_t *col[kMaxPack];
    int32_t shift[kMaxPack];
    int32_t k;
};

__device__ __forceinline__ void pack_row(const PackCols &pc, int64_t row, uint64_t &lo, uint64_t &hi) {
    lo = 0;
    hi = 0;
    for (int q = 0; q < pc.k; ++q) {
        const uint64_t v = (uint32_t)pc.col[q][row];
        const int sh = pc.shift[q];
        if (sh >= 64) {
            hi |= v << (sh - 64);
        } else {
            lo |= v << sh;
            if (sh > 32) hi |= v >> (64 - sh);
        }
    }
}

// packed keys of rows[0..n) (rows null: rows 0..n-1)
__global__ void k_pack(PackCols pc, const int64_t *rows, int64_t n, uint64_t *lo, uint64_t *hi, int64_t *pay) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t row = rows ? rows[i] : i;
    uint64_t a, b;
    pack_row(pc, row, a, b);
    lo[i] = a;
    if (hi) hi[i] = b;
    if (pay) pay[i] = row;
}

__global__ void k_minmax(const void *col, int dtype, int64_t n, unsigned long long *mn, unsigned long long *mx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t v = dtype == 4 ? (int64_t)((const int32_t *)col)[i] : ((const int64_t *)col)[i];
    const unsigned long long u = (unsigned long long)v ^ (1ull << 63);   // order-preserving
    atomicMin(mn, u);
    atomicMax(mx, u);
}

__global__ void k_offset_values(const void *col, int dtype, int64_t n, uint64_t lo_val, int64_t at, uint64_t *v,
                                int64_t *pay) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t x = dtype == 4 ? (int64_t)((const int32_t *)col)[i] : ((const int64_t *)col)[i];
    v[at + i] = ((uint64_t)x ^ (1ull << 63)) - lo_val;
    pay[at + i] = at + i;
}

__global__ void k_change_flags(const uint64_t *lo, const uint64_t *hi, int64_t n, int rshift, int64_t *flags) {
    // flags[i] = 1 at i = 0 and wherever (key >> rshift) differs from the previous key's
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) {
        flags[0] = 1;
        return;
    }
    uint64_t a = lo[i], b = hi ? hi[i] : 0, c = lo[i - 1], d = hi ? hi[i - 1] : 0;
    if (rshift >= 128) {
        a = b = c = d = 0;
    } else if (rshift >= 64) {
        a = b >> (rshift - 64);
        c = d >> (rshift - 64);
        b = d = 0;
    } else if (rshift > 0) {
        a = (a >> rshift) | (b << (64 - rshift));
        c = (c >> rshift) | (d << (64 - rshift));
        b >>= rshift;
        d >>= rshift;
    }
    flags[i] = (a != c || b != d) ? 1 : 0;
}

__global__ void k_scatter_ids(const int64_t *flags_excl, const int64_t *flags, const int64_t *pay, int64_t n,
                              int32_t *ids) {
    // the rank of sorted element i is (number of distinct values up to i) - 1
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ids[pay[i]] = (int32_t)(flags_excl[i] + flags[i] - 1);
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_alive_flags(const uint8_t *alive, int64_t n, int64_t *flags, int invert) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = invert ? !alive[i] : alive[i];
}

// keep the alive rows of the keep side whose shared key occurs among the
// probe side's alive keys (sorted, distinct)
__global__ void k_semijoin(PackCols pc, uint8_t *alive, int64_t n, const uint64_t *slo, const uint64_t *shi,
                           int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !alive[i]) return;
    uint64_t a, b;
    pack_row(pc, i, a, b);
    if (find_key(slo, shi, cnt, a, b) < 0) alive[i] = 0;
}

__global__ void k_gather_keys(const uint64_t *lo, const uint64_t *hi, const int64_t *at, int64_t n, uint64_t *olo,
                              uint64_t *ohi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    olo[i] = lo[at[i]];
    if (hi) ohi[i] = hi[at[i]];
}

__global__ void k_shift_keys(uint64_t *lo, uint64_t *hi, int64_t n, int rshift) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t a = lo[i], b = hi ? hi[i] : 0;
    if (rshift >= 128) {
        a = b = 0;
    } else if (rshift >= 64) {
        a = b >> (rshift - 64);
        b = 0;
    } else if (rshift > 0) {
        a = (a >> rshift) | (b << (64 - rshift));
        b >>= rshift;
    }
    lo[i] = a;
    if (hi) hi[i] = b;
}

// segment id of every position from its start flags: inclusive count - 1
__global__ void k_seg_id(const int64_t *excl, const int64_t *flags, int64_t n, int64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = excl[i] + flags[i] - 1;
}

__global__ void k_copy_i64(const int64_t *src, int64_t *dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

__global__ void k_zero_u64(uint64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// flags over items 0..n-1 marking the starts of the ranges [off[q], off[q+1])
__global__ void k_mark_starts(const int64_t *off, int64_t cnt, int64_t *flags) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < cnt) flags[off[q]] = 1;
}

// child index of key group g: the child's parent group holding the key of
// the group's first row
__global__ void k_child_index(PackCols pc, const int64_t *perm, const int64_t *seg_off, int64_t G,
                              const uint64_t *slo, const uint64_t *shi, int64_t cnt, int32_t *cidx, int *status) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    uint64_t a, b;
    pack_row(pc, perm[seg_off[g]], a, b);
    const int64_t q = find_key(slo, shi, cnt, a, b);
    if (q < 0) atomicOr(status, kStUnmatched);
    cidx[g] = (int32_t)(q < 0 ? 0 : q);
}

// ---------------------------------------------------------------------------
// Count queries (Algorithm 2)
// ---------------------------------------------------------------------------

constexpr int kMaxKids = kMaxChildren;
struct KidCounts {
    const int32_t *cidx[kMaxKids];
    const int64_t *phi_down[kMaxKids];
    uint64_t *acc[kMaxKids];
    int32_t k;
};

// a * b, with the overflow bit raised unless the product stays below 2^53
__device__ __forceinline__ uint64_t mul_exact(uint64_t a, uint64_t b, int *status) {
    const uint64_t hi = __umul64hi(a, b), lo = a * b;
    if (hi != 0 || lo >= kExact) atomicOr(status, kStOverflow);
    return lo;
}

// rows per key group, Theta (rows x the children's Phi-down of its keys)
__global__ void k_theta(const int64_t *seg_off, int64_t G, KidCounts kc, int64_t *theta, int *status) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    uint64_t th = (uint64_t)(seg_off[g + 1] - seg_off[g]);
    for (int c = 0; c < kc.k; ++c) th = mul_exact(th, (uint64_t)kc.phi_down[c][kc.cidx[c][g]], status);
    theta[g] = (int64_t)th;
}

// Phi-down of every parent group: the sum of Theta over its key groups
// (one wave per group, 128-bit partial sums)
__global__ void k_phi_down(const int64_t *theta, const int64_t *par_off, int64_t P, int64_t *phi_down, int *status) {
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= P) return;
    unsigned __int128 acc = 0;
    for (int64_t g = par_off[q] + lane; g < par_off[q + 1]; g += 64) acc += (uint64_t)theta[g];
    for (int s = 32; s > 0; s >>= 1) {
        const uint64_t lo = (uint64_t)acc, hi = (uint64_t)(acc >> 64);
        const uint64_t olo = __shfl_down(lo, s), ohi = __shfl_down(hi, s);
        acc += ((unsigned __int128)ohi << 64) | olo;
    }
    if (lane == 0) {
        if (acc >= kExact) atomicOr(status, kStOverflow);
        phi_down[q] = (int64_t)(uint64_t)acc;
    }
}

// full join size of every key group (Phi-up of its parent group times its
// Theta), Phi-circ = that / rows, and its share of every child's up-count
__global__ void k_top_down(const int64_t *seg_off, const int64_t *theta, const int64_t *gpar, const int64_t *phi_up,
                           int64_t G, KidCounts kc, int64_t *phi_circ, int *status) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const uint64_t up = phi_up ? (uint64_t)phi_up[gpar[g]] : 1;
    const uint64_t f = mul_exact(up, (uint64_t)theta[g], status);
    phi_circ[g] = (int64_t)(f / (uint64_t)(seg_off[g + 1] - seg_off[g]));
    for (int c = 0; c < kc.k; ++c) atomicAdd((unsigned long long *)&kc.acc[c][kc.cidx[c][g]], (unsigned long long)f);
}

__global__ void k_phi_up(const uint64_t *acc, const int64_t *phi_down, int64_t P, int64_t *phi_up, int *status) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const uint64_t d = (uint64_t)phi_down[q];
    if (acc[q] % d != 0) atomicOr(status, kStInexact);
    phi_up[q] = (int64_t)(acc[q] / d);
}

// sum of Theta over the root's key groups (the join size), 128-bit
__global__ void k_sum_u128(const int64_t *v, int64_t n, unsigned long long *out_lo, unsigned long long *out_hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long x = (unsigned long long)v[i];
    const unsigned long long old = atomicAdd(out_lo, x);
    if (old + x < old) atomicAdd(out_hi, 1ull);
}

// ---------------------------------------------------------------------------
// First level of a head/tail task
// ---------------------------------------------------------------------------

// piece starts: every chunk start (multiple of the tile) and group start
__global__ void k_piece_flags(const int64_t *group_flags, int64_t n, int64_t tile, int64_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (i % tile == 0 || group_flags[i]) ? 1 : 0;
}

__global__ void k_pid(const int64_t *excl, const int64_t *flags, int64_t n, int32_t *pid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pid[i] = (int32_t)(excl[i] + flags[i] - 1);
}

__global__ void k_chunks(const int32_t *pid, int64_t n, int64_t tile, int64_t nchunks, int64_t npieces, int64_t *cs,
                         int32_t *cp) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nchunks) return;
    cs[c] = c < nchunks ? c * tile : n;
    cp[c] = c < nchunks ? pid[c * tile] : (int32_t)npieces;
}

// the group of every piece (group id at its first item), and its count
// (unit items: its length; weighted: the sum of its items' counts, from the
// exclusive scan `wexcl` of the counts with wexcl[n] = total)
__global__ void k_piece_meta(const int64_t *pstart, int64_t npieces, const int64_t *gid, const int64_t *wexcl,
                             int64_t *pgroup, int64_t *pcount) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npieces) return;
    pgroup[q] = gid[pstart[q]];
    pcount[q] = wexcl ? wexcl[pstart[q + 1]] - wexcl[pstart[q]] : pstart[q + 1] - pstart[q];
}

// unit tails: scale sqrt(Phi-circ) of every piece's key group (one padding entry)
__global__ void k_phi_piece(const int64_t *pgroup, int64_t npieces, const int64_t *phi_circ, double *phi) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < npieces) phi[q] = __dsqrt_rn((double)phi_circ[pgroup[q]]);
    if (q == npieces) phi[q] = 0.0;
}

// weighted tails (Definition 2 with counts): W = count before the item in its
// piece, c = its count, ph = sqrt(Phi-up) of its parent group:
//   alpha = ph sqrt(W) / (sqrt(c) sqrt(W + c)),  beta = ph sqrt(c) / (sqrt(W) sqrt(W + c))
__global__ void k_alpha_beta(const int64_t *wexcl, const int64_t *theta, const int32_t *pid, const int64_t *pstart,
                             const int64_t *pgroup, const int64_t *phi_up, int64_t n, double *alpha, double *beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t q = pid[i];
    const int64_t W = wexcl[i] - wexcl[pstart[q]], c = theta[i];
    if (W == 0) {
        alpha[i] = 0.0;
        beta[i] = 0.0;
        return;
    }
    const double ph = __dsqrt_rn((double)phi_up[pgroup[q]]);
    const double sW = __dsqrt_rn((double)W), sc = __dsqrt_rn((double)c), sWi = __dsqrt_rn((double)(W + c));
    alpha[i] = __ddiv_rn(__dmul_rn(ph, sW), __dmul_rn(sc, sWi));
    beta[i] = __ddiv_rn(__dmul_rn(ph, sc), __dmul_rn(sW, sWi));
}

__global__ void k_sqrt_i64(const int64_t *v, int64_t n, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __dsqrt_rn((double)v[i]);
}

__global__ void k_inv_sqrt_i64(const int64_t *v, int64_t n, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __ddiv_rn(1.0, __dsqrt_rn((double)v[i]));
}

// join multipliers: own[g] = prod of the children's Phi-down, mult_c[g] =
// rows x prod over the other children (exact integers below 2^53)
__global__ void k_join_mults(const int64_t *seg_off, int64_t G, KidCounts kc, double *own, double **mult) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    uint64_t prod = 1;
    for (int c = 0; c < kc.k; ++c) prod *= (uint64_t)kc.phi_down[c][kc.cidx[c][g]];
    own[g] = (double)(int64_t)prod;
    for (int c = 0; c < kc.k; ++c) {
        uint64_t m = (uint64_t)(seg_off[g + 1] - seg_off[g]);
        for (int c2 = 0; c2 < kc.k; ++c2)
            if (c2 != c) m *= (uint64_t)kc.phi_down[c2][kc.cidx[c2][g]];
        mult[c][g] = (double)(int64_t)m;
    }
}

__global__ void k_count_into(const int32_t *idx, int64_t n, int64_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd((unsigned long long *)&cnt[idx[i]], 1ull);
}

__global__ void k_i32_from_i64(const int64_t *src, int64_t n, int32_t *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (int32_t)src[i];
}

__global__ void k_u64_from_i32(const int32_t *src, int64_t n, uint64_t *dst, int64_t *pay) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = (uint64_t)(uint32_t)src[i];
    pay[i] = i;
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------

#define DP_LAUNCH(kernel, n, ...) hipLaunchKernelGGL(kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, __VA_ARGS__)

struct Dev {
    figaro_plan_s *p;
    hipStream_t s;
    Temp T;
    std::vector<int32_t> attrs;              // distinct attribute ids
    std::vector<int> bits;                   // per attribute index
    std::vector<std::vector<int32_t *>> ids; // per relation, per key column: dense ids [m_in]
    std::vector<uint8_t *> alive;
    // per relation after segmentation
    std::vector<int> full_bits, xp_bits;
    std::vector<uint64_t *> plo, phi;       // parent-group keys [P] (X_p part)
    std::vector<int64_t *> gpar;            // parent group of every key group [G]
    std::vector<int64_t *> pflags;          // parent-group starts over key groups [G]
    std::vector<int64_t *> rows_seg_flags;  // key-group starts over plan rows [m]
    std::vector<std::vector<int32_t *>> cidx;
    std::vector<uint64_t *> acc;             // up-count accumulators [P]
    int *status = nullptr;

    int attr_index(int32_t a) const { return (int)(std::lower_bound(attrs.begin(), attrs.end(), a) - attrs.begin()); }
    int key_pos(int i, int32_t a) const {
        const auto &at = p->rel[i].attrs;
        for (size_t q = 0; q < at.size(); ++q)
            if (at[q] == a) return (int)q;
        return -1;
    }
    std::vector<int32_t> shared(int i, int j) const {
        std::vector<int32_t> out;
        for (int32_t a : p->rel[i].attrs)
            if (key_pos(j, a) >= 0) out.push_back(a);
        std::sort(out.begin(), out.end());
        return out;
    }
    // dense-id columns of relation i for the attributes `as` packed in that
    // order, first highest; total bits in *total
    PackCols packer(int i, const std::vector<int32_t> &as, int *total) const {
        PackCols pc{};
        int tb = 0;
        for (int32_t a : as) tb += bits[attr_index(a)];
        *total = tb;
        int sh = tb;
        pc.k = (int32_t)as.size();
        for (size_t q = 0; q < as.size(); ++q) {
            sh -= bits[attr_index(as[q])];
            pc.col[q] = ids[i][key_pos(i, as[q])];
            pc.shift[q] = sh;
        }
        return pc;
    }
};

int64_t *segment_ids(Dev &D, const int64_t *flags, int64_t n) {
    hipStream_t s = D.s;
    int64_t *ex = D.T.get<int64_t>(n), *id = D.T.get<int64_t>(n);
    scan_excl(flags, ex, n, D.T, s);
    DP_LAUNCH(k_seg_id, n, ex, flags, n, id);
    return id;
}

figaro_status check_launch(figaro_plan_s *p) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FIGARO_OK : set_error(p, FIGARO_EHIP, std::string("plan kernel: ") + hipGetErrorString(e));
}

// distinct sorted packed keys of the alive rows of relation j on attributes
// `as` (lo, hi arrays; hi null when they fit 64 bits); returns their count
int64_t distinct_keys(Dev &D, int j, const std::vector<int32_t> &as, uint64_t **olo, uint64_t **ohi) {
    hipStream_t s = D.s;
    const int64_t m = D.p->rel[j].m_in;
    int tb = 0;
    const PackCols pc = D.packer(j, as, &tb);
    int64_t *flags = D.T.get<int64_t>(m), *rows = D.T.get<int64_t>(m);
    DP_LAUNCH(k_alive_flags, m, D.alive[j], m, flags, 0);
    const int64_t n = compact(flags, m, rows, D.T, s);
    uint64_t *lo = D.T.get<uint64_t>(n), *hi = tb > 64 ? D.T.get<uint64_t>(n) : nullptr;
    int64_t *pay = D.T.get<int64_t>(n);
    DP_LAUNCH(k_pack, n, pc, rows, n, lo, hi, pay);
    radix_sort(lo, hi, pay, n, tb, D.T, s);
    int64_t *ch = D.T.get<int64_t>(n), *at = D.T.get<int64_t>(n);
    DP_LAUNCH(k_change_flags, n, lo, hi, n, 0, ch);
    const int64_t cnt = compact(ch, n, at, D.T, s);
    uint64_t *dlo = D.T.get<uint64_t>(cnt), *dhi = hi ? D.T.get<uint64_t>(cnt) : nullptr;
    DP_LAUNCH(k_gather_keys, cnt, lo, hi, at, cnt, dlo, dhi);
    *olo = dlo;
    *ohi = dhi;
    return cnt;
}

// first level of a head/tail task on the device, then the upper levels on
// the host.  group_flags: [items] group starts; gid: [items] group id;
// wcounts: per-item counts (null: unit items); phi_src: the per-group count
// whose square root scales the tails (Phi-circ per key group for unit
// items, Phi-up per parent group for weighted ones).
figaro_status device_task(Dev &D, Task &T, int64_t items, int64_t ngroups, const int64_t *group_flags,
                          const int64_t *gid, const int64_t *wcounts, const int64_t *phi_src, int tile) {
    figaro_plan_s *p = D.p;
    hipStream_t s = D.s;
    Level L;
    L.items = items;
    L.unit = wcounts == nullptr;
    L.variant = T.variant;
    int64_t *flags = D.T.get<int64_t>(items), *excl = D.T.get<int64_t>(items);
    DP_LAUNCH(k_piece_flags, items, group_flags, items, (int64_t)tile, flags);
    scan_excl(flags, excl, items, D.T, s);
    const int64_t npieces = read_i64(excl + items - 1, s) + read_i64(flags + items - 1, s);
    if (npieces >= (int64_t(1) << 31) - 2)
        return set_error(p, FIGARO_EUNSUPPORTED, "too many pieces in one head/tail level");
    L.npieces = npieces;
    L.nchunks = (items + tile - 1) / tile;
    if (dev_alloc(p, (void **)&L.d_pid, sizeof(int32_t) * (size_t)items) != hipSuccess ||
        dev_alloc(p, (void **)&L.d_piece_start, sizeof(int64_t) * (size_t)(npieces + 1)) != hipSuccess ||
        dev_alloc(p, (void **)&L.d_chunk_start, sizeof(int64_t) * (size_t)(L.nchunks + 1)) != hipSuccess ||
        dev_alloc(p, (void **)&L.d_chunk_piece0, sizeof(int32_t) * (size_t)(L.nchunks + 1)) != hipSuccess)
        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    DP_LAUNCH(k_pid, items, excl, flags, items, L.d_pid);
    DP_LAUNCH(k_compact, items, flags, excl, items, L.d_piece_start);
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, L.d_piece_start + npieces, items);
    DP_LAUNCH(k_chunks, L.nchunks + 1, L.d_pid, items, (int64_t)tile, L.nchunks, npieces, L.d_chunk_start,
              L.d_chunk_piece0);
    // exclusive scan of the counts with the total at [items]
    int64_t *wexcl = nullptr;
    if (wcounts) {
        int64_t *pad = D.T.get<int64_t>(items + 1);
        DP_LAUNCH(k_copy_i64, items, wcounts, pad, items);
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, pad + items, (int64_t)0);
        wexcl = D.T.get<int64_t>(items + 1);
        scan_excl(pad, wexcl, items + 1, D.T, s);
    }
    int64_t *pgroup = D.T.get<int64_t>(npieces), *pcount = D.T.get<int64_t>(npieces);
    DP_LAUNCH(k_piece_meta, npieces, L.d_piece_start, npieces, gid, wexcl, pgroup, pcount);
    if (wcounts) {
        if (dev_alloc(p, (void **)&L.d_alpha, sizeof(double) * (size_t)items) != hipSuccess ||
            dev_alloc(p, (void **)&L.d_beta, sizeof(double) * (size_t)items) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        DP_LAUNCH(k_alpha_beta, items, wexcl, wcounts, L.d_pid, L.d_piece_start, pgroup, phi_src, items, L.d_alpha,
                  L.d_beta);
    } else {
        if (dev_alloc(p, (void **)&L.d_phi_piece, sizeof(double) * (size_t)(npieces + 1)) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        DP_LAUNCH(k_phi_piece, npieces + 1, pgroup, npieces, phi_src, L.d_phi_piece);
    }
    if (dev_alloc(p, (void **)&L.d_pieces, sizeof(double) * (size_t)T.ncols * (size_t)npieces) != hipSuccess ||
        dev_alloc(p, (void **)&L.d_gpieces, sizeof(double) * (size_t)T.ncols * (size_t)npieces) != hipSuccess)
        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
    L.waves = (int32_t)std::max<int64_t>(1, std::min<int64_t>(L.nchunks, p->waves_cap));
    figaro_status st = check_launch(p);
    if (st != FIGARO_OK) return st;
    T.levels.push_back(L);
    if (npieces == ngroups) return FIGARO_OK;
    // the upper levels (items: the pieces) on the host
    std::vector<int64_t> hg(npieces), hc(npieces);
    std::vector<double> phi(ngroups);
    double *dphi = D.T.get<double>(ngroups);
    DP_LAUNCH(k_sqrt_i64, ngroups, phi_src, ngroups, dphi);
    if (hipMemcpyAsync(hg.data(), pgroup, sizeof(int64_t) * npieces, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hc.data(), pcount, sizeof(int64_t) * npieces, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(phi.data(), dphi, sizeof(double) * ngroups, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(p, FIGARO_EHIP, "reading the first level's pieces failed");
    std::vector<int64_t> goff(ngroups + 1, 0);
    for (int64_t q = 0; q < npieces; ++q) goff[hg[q] + 1]++;
    for (int64_t g = 0; g < ngroups; ++g) goff[g + 1] += goff[g];
    return build_task_levels(p, T, 1, npieces, goff, hc, false, phi, tile);
}

}  // namespace

figaro_status build_keys_on_device(figaro_plan_s *p, const figaro_relation_desc *rels, hipStream_t s) {
    Dev D;
    D.p = p;
    D.s = s;
    const int r = p->r;
    for (int i = 0; i < r; ++i) D.attrs.insert(D.attrs.end(), p->rel[i].attrs.begin(), p->rel[i].attrs.end());
    std::sort(D.attrs.begin(), D.attrs.end());
    D.attrs.erase(std::unique(D.attrs.begin(), D.attrs.end()), D.attrs.end());
    D.bits.assign(D.attrs.size(), 1);
    D.ids.assign(r, {});
    for (int i = 0; i < r; ++i) {
        D.ids[i].assign(p->rel[i].attrs.size(), nullptr);
        for (auto &c : D.ids[i]) c = D.T.get<int32_t>(p->rel[i].m_in);
    }
    D.status = D.T.get<int>(1);
    if (hipMemsetAsync(D.status, 0, sizeof(int), s) != hipSuccess) return set_error(p, FIGARO_EHIP, "hipMemsetAsync");
    // ---- dictionary encoding: dense ids in increasing key order over every
    // relation holding the attribute
    for (size_t ai = 0; ai < D.attrs.size(); ++ai) {
        const int32_t a = D.attrs[ai];
        int64_t N = 0;
        for (int i = 0; i < r; ++i)
            if (D.key_pos(i, a) >= 0) N += p->rel[i].m_in;
        if (N == 0) continue;
        unsigned long long *mm = D.T.get<unsigned long long>(2);
        const unsigned long long init[2] = {~0ull, 0ull};
        if (hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "hipMemcpyAsync");
        for (int i = 0; i < r; ++i) {
            const int kp = D.key_pos(i, a);
            if (kp < 0 || p->rel[i].m_in == 0) continue;
            const char *col = (const char *)rels[i].key_cols + (size_t)kp * rels[i].rows * rels[i].key_dtype;
            DP_LAUNCH(k_minmax, p->rel[i].m_in, (const void *)col, rels[i].key_dtype, p->rel[i].m_in, mm, mm + 1);
        }
        unsigned long long hmm[2];
        if (hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "reading a key range failed");
        const uint64_t range = hmm[1] - hmm[0];
        int rbits = 0;
        while (rbits < 64 && (range >> rbits) != 0) ++rbits;
        uint64_t *v = D.T.get<uint64_t>(N);
        int64_t *pay = D.T.get<int64_t>(N);
        int64_t at = 0;
        for (int i = 0; i < r; ++i) {
            const int kp = D.key_pos(i, a);
            if (kp < 0) continue;
            const char *col = (const char *)rels[i].key_cols + (size_t)kp * rels[i].rows * rels[i].key_dtype;
            DP_LAUNCH(k_offset_values, p->rel[i].m_in, (const void *)col, rels[i].key_dtype, p->rel[i].m_in,
                      (uint64_t)hmm[0], at, v, pay);
            at += p->rel[i].m_in;
        }
        uint64_t *hi = nullptr;
        radix_sort(v, hi, pay, N, rbits, D.T, s);
        int64_t *ch = D.T.get<int64_t>(N), *ex = D.T.get<int64_t>(N);
        DP_LAUNCH(k_change_flags, N, v, (const uint64_t *)nullptr, N, 0, ch);
        scan_excl(ch, ex, N, D.T, s);
        int32_t *cat = D.T.get<int32_t>(N);
        DP_LAUNCH(k_scatter_ids, N, ex, ch, pay, N, cat);
        const int64_t distinct = read_i64(ex + N - 1, s) + read_i64(ch + N - 1, s);
        int b = 1;
        while ((int64_t(1) << b) < distinct) ++b;
        D.bits[ai] = b;
        at = 0;
        for (int i = 0; i < r; ++i) {
            const int kp = D.key_pos(i, a);
            if (kp < 0) continue;
            if (p->rel[i].m_in > 0 &&
                hipMemcpyAsync(D.ids[i][kp], cat + at, sizeof(int32_t) * (size_t)p->rel[i].m_in,
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
                return set_error(p, FIGARO_EHIP, "hipMemcpyAsync");
            at += p->rel[i].m_in;
        }
    }
    for (int i = 0; i < r; ++i) {
        int tb = 0;
        (void)D.packer(i, p->rel[i].attrs, &tb);
        if (tb > 127)
            return set_error(p, FIGARO_EUNSUPPORTED,
                             "composite key of relation " + std::to_string(i) + " needs more than 127 bits");
    }
    figaro_status st = check_launch(p);
    if (st != FIGARO_OK) return st;
    // ---- semi-join reduction: bottom-up, then top-down
    D.alive.assign(r, nullptr);
    for (int i = 0; i < r; ++i) {
        D.alive[i] = D.T.get<uint8_t>(p->rel[i].m_in);
        DP_LAUNCH(k_fill_u8, p->rel[i].m_in, D.alive[i], p->rel[i].m_in, (uint8_t)1);
    }
    auto semijoin = [&](int keep, int probe) -> figaro_status {
        const std::vector<int32_t> sh = D.shared(keep, probe);
        uint64_t *slo = nullptr, *shi = nullptr;
        const int64_t cnt = distinct_keys(D, probe, sh, &slo, &shi);
        int tb = 0;
        const PackCols pc = D.packer(keep, sh, &tb);
        const int64_t m = p->rel[keep].m_in;
        if (cnt == 0) {
            DP_LAUNCH(k_fill_u8, m, D.alive[keep], m, (uint8_t)0);
        } else {
            DP_LAUNCH(k_semijoin, m, pc, D.alive[keep], m, slo, shi, cnt);
        }
        return check_launch(p);
    };
    for (int v : p->post)
        if (p->rel[v].parent >= 0 && (st = semijoin(p->rel[v].parent, v)) != FIGARO_OK) return st;
    for (auto it = p->post.rbegin(); it != p->post.rend(); ++it)
        if (p->rel[*it].parent >= 0 && (st = semijoin(*it, p->rel[*it].parent)) != FIGARO_OK) return st;
    // ---- sort, segment, parent groups
    D.full_bits.assign(r, 0);
    D.xp_bits.assign(r, 0);
    D.plo.assign(r, nullptr);
    D.phi.assign(r, nullptr);
    D.gpar.assign(r, nullptr);
    D.pflags.assign(r, nullptr);
    D.rows_seg_flags.assign(r, nullptr);
    for (int i = 0; i < r; ++i) {
        auto &R = p->rel[i];
        R.host_arrays = false;
        const std::vector<int32_t> xp = R.parent >= 0 ? D.shared(i, R.parent) : std::vector<int32_t>{};
        std::vector<int32_t> rest;
        for (int32_t a : R.attrs)
            if (std::find(xp.begin(), xp.end(), a) == xp.end()) rest.push_back(a);
        std::sort(rest.begin(), rest.end());
        std::vector<int32_t> order = xp;
        order.insert(order.end(), rest.begin(), rest.end());
        int fb = 0, xb = 0;
        const PackCols pc = D.packer(i, order, &fb);
        (void)D.packer(i, xp, &xb);
        D.full_bits[i] = fb;
        D.xp_bits[i] = xb;
        const int64_t m_in = R.m_in;
        int64_t *af = D.T.get<int64_t>(m_in), *rows = D.T.get<int64_t>(m_in);
        DP_LAUNCH(k_alive_flags, m_in, D.alive[i], m_in, af, 0);
        const int64_t m = compact(af, m_in, rows, D.T, s);
        R.m = m;
        if (m == 0) return set_error(p, FIGARO_EEMPTY_JOIN, "the join is empty");
        uint64_t *lo = D.T.get<uint64_t>(m), *hi = fb > 64 ? D.T.get<uint64_t>(m) : nullptr;
        int64_t *pay = D.T.get<int64_t>(m);
        DP_LAUNCH(k_pack, m, pc, rows, m, lo, hi, pay);
        radix_sort(lo, hi, pay, m, fb, D.T, s);
        if (dev_alloc(p, (void **)&R.d_perm, sizeof(int64_t) * (size_t)std::max<int64_t>(m_in, 1)) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        DP_LAUNCH(k_copy_i64, m, pay, R.d_perm, m);
        if (m < m_in) {
            DP_LAUNCH(k_alive_flags, m_in, D.alive[i], m_in, af, 1);
            (void)compact(af, m_in, R.d_perm + m, D.T, s);
        }
        // key groups
        int64_t *sf = D.T.get<int64_t>(m);
        DP_LAUNCH(k_change_flags, m, lo, hi, m, 0, sf);
        D.rows_seg_flags[i] = sf;
        if (dev_alloc(p, (void **)&R.d_seg_off, sizeof(int64_t) * (size_t)(m + 1)) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        const int64_t G = compact(sf, m, R.d_seg_off, D.T, s);
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, R.d_seg_off + G, m);
        R.G = G;
        R.singleton = G == m;
        // parent groups: changes of the X_p part (the high bits) between key groups
        if (R.parent >= 0) {
            uint64_t *glo = D.T.get<uint64_t>(G), *ghi = hi ? D.T.get<uint64_t>(G) : nullptr;
            DP_LAUNCH(k_gather_keys, G, lo, hi, R.d_seg_off, G, glo, ghi);
            DP_LAUNCH(k_shift_keys, G, glo, ghi, G, fb - xb);
            uint64_t *ghi2 = xb > 64 ? ghi : nullptr;
            int64_t *pf = D.T.get<int64_t>(G);
            DP_LAUNCH(k_change_flags, G, glo, ghi2, G, 0, pf);
            if (dev_alloc(p, (void **)&R.d_par_off, sizeof(int64_t) * (size_t)(G + 1)) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            const int64_t P = compact(pf, G, R.d_par_off, D.T, s);
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, R.d_par_off + P, G);
            R.P = P;
            D.plo[i] = D.T.get<uint64_t>(P);
            D.phi[i] = ghi2 ? D.T.get<uint64_t>(P) : nullptr;
            DP_LAUNCH(k_gather_keys, P, glo, ghi2, R.d_par_off, P, D.plo[i], D.phi[i]);
            // parent group of every key group
            D.gpar[i] = segment_ids(D, pf, G);
            D.pflags[i] = pf;
        } else {
            R.P = 0;
        }
        if ((st = check_launch(p)) != FIGARO_OK) return st;
    }
    // ---- child index of every key group
    D.cidx.assign(r, {});
    for (int i = 0; i < r; ++i) {
        auto &R = p->rel[i];
        for (int c : R.children) {
            int tb = 0;
            const PackCols pc = D.packer(i, D.shared(c, i), &tb);   // the child's X_p, its packing
            int32_t *ci = nullptr;
            if (dev_alloc(p, (void **)&ci, sizeof(int32_t) * (size_t)R.G) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            DP_LAUNCH(k_child_index, R.G, pc, R.d_perm, R.d_seg_off, R.G, D.plo[c], D.phi[c], p->rel[c].P, ci,
                      D.status);
            D.cidx[i].push_back(ci);
        }
    }
    // ---- count queries (Algorithm 2): Theta and Phi-down bottom-up
    auto kids = [&](int v) {
        KidCounts kc{};
        const auto &R = p->rel[v];
        kc.k = (int32_t)R.children.size();
        for (size_t c = 0; c < R.children.size() && c < (size_t)kMaxKids; ++c) {
            kc.cidx[c] = D.cidx[v][c];
            kc.phi_down[c] = p->rel[R.children[c]].d_phi_down;
        }
        return kc;
    };
    for (int v : p->post) {
        auto &R = p->rel[v];
        if (R.children.size() > (size_t)kMaxChildren)
            return set_error(p, FIGARO_EUNSUPPORTED, "more than 16 children of one relation");
        if (dev_alloc(p, (void **)&R.d_theta, sizeof(int64_t) * (size_t)R.G) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        DP_LAUNCH(k_theta, R.G, R.d_seg_off, R.G, kids(v), R.d_theta, D.status);
        if (R.parent >= 0) {
            if (dev_alloc(p, (void **)&R.d_phi_down, sizeof(int64_t) * (size_t)R.P) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            hipLaunchKernelGGL(k_phi_down, dim3((unsigned)((R.P + 3) / 4)), dim3(kBlock), 0, s, R.d_theta,
                               R.d_par_off, R.P, R.d_phi_down, D.status);
        }
    }
    {
        auto &Rr = p->rel[p->root];
        unsigned long long *tot = D.T.get<unsigned long long>(2);
        DP_LAUNCH(k_zero_u64, 2, (uint64_t *)tot, (int64_t)2);
        DP_LAUNCH(k_sum_u128, Rr.G, Rr.d_theta, Rr.G, tot, tot + 1);
        unsigned long long h[2];
        if (hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "reading the join size failed");
        if (h[1] != 0 || h[0] >= kExact) return set_error(p, FIGARO_EOVERFLOW, "the join size reaches 2^53");
        p->join_rows = (double)(int64_t)h[0];
    }
    // top-down: full join sizes, Phi-circ, the children's Phi-up
    for (auto it = p->post.rbegin(); it != p->post.rend(); ++it) {
        const int v = *it;
        auto &R = p->rel[v];
        KidCounts kc = kids(v);
        for (size_t c = 0; c < R.children.size(); ++c) {
            const int64_t Pc = p->rel[R.children[c]].P;
            kc.acc[c] = D.T.get<uint64_t>(Pc);
            DP_LAUNCH(k_zero_u64, Pc, kc.acc[c], Pc);
        }
        if (dev_alloc(p, (void **)&R.d_phi_circ, sizeof(int64_t) * (size_t)R.G) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        DP_LAUNCH(k_top_down, R.G, R.d_seg_off, R.d_theta, D.gpar[v], R.parent >= 0 ? R.d_phi_up : nullptr, R.G, kc,
                  R.d_phi_circ, D.status);
        for (size_t c = 0; c < R.children.size(); ++c) {
            auto &C = p->rel[R.children[c]];
            if (dev_alloc(p, (void **)&C.d_phi_up, sizeof(int64_t) * (size_t)C.P) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            DP_LAUNCH(k_phi_up, C.P, kc.acc[c], C.d_phi_down, C.P, C.d_phi_up, D.status);
        }
    }
    {
        int hs = 0;
        if (hipMemcpyAsync(&hs, D.status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(p, FIGARO_EHIP, "reading the plan status failed");
        if ((st = check_launch(p)) != FIGARO_OK) return st;
        if (hs & kStOverflow) return set_error(p, FIGARO_EOVERFLOW, "a count query reaches 2^53");
        if (hs & kStUnmatched) return set_error(p, FIGARO_EINVAL, "internal: unmatched key after reduction");
        if (hs & kStInexact) return set_error(p, FIGARO_EINVAL, "internal: inexact division in the count queries");
    }
    // ---- subtree columns, scale factors, head/tail tasks
    const int32_t n = p->n;
    std::vector<std::vector<int32_t>> subtree_cols(r);
    for (int v : p->post) {
        auto &R = p->rel[v];
        std::vector<int32_t> cols;
        for (int c = 0; c < R.ncols; ++c) cols.push_back(R.col0 + c);
        for (int c : R.children) cols.insert(cols.end(), subtree_cols[c].begin(), subtree_cols[c].end());
        std::sort(cols.begin(), cols.end());
        subtree_cols[v] = cols;
        R.sub_cols = cols;
        R.nsub = (int32_t)cols.size();
        R.own_pos = (int32_t)(std::lower_bound(cols.begin(), cols.end(), R.col0) - cols.begin());
    }
    for (int v : p->post) {
        auto &R = p->rel[v];
        R.a2.variant = p->variant;
        const int tile_a2 = p->tile_items > 0 ? std::min(p->tile_items, tile_items_for(R.ncols, p->variant))
                                              : tile_items_for(R.ncols, p->variant);
        if (!R.singleton) {   // heads_and_tails of S_v: unit items, key groups
            R.a2.active = true;
            R.a2.ncols = R.ncols;
            R.a2.block_id = 3 * v + 0;
            for (int c = 0; c < R.ncols; ++c) R.a2.cols.push_back(R.col0 + c);
            int64_t *gid = segment_ids(D, D.rows_seg_flags[v], R.m);
            if ((st = device_task(D, R.a2, R.m, R.G, D.rows_seg_flags[v], gid, nullptr, R.d_phi_circ, tile_a2)) !=
                FIGARO_OK)
                return st;
            if ((st = finish_task(p, R.a2, n)) != FIGARO_OK) return st;
        }
        if (!R.children.empty()) {
            R.col_src.assign(R.nsub, -1);
            R.col_idx.assign(R.nsub, 0);
            for (int c = 0; c < R.ncols; ++c) {
                R.col_src[R.own_pos + c] = -1;
                R.col_idx[R.own_pos + c] = (int16_t)c;
            }
            std::vector<double *> mults(R.children.size(), nullptr);
            if (dev_alloc(p, (void **)&R.d_own_mult, sizeof(double) * (size_t)R.G) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            for (auto &m : mults)
                if (dev_alloc(p, (void **)&m, sizeof(double) * (size_t)R.G) != hipSuccess)
                    return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            double **dm = nullptr;
            if (dev_upload(p, &dm, mults) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            DP_LAUNCH(k_join_mults, R.G, R.d_seg_off, R.G, kids(v), R.d_own_mult, dm);
            for (size_t c = 0; c < R.children.size(); ++c) {
                std::vector<int32_t> pos;
                for (int32_t col : subtree_cols[R.children[c]])
                    pos.push_back((int32_t)(std::lower_bound(R.sub_cols.begin(), R.sub_cols.end(), col) -
                                            R.sub_cols.begin()));
                int32_t *dp = nullptr;
                if (dev_upload(p, &dp, pos) != hipSuccess) return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                for (size_t q = 0; q < pos.size(); ++q) {
                    R.col_src[pos[q]] = (int16_t)c;
                    R.col_idx[pos[q]] = (int16_t)q;
                }
                R.d_cidx.push_back(D.cidx[v][c]);
                R.d_mult.push_back(mults[c]);
                R.d_colpos.push_back(dp);
            }
            if (dev_upload(p, &R.d_col_src, R.col_src) != hipSuccess ||
                dev_upload(p, &R.d_col_idx, R.col_idx) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            // (the in-place view carries its column codes by value: at most
            // kMaxCols subtree columns)
            R.fuse_join = R.parent >= 0 && R.P < R.G && R.children.size() <= (size_t)kFuseMaxChildren &&
                          R.nsub <= kMaxCols && !p->separate_join;
            if (R.fuse_join)
                for (int ch : R.children) {
                    double *rm;
                    const auto &C = p->rel[ch];
                    if (dev_alloc(p, (void **)&rm, sizeof(double) * (size_t)C.P * (size_t)C.nsub) != hipSuccess)
                        return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                    R.d_sigma_rm.push_back(rm);
                }
            R.ld_s = (R.G + 15) / 16 * 16;
            if (dev_alloc(p, (void **)&R.d_s, sizeof(double) * (size_t)R.nsub * (size_t)R.ld_s) != hipSuccess ||
                dev_alloc(p, (void **)&R.d_gs, sizeof(double) * (size_t)R.nsub * (size_t)R.G) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            // inverse of the child index: parent key groups grouped by child
            // group, in increasing order within a group (stable sort)
            for (size_t c = 0; c < R.children.size(); ++c) {
                const int64_t Pc = p->rel[R.children[c]].P;
                int64_t *cnt = D.T.get<int64_t>(Pc + 1);
                DP_LAUNCH(k_zero_u64, Pc + 1, (uint64_t *)cnt, Pc + 1);
                DP_LAUNCH(k_count_into, R.G, D.cidx[v][c], R.G, cnt);
                int64_t *off = nullptr;
                int32_t *idx = nullptr;
                if (dev_alloc(p, (void **)&off, sizeof(int64_t) * (size_t)(Pc + 1)) != hipSuccess ||
                    dev_alloc(p, (void **)&idx, sizeof(int32_t) * (size_t)R.G) != hipSuccess)
                    return set_error(p, FIGARO_ENOMEM, "hipMalloc");
                scan_excl(cnt, off, Pc + 1, D.T, s);
                uint64_t *key = D.T.get<uint64_t>(R.G), *nohi = nullptr;
                int64_t *pay = D.T.get<int64_t>(R.G);
                DP_LAUNCH(k_u64_from_i32, R.G, D.cidx[v][c], R.G, key, pay);
                int kb = 1;
                while ((int64_t(1) << kb) < Pc) ++kb;
                radix_sort(key, nohi, pay, R.G, kb, D.T, s);
                DP_LAUNCH(k_i32_from_i64, R.G, pay, R.G, idx);
                R.d_inv_off.push_back(off);
                R.d_inv_idx.push_back(idx);
                // the chunking of long inverse lists is planned on the host
                std::vector<int64_t> off_h(Pc + 1);
                if (hipMemcpyAsync(off_h.data(), off, sizeof(int64_t) * (size_t)(Pc + 1), hipMemcpyDeviceToHost, s) !=
                        hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return set_error(p, FIGARO_EHIP, "copying the inverse child index offsets");
                if ((st = join_chunks(p, R, c, off_h)) != FIGARO_OK) return st;
            }
            if (R.parent >= 0 && R.P < R.G) {   // project_away_join_attributes: weighted items
                R.a4.active = true;
                R.a4.ncols = R.nsub;
                R.a4.block_id = 3 * v + 1;
                R.a4.cols = R.sub_cols;
                R.a4.variant = p->variant;
                const int tile_a4 = p->tile_items > 0 ? std::min(p->tile_items, tile_items_for(R.nsub, p->variant))
                                                      : tile_items_for(R.nsub, p->variant);
                if ((st = device_task(D, R.a4, R.G, R.P, D.pflags[v], D.gpar[v], R.d_theta, R.d_phi_up, tile_a4)) !=
                    FIGARO_OK)
                    return st;
                if ((st = finish_task(p, R.a4, n)) != FIGARO_OK) return st;
            }
        }
        if (R.parent < 0) {
            if (dev_alloc(p, (void **)&R.d_inv_sqrt_c, sizeof(double) * (size_t)R.G) != hipSuccess)
                return set_error(p, FIGARO_ENOMEM, "hipMalloc");
            DP_LAUNCH(k_inv_sqrt_i64, R.G, R.d_theta, R.G, R.d_inv_sqrt_c);
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(p, FIGARO_EHIP, "hipStreamSynchronize failed");
    return check_launch(p);
}

figaro_status enumeration_arrays(figaro_plan_s *p, hipStream_t s) {
    Temp T;
    for (auto &R : p->rel) {
        if (dev_alloc(p, (void **)&R.d_theta_excl, sizeof(int64_t) * (size_t)(R.G + 1)) != hipSuccess)
            return set_error(p, FIGARO_ENOMEM, "hipMalloc");
        int64_t *pad = T.get<int64_t>(R.G + 1);
        DP_LAUNCH(k_copy_i64, R.G, R.d_theta, pad, R.G);
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, pad + R.G, (int64_t)0);
        scan_excl(pad, R.d_theta_excl, R.G + 1, T, s);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(p, FIGARO_EHIP, "hipStreamSynchronize failed");
    return check_launch(p);
}

figaro_status fetch_host_arrays(figaro_plan_s *p, int32_t i) {
    auto &R = p->rel[i];
    if (R.host_arrays) return FIGARO_OK;
    auto get = [&](std::vector<int64_t> &dst, const int64_t *src, int64_t count) {
        dst.resize((size_t)count);
        return count == 0 || hipMemcpy(dst.data(), src, sizeof(int64_t) * (size_t)count, hipMemcpyDeviceToHost) ==
                                 hipSuccess;
    };
    bool ok = get(R.perm, R.d_perm, R.m_in) && get(R.seg_off, R.d_seg_off, R.G + 1) && get(R.theta, R.d_theta, R.G) &&
              get(R.phi_circ, R.d_phi_circ, R.G);
    if (ok && R.parent >= 0)
        ok = get(R.par_off, R.d_par_off, R.P + 1) && get(R.phi_up, R.d_phi_up, R.P) && get(R.phi_down, R.d_phi_down, R.P);
    if (!ok) return set_error(p, FIGARO_EHIP, "copying plan arrays to the host failed");
    R.rpk.resize((size_t)R.G);
    for (int64_t g = 0; g < R.G; ++g) R.rpk[g] = R.seg_off[g + 1] - R.seg_off[g];
    R.host_arrays = true;
    return FIGARO_OK;
}

}  // namespace figaro
