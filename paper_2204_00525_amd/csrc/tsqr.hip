// The post-processing QR (section "Post-processing") on its own: R of a
// plain tall matrix, e.g. the matrix R0 of Theorem 6 that figaro_r0()
// materialises.  The levels are those of the forward pass: the first level
// folds the rows of A into one partial R per workgroup, every further level
// folds the stacked partial R's of the level before, and the last level (a
// single workgroup) sign-normalises.
//
// Two entry points share the levels and the kernels: figaro_tsqr() keeps
// the partial R's in a workspace the caller passes, figaro_tsqr_noalloc() in
// `scratch`, a static device array of this file (one copy per GPU, held
// until the process ends).  The number of workgroups of a level is capped
// so that two consecutive levels' partial R's fit half of that array each;
// a larger input gives the first level more tiles per workgroup rather than
// more workgroups, so the row count is not limited by the array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace figaro {
extern thread_local std::string g_thread_error;
}  // namespace figaro

using namespace figaro;

namespace {

// bound on the partial R's of two consecutive levels together
constexpr int64_t kScratchBytes = 8ll << 20;
constexpr int64_t kScratchDoubles = kScratchBytes / 8;
constexpr int kMaxDevices = 64;

// Device memory of the allocation-free entry point.  In host code this name
// is a stand-in for the device symbol, not a device address: the address of
// each GPU's copy comes from hipGetSymbolAddress() and is kept per device.
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

figaro_status fail(figaro_status st, const std::string &msg) {
    g_thread_error = msg;
    return st;
}

// Workgroups of one level: enough to fill the chip, capped so that the
// partial R's of two consecutive levels fit half of the static array each.
int64_t max_workgroups(int32_t n) {
    return std::max<int64_t>(1, std::min<int64_t>(4096, kScratchDoubles / 2 / ((int64_t)n * n)));
}

struct Levels {
    std::vector<DenseLevel> lv;
    int64_t buf_rows[2] = {0, 0};   // rows of the two ping-pong buffers
};

// Level l reads A (l = 0) or buffer (l - 1) % 2 and writes buffer l % 2, or R
// at the last level.  Narrow matrices (n <= 40) fold one tile (or one tile per
// wave) per workgroup at every level above the first, wide ones four; the
// last level holds at most one such step (eight for wide matrices).
Levels plan_levels(int64_t rows, int32_t n) {
    Levels L;
    const int64_t step = (int64_t)dense_waves_per_block(n) * dense_tile_rows_for(n, 0);
    const bool wide = n > kFusedMaxCols;
    const int64_t mid_tpw = wide ? 4 : 1, final_tiles = wide ? 8 : 1;
    const int64_t wmax = max_workgroups(n);
    int64_t cur = rows;
    for (int l = 0;; ++l) {
        DenseLevel D;
        D.rows = cur;
        if (cur <= final_tiles * step) {
            D.waves = 1;
            D.tiles_per_wave = std::max<int64_t>(1, (cur + step - 1) / step);
            L.lv.push_back(D);
            break;
        }
        int64_t w = std::min<int64_t>(wmax, (cur + mid_tpw * step - 1) / (mid_tpw * step));
        D.tiles_per_wave = (cur + w * step - 1) / (w * step);
        D.waves = (int32_t)((cur + D.tiles_per_wave * step - 1) / (D.tiles_per_wave * step));
        L.lv.push_back(D);
        cur = (int64_t)D.waves * n;
        L.buf_rows[l % 2] = std::max(L.buf_rows[l % 2], cur);
    }
    return L;
}

int64_t workspace_doubles(const Levels &L, int32_t n) { return (L.buf_rows[0] + L.buf_rows[1]) * (int64_t)n; }

figaro_status check(int64_t rows, int32_t n, const double *A, int64_t lda, const double *R) {
    if (n < 1 || n > kMaxCols) return fail(FIGARO_EUNSUPPORTED, "n must be between 1 and 128");
    // A may be NULL when it has no rows (nothing is read)
    if (rows < 0 || (!A && rows > 0) || !R || lda < std::max<int64_t>(rows, 1))
        return fail(FIGARO_EINVAL, "bad argument");
    return FIGARO_OK;
}

// Enqueue the levels; buf[0] and buf[1] hold buf_rows[0] and buf_rows[1]
// rows of n columns (leading dimensions = those row counts).
figaro_status run_levels(const Levels &L, int32_t n, const double *A, int64_t lda, double *R, double *buf0,
                         double *buf1, hipStream_t s) {
    double *buf[2] = {buf0, buf1};
    const double *in = A;
    int64_t ld_in = lda;
    for (size_t l = 0; l < L.lv.size(); ++l) {
        const DenseLevel &D = L.lv[l];
        DenseArgs a{};
        a.in = in;
        a.ld_in = ld_in;
        a.rows = D.rows;
        a.n = n;
        a.out = buf[l % 2];
        a.ld_out = std::max<int64_t>(L.buf_rows[l % 2], 1);
        a.waves = D.waves;
        a.tiles_per_wave = D.tiles_per_wave;
        a.final_r = R;
        hipError_t e = launch_dense(a, 0, s);
        if (e != hipSuccess) return fail(FIGARO_EHIP, std::string("dense TSQR launch: ") + hipGetErrorString(e));
        in = buf[l % 2];
        ld_in = a.ld_out;
    }
    return FIGARO_OK;
}

}  // namespace

extern "C" {

int64_t figaro_tsqr_workspace_bytes(int64_t rows, int32_t n) {
    if (n < 1 || n > kMaxCols || rows < 0) return -1;
    return 8 * workspace_doubles(plan_levels(rows, n), n);
}

figaro_status figaro_tsqr(int64_t rows, int32_t n, const double *A, int64_t lda, double *R, void *workspace,
                          int64_t workspace_bytes, hipStream_t stream) {
    figaro_status st = check(rows, n, A, lda, R);
    if (st != FIGARO_OK) return st;
    const Levels L = plan_levels(rows, n);
    const int64_t need = workspace_doubles(L, n);
    if (need > 0 && (!workspace || workspace_bytes < 8 * need))
        return fail(FIGARO_EINVAL, "workspace smaller than figaro_tsqr_workspace_bytes()");
    double *w = static_cast<double *>(workspace);
    return run_levels(L, n, A, lda, R, w, w ? w + L.buf_rows[0] * n : nullptr, stream);
}

figaro_status figaro_tsqr_noalloc(int64_t rows, int32_t n, const double *A, int64_t lda, double *R,
                                  hipStream_t stream) {
    figaro_status st = check(rows, n, A, lda, R);
    if (st != FIGARO_OK) return st;
    const Levels L = plan_levels(rows, n);
    if (workspace_doubles(L, n) > kScratchDoubles)   // excluded by the workgroup cap
        return fail(FIGARO_EUNSUPPORTED, "partial R factors exceed the 8 MiB static scratch array");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FIGARO_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(FIGARO_EUNSUPPORTED, "device index beyond 63");
    double *base = nullptr;
    {
        // first call on this device (the current one): the address of its
        // copy of the array
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(FIGARO_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            g_scratch_ptr[dev] = static_cast<double *>(ptr);
        }
        base = g_scratch_ptr[dev];
    }
    return run_levels(L, n, A, lda, R, base, base + L.buf_rows[0] * n, stream);
}

}  // extern "C"
