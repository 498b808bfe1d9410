// Device helpers shared by the forward and backward kernels (wave64 lane
// movement with DPP, wave reductions, segmented scans).  Internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace figaro {
namespace {

constexpr int kWavesPerBlock = 4;

// s_waitcnt operand for "all vector memory operations done" (vmcnt 0,
// expcnt and lgkmcnt at their maxima)
constexpr int kWaitVm0 = 0x0F70;

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

__device__ __forceinline__ int64_t readlane64(int64_t v, int src) {
    const int lo = __builtin_amdgcn_readlane((int)(uint64_t)v, src);
    const int hi = __builtin_amdgcn_readlane((int)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Move a double across lanes with a DPP control (two 32-bit halves); lanes
// that a row mask disables keep `old`.
template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF, bool BOUND_CTRL = true>
__device__ __forceinline__ double dpp(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROW_MASK, BANK_MASK,
                                               BOUND_CTRL);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROW_MASK, BANK_MASK,
                                               BOUND_CTRL);
    return __hiloint2double(hi, lo);
}

// Whole-wave shifts by one lane with DPP (wave_shr:1 / wave_shl:1): lane l
// receives lane l-1 (resp. l+1); lane 0 (resp. 63) keeps its own value.
// Unlike a shuffle these stay in the vector ALU and never touch the LDS
// pipe.
__device__ __forceinline__ int wave_shr1(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int wave_shl1(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ double wave_shr1(double v) { return dpp<0x138, 0xF, 0xF, false>(v, v); }

// Sum over the 64 lanes with DPP moves: quad butterflies, half-row and row
// mirrors give every lane its 16-lane row sum; two row broadcasts then fold
// rows 0-2 into row 3, and lane 63 is read into scalar registers.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp<0xB1>(v, 0.0);                  // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v, 0.0);                  // quad_perm [2,3,0,1]
    v += dpp<0x141>(v, 0.0);                 // row_half_mirror
    v += dpp<0x140>(v, 0.0);                 // row_mirror
    v += dpp<0x142, 0xA, 0xF, false>(v, 0.0);  // row_bcast:15 into rows 1, 3
    v += dpp<0x143, 0xC, 0xF, false>(v, 0.0);  // row_bcast:31 into rows 2, 3
    return lane_value(v, 63);
}

// Inclusive segmented scan over the lanes of per-lane aggregates acc[c]
// (segments start at lanes whose bit is set in `mask`), then converted to the
// exclusive carry into each lane (the inclusive value of the lane before).
// Within 16-lane rows: row_shr by 1, 2, 4, 8; across rows: row_bcast:15 into
// rows 1 and 3, row_bcast:31 into rows 2 and 3.  A lane adds what it
// receives only if no segment starts in the window between the source and
// itself, which is read off the ballot mask.
__device__ __forceinline__ bool flag_in(uint64_t mask, int lo, int hi) {
    // any bit of mask in lanes [lo, hi] (lo <= hi)
    const uint64_t width = (uint64_t)(hi - lo + 1);
    const uint64_t m = (width >= 64) ? ~0ull : ((1ull << width) - 1ull);
    return ((mask >> lo) & m) != 0ull;
}

template <int NB>
__device__ __forceinline__ void segmented_carry(double (&acc)[NB], uint64_t mask, int lane) {
    const int row0 = lane & ~15;
    const bool a1 = (lane - 1 >= row0) && !flag_in(mask, lane, lane);
    const bool a2 = (lane - 2 >= row0) && !flag_in(mask, lane - 1, lane);
    const bool a4 = (lane - 4 >= row0) && !flag_in(mask, lane - 3, lane);
    const bool a8 = (lane - 8 >= row0) && !flag_in(mask, lane - 7, lane);
    const int row = lane >> 4;
    const bool b15 = (row == 1 || row == 3) && !flag_in(mask, row0, lane);
    const bool b31 = (row >= 2) && !flag_in(mask, 32, lane);
    // 0/1 factors instead of selects (one FMA per step)
    const double m1 = a1 ? 1.0 : 0.0, m2 = a2 ? 1.0 : 0.0, m4 = a4 ? 1.0 : 0.0, m8 = a8 ? 1.0 : 0.0;
    const double m15 = b15 ? 1.0 : 0.0, m31 = b31 ? 1.0 : 0.0, m0 = (lane == 0) ? 0.0 : 1.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        double v = acc[c];
        v = fma(dpp<0x111>(v, 0.0), m1, v);   // row_shr:1
        v = fma(dpp<0x112>(v, 0.0), m2, v);   // row_shr:2
        v = fma(dpp<0x114>(v, 0.0), m4, v);   // row_shr:4
        v = fma(dpp<0x118>(v, 0.0), m8, v);   // row_shr:8
        v = fma(dpp<0x142, 0xA, 0xF, false>(v, 0.0), m15, v);
        v = fma(dpp<0x143, 0xC, 0xF, false>(v, 0.0), m31, v);
        acc[c] = wave_shr1(v) * m0;
    }
}

}  // namespace
}  // namespace figaro
