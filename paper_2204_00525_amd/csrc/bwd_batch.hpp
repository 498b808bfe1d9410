// Backward head/tail levels of independent tasks in one launch
// (backward.hip): task t owns workgroups [wg0[t], wg0[t + 1]).
#pragma once

#include "internal.hpp"

namespace figaro {

constexpr int kHelmertBwdBatch = 4;
struct HelmertBwdBatch {
    HelmertBwdArgs a[kHelmertBwdBatch];
    int32_t wg0[kHelmertBwdBatch + 1];
    int32_t count;
};

// Tile-shape class of a backward level (0: a wide level, never batched).
int helmert_bwd_shape_class(int ncols);
// One level of up to kHelmertBwdBatch tasks of one shape class and count
// mode, column-major outputs.
hipError_t launch_helmert_bwd_batch(const HelmertBwdBatch &b, bool unit, hipStream_t s);

}  // namespace figaro
