// Kinematic bones with the linear-blend warm start of Sec. 8.2 (launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "viper_dev.h"

namespace viper {

// The bones moved from T_prev (device, [nb*12]) to T_cur (`cur`, HOST memory, [nb*12]; each
// [A | b], 3x4 row-major, FP64): delta_b = T_cur,b T_prev,b^-1, T_prev <- T_cur; then every
// pill with positive weight moves to sum_k w_k delta_{b_k} x / sum_k w_k (world coordinates;
// pinned pills too).  `pb` [2P] bone ids, `pw` [2P] weights (device; ids are read only where
// the weight is positive).  T_cur travels in the launch arguments, kBoneChunk bones per
// launch, so `cur` has been read when the call returns.
constexpr int kBoneChunk = 32;
template <class T>
hipError_t launch_bone_warm(const Dev<T>& d, int nb, const double* cur, double* prev, double* delta,
                            const int32_t* pb, const double* pw, hipStream_t st);

}  // namespace viper
