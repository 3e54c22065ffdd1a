// rfa_warp.h -- host-side launcher of the breathing-motion warp kernel
// (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rfa_kernels.h"

namespace rfa {

// out[x] = 37 + trilinear sample of the float-float excess temperature
// (hi, lo) at the voxel position x + s(x), s_a(x) = scale[a] * v_a(x)
// (+ scale2[a] * v2_a(x) when v2 is not null; voxels), clamped to the
// grid (Eq. (eq:breathing)), rounded once to float.  v and v2 are [3][n]
// (x, y, z components), n < 2^31; the factors are applied as float-float
// pairs (c_hi + c_lo), positions formed to ~2^-47 relative.
hipError_t launch_warp(Grid3 g, const float* hi, const float* lo, const float* v,
                       const double (&scale)[3], const float* v2, const double (&scale2)[3],
                       float* out, hipStream_t st);

}  // namespace rfa
