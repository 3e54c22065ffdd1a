// rfa_warp.h -- host-side launcher of the breathing-motion warp kernel
// (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rfa_kernels.h"

namespace rfa {

// out[x] = 37 + trilinear sample of the excess temperature hi at the voxel
// position x + s(x), s_a(x) = scale_a * v_a(x) (voxels), clamped to the grid
// (Eq. (eq:breathing)).  v is [3][n] (x, y, z components), n < 2^31.
hipError_t launch_warp(Grid3 g, const float* hi, const float* v, float scale_x, float scale_y,
                       float scale_z, float* out, hipStream_t st);

}  // namespace rfa
