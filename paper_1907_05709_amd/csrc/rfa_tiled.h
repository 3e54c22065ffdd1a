// rfa_tiled.h -- launcher of the 2.5-D tiled step kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rfa_kernels.h"

namespace rfa {

struct TiledShape {
  int ty;        // waves (y rows) per work-group: 4, 8 or 16
  int xc;        // x planes per work-group
  int tiles_z, tiles_y, chunks_x;
  int nwg;       // work-groups per launch
};

TiledShape tiled_shape(Grid3 g, int ty, int xc);
// Whether a chunk of xc planes fits the kernel's 32-bit plane offsets.
bool tiled_fits(Grid3 g, int xc);
hipError_t launch_step_tiled(const TiledShape& s, Grid3 g, const StepBuffers& b,
                             const StepConst& K, hipStream_t st);

}  // namespace rfa
