// rfa_tiled.h -- launcher of the 2.5-D tiled step kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rfa_kernels.h"

namespace rfa {

// Store cache policy of a step launch.
enum StorePolicy { kPolicyBack = 0, kPolicyThrough = 1, kPolicyStream = 2 };

struct TiledShape {
  int ty;        // waves (y rows of the footprint) per work-group: 4, 8 or 16
  int xc;        // x planes per work-group
  int tiles_z, tiles_y, chunks_x;
  int nwg;       // work-groups per launch
};

// One grid of a batch: its arrays, per-dt tables and step constants, and
// the x-chunk length of its tiles.  Image 0 is the current image at batch
// parity 0; a step at parity p reads image p and writes image 1 - p.
struct BatchInstance {
  float* hi[2];
  float* lo[2];
  uint8_t* lab;
  const float* src;
  float* om;
  const float* perf;
  const Tables* tab;
  StepConst K;
  int n_classes;
  int nx, ny, nz;
  int xc;
};

// One work item of a batch step: tile (tz, ty) over x-chunk tx of an instance.
struct BatchItem {
  int inst, tz, ty, tx;
};

// One step of the items [first_item, first_item + n_items) of a batch, all
// of instances with (perf) or without a perfusion field: n_wg > 0 persistent
// work-groups of 64*ty threads walk the items, n_wg == 0 launches one
// work-group per item.  Items are 2.5-D tiles of tiled_shape (ty = 4 or 8)
// or, with flat, plane segments of flat_shape (ty = 8 or 16 waves, grids
// with nz <= flat_max_nz(ty)).  partials (nullable) receives 3 floats per
// item, indexed by item.
hipError_t launch_step_batch(int ty, bool flat, bool perf, const BatchInstance* inst,
                             const BatchItem* items, int first_item, int n_items, int n_wg,
                             int parity, float* partials, hipStream_t st);

TiledShape tiled_shape(Grid3 g, int ty, int xc);
// Flat plane segments of 64 ty voxels (tiles_z = segments per plane,
// tiles_y = 1) and the largest nz they support.
TiledShape flat_shape(Grid3 g, int ty, int xc);
int flat_max_nz(int ty);
// Whether a chunk of xc planes fits the kernel's 32-bit plane offsets.
bool tiled_fits(Grid3 g, int xc);
// store: StorePolicy of the launch's stores.
hipError_t launch_step_tiled(const TiledShape& s, Grid3 g, const StepBuffers& b,
                             const StepConst& K, int store, hipStream_t st);

// One step with zv (2 or 4) consecutive z voxels per lane, ty = 4 or 8;
// needs nz % zv == 0.
TiledShape wide_shape(Grid3 g, int zv, int ty, int xc);
bool wide_fits(Grid3 g, int zv, int xc);
hipError_t launch_step_wide(int zv, const TiledShape& s, Grid3 g, const StepBuffers& b,
                            const StepConst& K, int store, hipStream_t st);
// The same step writing only the temperature (hi, lo): the damage integral
// and class bytes are neither read nor written.  Valid without
// damage-coupled perfusion, where the temperature does not depend on them.
hipError_t launch_step_wide_temperature(int zv, const TiledShape& s, Grid3 g,
                                        const StepBuffers& b, const StepConst& K, int store,
                                        hipStream_t st);

// Two steps per launch (temporal blocking, ty = 8 or 16): tiles own
// 62 x (ty - 2) columns and recompute a one-voxel rim of the first step.
// The partials receive the sums of both steps.
TiledShape tiled2_shape(Grid3 g, int ty, int xc);
bool tiled2_fits(Grid3 g, int xc);
hipError_t launch_step_tiled2(const TiledShape& s, Grid3 g, const StepBuffers& b,
                              const StepConst& K, int store, hipStream_t st);

}  // namespace rfa
