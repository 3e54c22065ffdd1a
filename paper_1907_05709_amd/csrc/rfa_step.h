// rfa_step.h -- step scheduling: kernel choice, launch shape, launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rfa.h"
#include "rfa_kernels.h"
#include "rfa_tiled.h"

namespace rfa {

constexpr int kMaxDepth = 2;

enum StepKind { kStepNaive = 1, kStepTiled = 2 };

struct StepPlan {
  int kind = 0;    // StepKind
  int depth = 1;   // steps per launch (1, or 2 with the tiled kernel)
  int ty = 4;      // tile rows (y) per work-group (tiled)
  int xc = 1;      // x planes per work-group (tiled)
  int nwg = 0;     // work-groups per launch (stride of the partials)
  int zv = 1;      // consecutive z voxels per lane (tiled, one step per launch)
  int store = 0;   // StorePolicy of the step launches
  // one-step plan for step counts not divisible by depth (equal to the
  // plan itself when depth == 1)
  int one_kind = 0, one_ty = 4, one_xc = 1, one_nwg = 0, one_zv = 1;
};

StepPlan plan_naive(Grid3 g);
StepPlan plan_tiled(Grid3 g, int ty, int xc);
StepPlan plan_tiled2(Grid3 g, int ty, int xc);
StepPlan plan_wide(Grid3 g, int zv, int ty, int xc);
// The one-step plan that accompanies a plan.
StepPlan plan_one(const StepPlan& p);
// Heuristic plan from the options (kernel, depth, tile_y, tile_x, z_vec,
// store = 1 + StorePolicy; 0 = automatic).
StepPlan plan_default(Grid3 g, int kernel, int depth, int tile_y, int tile_x, int zv,
                      int store = 0);
// Candidate plans for tuning (depth 1, and depth 2 if max_depth >= 2).
int plan_candidates(Grid3 g, int max_depth, StepPlan* out, int max_out);
// Largest partial stride any plan of this grid can need.
int plan_max_wg(Grid3 g);

struct StepState {
  float** hi;       // [2] ping-pong
  float** lo;       // [2]
  int* cur;         // index of the current image
  uint8_t* lab;
  const float* src;
  float* om;
  const float* perf;
  const Tables* tab;
  int n_classes;
  // Trajectory mode (traj not null, one-step plans only): the hi image of
  // step *traj_t is read from traj[*traj_t] and written to traj[*traj_t + 1]
  // (images of traj_n voxels); lo keeps ping-ponging in lo[2].
  float* traj = nullptr;
  int* traj_t = nullptr;
  size_t traj_n = 0;
};

// One launch of the plan (plan.depth steps) from b's input to its output image.
hipError_t launch_plan(Grid3 g, const StepPlan& plan, const StepBuffers& b, const StepConst& K,
                       hipStream_t st);
// One step of a one-step plan where only the temperature must come out
// right (no damage-coupled perfusion): the wide kernel then skips the damage
// integral and the class bytes; other plans run their full step.
hipError_t launch_plan_temperature(Grid3 g, const StepPlan& plan, const StepBuffers& b,
                                   const StepConst& K, hipStream_t st);

// Advance n_steps: n_steps / depth launches of the plan, then the rest with
// its one-step plan.  partials (nullable) has room for `slots` launches and
// is folded into dacc[3] every `slots` launches and at the end.  If events
// is not null, each block of `period` consecutive launches of the plan (the
// last one may be shorter) is bracketed by the event pair events[2j],
// events[2j+1] (j = 0, 1, ...; *n_timed receives the number of blocks and
// *n_launches the launches inside them); one-step launches are not timed.
rfa_status run_steps(Grid3 g, const StepPlan& plan, StepState& s, const StepConst& K,
                     int n_steps, float* partials, int slots, double* dacc,
                     hipEvent_t* events, int period, int* n_timed, int* n_launches,
                     hipStream_t st);

}  // namespace rfa
