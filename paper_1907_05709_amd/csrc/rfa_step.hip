// rfa_step.hip -- step scheduling (kernel choice, launch shapes, launch loop).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rfa_step.h"

namespace rfa {

namespace {
constexpr int kTargetWg = 1536;  // ~6 work-groups per CU on 256 CUs
}

StepPlan plan_naive(Grid3 g) {
  StepPlan p;
  p.kind = kStepNaive;
  p.depth = 1;
  p.ty = 4;
  p.xc = 1;
  p.nwg = naive_wg_count(g);
  return p;
}

StepPlan plan_tiled(Grid3 g, int ty, int xc) {
  const TiledShape s = tiled_shape(g, ty, xc);
  StepPlan p;
  p.kind = kStepTiled;
  p.depth = 1;
  p.ty = ty;
  p.xc = xc;
  p.nwg = s.nwg;
  return p;
}

StepPlan plan_default(Grid3 g, int kernel, int tile_y, int tile_x) {
  if (kernel == kStepNaive || !tiled_fits(g, 4)) return plan_naive(g);
  int ty = tile_y;
  if (ty == 0) ty = g.ny >= 64 ? 8 : 4;
  int xc = tile_x;
  if (xc == 0) {
    const int tiles = ((g.nz + 63) / 64) * ((g.ny + ty - 1) / ty);
    const int chunks = std::max(1, (kTargetWg + tiles - 1) / tiles);
    xc = std::max(4, (g.nx + chunks - 1) / chunks);
  }
  xc = std::min(xc, g.nx);
  while (xc > 4 && !tiled_fits(g, xc)) xc /= 2;
  return plan_tiled(g, ty, xc);
}

int plan_candidates(Grid3 g, StepPlan* out, int max_out) {
  int n = 0;
  const int tys[] = {4, 8, 16};
  const int xcs[] = {4, 8, 16, 32, 64};
  for (int ty : tys)
    for (int xc : xcs) {
      if (n >= max_out) return n;
      if ((xc > g.nx && xc != 4) || !tiled_fits(g, std::min(xc, g.nx))) continue;
      out[n++] = plan_tiled(g, ty, std::min(xc, g.nx));
    }
  return n;
}

int plan_max_wg(Grid3 g) {
  int m = naive_wg_count(g);
  const int tys[] = {4, 8, 16};
  for (int ty : tys) m = std::max(m, tiled_shape(g, ty, 1).nwg);
  return m;
}

hipError_t launch_plan(Grid3 g, const StepPlan& plan, const StepBuffers& b, const StepConst& K,
                       hipStream_t st) {
  if (plan.kind == kStepNaive) return launch_step_naive(g, b, K, st);
  return launch_step_tiled(tiled_shape(g, plan.ty, plan.xc), g, b, K, st);
}

rfa_status run_steps(Grid3 g, const StepPlan& plan, StepState& s, const StepConst& K,
                     int n_steps, float* partials, int slots, double* dacc, hipEvent_t* events,
                     int period, int* n_timed, hipStream_t st) {
  int pending = 0;
  int timed = 0;
  for (int n = 0; n < n_steps; ++n) {
    StepBuffers b;
    b.hi_in = s.hi[*s.cur];
    b.lo_in = s.lo[*s.cur];
    b.hi_out = s.hi[1 - *s.cur];
    b.lo_out = s.lo[1 - *s.cur];
    b.lab = s.lab;
    b.src = s.src;
    b.omega = s.om;
    b.perf = s.perf;
    b.tab = s.tab;
    b.n_classes = s.n_classes;
    b.partials = partials ? partials + (size_t)pending * plan.nwg * 3 : nullptr;
    // Blocks of `period` consecutive launches are bracketed by one event pair
    // (the diagnostic reductions fall between blocks, never inside one).
    const bool open = events && (n % period) == 0;
    const bool close = events && ((n % period) == period - 1 || n == n_steps - 1);
    if (open && hipEventRecord(events[2 * timed], st) != hipSuccess) return RFA_ERR_HIP;
    if (launch_plan(g, plan, b, K, st) != hipSuccess) return RFA_ERR_HIP;
    if (close) {
      if (hipEventRecord(events[2 * timed + 1], st) != hipSuccess) return RFA_ERR_HIP;
      ++timed;
    }
    *s.cur = 1 - *s.cur;
    if (partials && ++pending == slots) {
      if (launch_reduce_partials(partials, pending, plan.nwg, dacc, st) != hipSuccess)
        return RFA_ERR_HIP;
      pending = 0;
    }
  }
  if (partials && pending > 0)
    if (launch_reduce_partials(partials, pending, plan.nwg, dacc, st) != hipSuccess)
      return RFA_ERR_HIP;
  if (n_timed) *n_timed = timed;
  return RFA_OK;
}

}  // namespace rfa
