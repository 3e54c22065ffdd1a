// rfa_step.hip -- step scheduling (kernel choice, launch shapes, launch loop).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rfa_step.h"

namespace rfa {

namespace {
constexpr int kTargetWg = 1024;  // ~4 work-groups per CU on 256 CUs

// Stepping working set (two state images, class bytes, source, damage:
// ~29 B per voxel) beyond ~3/4 of the 256 MB last-level cache: stream the
// stores instead of writing them through.
int store_for(Grid3 g) {
  return (double)g.n() * 29.0 > 192.0 * (1 << 20) ? kPolicyStream : kPolicyThrough;
}
}

namespace {
StepPlan with_one(StepPlan p, const StepPlan& one) {
  p.one_kind = one.kind;
  p.one_ty = one.ty;
  p.one_xc = one.xc;
  p.one_nwg = one.nwg;
  p.one_zv = one.zv;
  return p;
}

StepPlan with_store(StepPlan p, Grid3 g) {
  p.store = store_for(g);
  return p;
}

// x chunk giving about `target` work-groups for `tiles` tiles per plane,
// rounded up to the kernels' four-plane unroll
int default_xc(Grid3 g, int tiles, int target = kTargetWg) {
  const int chunks = std::max(1, (target + tiles - 1) / tiles);
  const int xc = (g.nx + chunks - 1) / chunks;
  return std::min(g.nx, std::max(4, (xc + 3) / 4 * 4));
}

// Work-groups that fit the chip at once with the wide kernel (4-wave
// work-groups, 2 resident waves per SIMD with 4 voxels per lane, 4 with 2).
int wide_target_wg(int zv) { return zv == 4 ? 512 : 1024; }
}  // namespace

StepPlan plan_naive(Grid3 g) {
  StepPlan p;
  p.kind = kStepNaive;
  p.depth = 1;
  p.ty = 4;
  p.xc = 1;
  p.nwg = naive_wg_count(g);
  p.zv = 1;
  p.store = kPolicyBack;
  return with_one(p, p);
}

StepPlan plan_tiled(Grid3 g, int ty, int xc) {
  const TiledShape s = tiled_shape(g, ty, xc);
  StepPlan p;
  p.kind = kStepTiled;
  p.depth = 1;
  p.ty = ty;
  p.xc = xc;
  p.nwg = s.nwg;
  p.zv = 1;
  return with_one(with_store(p, g), p);
}

StepPlan plan_wide(Grid3 g, int zv, int ty, int xc) {
  const TiledShape s = wide_shape(g, zv, ty, xc);
  StepPlan p;
  p.kind = kStepTiled;
  p.depth = 1;
  p.ty = ty;
  p.xc = xc;
  p.nwg = s.nwg;
  p.zv = zv;
  return with_one(with_store(p, g), p);
}

StepPlan plan_tiled2(Grid3 g, int ty, int xc) {
  const TiledShape s = tiled2_shape(g, ty, xc);
  StepPlan p;
  p.kind = kStepTiled;
  p.depth = 2;
  p.ty = ty;
  p.xc = xc;
  p.nwg = s.nwg;
  p.zv = 1;
  return with_one(with_store(p, g), plan_default(g, kStepTiled, 1, 0, 0, 0));
}

StepPlan plan_one(const StepPlan& p) {
  StepPlan o = p;
  o.kind = p.one_kind;
  o.depth = 1;
  o.ty = p.one_ty;
  o.xc = p.one_xc;
  o.nwg = p.one_nwg;
  o.zv = p.one_zv;
  return o;
}

namespace {
StepPlan default_shape(Grid3 g, int kernel, int depth, int tile_y, int tile_x, int zv) {
  if (kernel == kStepNaive || !tiled_fits(g, 4)) return plan_naive(g);
  // automatic: four z voxels per lane once a tile row spans 256 voxels, two
  // (with 8-row tiles) from 96
  if (zv == 0 && depth != 2 && g.nz >= 256 && g.nz % 4 == 0) zv = 4;
  if (zv == 0 && depth != 2 && g.nz >= 96 && g.nz % 2 == 0) zv = 2;
  if (depth != 2 && (zv == 2 || zv == 4) && wide_fits(g, zv, 4) && tile_y != 16) {
    const int ty = tile_y ? tile_y : (zv == 2 ? 8 : 4);
    const int tiles = ((g.nz + 64 * zv - 1) / (64 * zv)) * ((g.ny + ty - 1) / ty);
    int xc = tile_x ? std::min(tile_x, g.nx) : default_xc(g, tiles, wide_target_wg(zv));
    while (xc > 4 && !wide_fits(g, zv, xc)) xc /= 2;
    return plan_wide(g, zv, ty, xc);
  }
  if (depth == 2 && tiled2_fits(g, 4)) {
    const int ty = tile_y == 16 ? 16 : 8;
    const int tiles = ((g.nz + 61) / 62) * ((g.ny + ty - 3) / (ty - 2));
    // the x-march runs planes x0 - 1 .. x0 + xc four at a time: xc = 2 mod 4
    // leaves no pass over planes outside the chunk
    int xc = tile_x ? std::min(tile_x, g.nx) : std::min(g.nx, default_xc(g, tiles) + 2);
    while (xc > 4 && !tiled2_fits(g, xc)) xc /= 2;
    return plan_tiled2(g, ty, xc);
  }
  int ty = tile_y;
  if (ty == 0) ty = g.ny >= 192 ? 8 : 4;
  const int tiles = ((g.nz + 63) / 64) * ((g.ny + ty - 1) / ty);
  int xc = tile_x ? std::min(tile_x, g.nx) : default_xc(g, tiles);
  while (xc > 4 && !tiled_fits(g, xc)) xc /= 2;
  return plan_tiled(g, ty, xc);
}
}  // namespace

StepPlan plan_default(Grid3 g, int kernel, int depth, int tile_y, int tile_x, int zv,
                      int store) {
  StepPlan p = default_shape(g, kernel, depth, tile_y, tile_x, zv);
  if (store > 0 && p.kind != kStepNaive) p.store = store - 1;
  return p;
}

int plan_candidates(Grid3 g, int max_depth, StepPlan* out, int max_out) {
  int n = 0;
  const int xcs[] = {4, 8, 16, 32, 64};
  const int tys[] = {4, 8, 16};
  for (int ty : tys)
    for (int xc : xcs) {
      if (n >= max_out) return n;
      if ((xc > g.nx && xc != 4) || !tiled_fits(g, std::min(xc, g.nx))) continue;
      out[n++] = plan_tiled(g, ty, std::min(xc, g.nx));
    }
  const int zvs[] = {2, 4};
  const int tysw[] = {4, 8};
  const int xcsw[] = {4, 8, 16, 32, 64};
  for (int zv : zvs)
    for (int ty : tysw)
      for (int xc : xcsw) {
        if (n >= max_out) return n;
        if ((xc > g.nx && xc != 4) || !wide_fits(g, zv, std::min(xc, g.nx))) continue;
        out[n++] = plan_wide(g, zv, ty, std::min(xc, g.nx));
      }
  if (max_depth < 2) return n;
  const int tys2[] = {8, 16};
  const int xcs2[] = {6, 14, 30, 62};  // 2 mod 4: no pass outside the chunk
  for (int ty : tys2)
    for (int xc : xcs2) {
      if (n >= max_out) return n;
      if ((xc > g.nx && xc != 4) || !tiled2_fits(g, std::min(xc, g.nx))) continue;
      out[n++] = plan_tiled2(g, ty, std::min(xc, g.nx));
    }
  return n;
}

int plan_max_wg(Grid3 g) {
  int m = naive_wg_count(g);
  const int tys[] = {4, 8, 16};
  for (int ty : tys) m = std::max(m, tiled_shape(g, ty, 1).nwg);
  m = std::max(m, tiled2_shape(g, 8, 1).nwg);
  return m;
}

hipError_t launch_plan(Grid3 g, const StepPlan& plan, const StepBuffers& b, const StepConst& K,
                       hipStream_t st) {
  if (plan.kind == kStepNaive) return launch_step_naive(g, b, K, st);
  if (plan.depth == 2)
    return launch_step_tiled2(tiled2_shape(g, plan.ty, plan.xc), g, b, K, plan.store, st);
  if (plan.zv > 1)
    return launch_step_wide(plan.zv, wide_shape(g, plan.zv, plan.ty, plan.xc), g, b, K,
                            plan.store, st);
  return launch_step_tiled(tiled_shape(g, plan.ty, plan.xc), g, b, K, plan.store, st);
}

hipError_t launch_plan_temperature(Grid3 g, const StepPlan& plan, const StepBuffers& b,
                                   const StepConst& K, hipStream_t st) {
  if (plan.kind != kStepNaive && plan.depth == 1 && plan.zv > 1)
    return launch_step_wide_temperature(plan.zv, wide_shape(g, plan.zv, plan.ty, plan.xc), g, b,
                                        K, plan.store, st);
  return launch_plan(g, plan, b, K, st);
}

rfa_status run_steps(Grid3 g, const StepPlan& plan, StepState& s, const StepConst& K,
                     int n_steps, float* partials, int slots, double* dacc, hipEvent_t* events,
                     int period, int* n_timed, int* n_launches, hipStream_t st) {
  if (s.traj && plan.depth != 1) return RFA_ERR_ARG;
  auto buffers = [&]() {
    StepBuffers b;
    b.hi_in = s.hi[*s.cur];
    b.lo_in = s.lo[*s.cur];
    b.hi_out = s.hi[1 - *s.cur];
    b.lo_out = s.lo[1 - *s.cur];
    if (s.traj) {
      float* h = s.traj + (size_t)*s.traj_t * s.traj_n;
      b.hi_in = h;
      b.hi_out = h + s.traj_n;
    }
    b.lab = s.lab;
    b.src = s.src;
    b.omega = s.om;
    b.perf = s.perf;
    b.tab = s.tab;
    b.n_classes = s.n_classes;
    b.partials = nullptr;
    return b;
  };
  const int n_main = n_steps / plan.depth;
  const int n_rest = n_steps - n_main * plan.depth;
  int pending = 0;
  int timed = 0;
  for (int n = 0; n < n_main; ++n) {
    StepBuffers b = buffers();
    b.partials = partials ? partials + (size_t)pending * plan.nwg * 3 : nullptr;
    // Blocks of `period` consecutive launches are bracketed by one event pair
    // (the diagnostic reductions fall between blocks, never inside one).
    const bool open = events && (n % period) == 0;
    const bool close = events && ((n % period) == period - 1 || n == n_main - 1);
    if (open && hipEventRecord(events[2 * timed], st) != hipSuccess) return RFA_ERR_HIP;
    if (launch_plan(g, plan, b, K, st) != hipSuccess) return RFA_ERR_HIP;
    if (s.traj) ++*s.traj_t;
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
  const StepPlan one = plan_one(plan);
  for (int r = 0; r < n_rest; ++r) {
    StepBuffers b = buffers();
    b.partials = partials;
    if (launch_plan(g, one, b, K, st) != hipSuccess) return RFA_ERR_HIP;
    *s.cur = 1 - *s.cur;
    if (partials && launch_reduce_partials(partials, 1, one.nwg, dacc, st) != hipSuccess)
      return RFA_ERR_HIP;
  }
  if (n_timed) *n_timed = timed;
  if (n_launches) *n_launches = events ? n_main : 0;
  return RFA_OK;
}

}  // namespace rfa
