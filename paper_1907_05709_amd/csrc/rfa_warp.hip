// rfa_warp.hip -- breathing-motion view of the temperature image.
//
// The simulated temperature is shown in the breathing phase given by a
// surrogate signal beta(t) by pulling it back through the inverse motion
// field (Eq. (eq:breathing)): T_view(x) = T(x + beta v(x)).  One thread per
// output voxel; z is the fastest index, so a wave covers 64 consecutive z
// voxels and, the motion being smooth, its eight corner gathers fall on a few
// contiguous cache lines of four source rows.  Bytes that must move per
// voxel: the three displacement components, one output, and the source image
// once (20 bytes); the 2 x 2 corner re-reads are served by the caches.
#include "rfa_warp.h"
#include "rfa_tile_common.h"

namespace rfa {
namespace {

constexpr int kWarpThreads = 256;

// Split the position i + s (voxels) into a base index k in [0, n - 2] and a
// fraction f in [0, 1], positions beyond the walls taken at the wall.  f is
// exact: s - floor(s) has no rounding for |s| < 2^23.  A non-finite s lands
// on a wall, so every gather stays inside the grid.
__device__ __forceinline__ void locate(float s, int i, int n, int& k, float& f) {
  const float lim = (float)n;
  if (!(s >= -lim)) s = -lim;  // also NaN
  if (!(s <= lim)) s = lim;
  const float fl = floorf(s);
  f = s - fl;
  k = i + (int)fl;
  if (k < 0) {
    k = 0;
    f = 0.0f;
  } else if (k >= n - 1) {
    k = n - 2;
    f = 1.0f;
  }
}

__device__ __forceinline__ float lerp(float a, float b, float t) {
  return __builtin_fmaf(t, b - a, a);
}

__global__ __launch_bounds__(kWarpThreads) void k_warp(
    const float* __restrict__ hi, const float* __restrict__ vx, const float* __restrict__ vy,
    const float* __restrict__ vz, float* __restrict__ out, int nx, int ny, int nz,
    unsigned n, float cx, float cy, float cz) {
  const int wg = tile::remap_xcd(blockIdx.x, gridDim.x);
  const unsigned q = (unsigned)wg * kWarpThreads + threadIdx.x;
  if (q >= n) return;
  const unsigned row = q / (unsigned)nz;
  const int z = (int)(q - row * (unsigned)nz);
  const int x = (int)(row / (unsigned)ny);
  const int y = (int)(row - (unsigned)x * (unsigned)ny);

  int kx, ky, kz;
  float fx, fy, fz;
  locate(cx * __builtin_nontemporal_load(vx + q), x, nx, kx, fx);
  locate(cy * __builtin_nontemporal_load(vy + q), y, ny, ky, fy);
  locate(cz * __builtin_nontemporal_load(vz + q), z, nz, kz, fz);

  const unsigned sy = (unsigned)nz, sx = (unsigned)ny * (unsigned)nz;
  const float* p = hi + ((unsigned)kx * sx + (unsigned)ky * sy + (unsigned)kz);
  const float c000 = p[0], c001 = p[1];
  const float c010 = p[sy], c011 = p[sy + 1];
  const float c100 = p[sx], c101 = p[sx + 1];
  const float c110 = p[sx + sy], c111 = p[sx + sy + 1];
  const float e00 = lerp(c000, c001, fz), e01 = lerp(c010, c011, fz);
  const float e10 = lerp(c100, c101, fz), e11 = lerp(c110, c111, fz);
  const float d0 = lerp(e00, e01, fy), d1 = lerp(e10, e11, fy);
  __builtin_nontemporal_store(37.0f + lerp(d0, d1, fx), out + q);
}

}  // namespace

hipError_t launch_warp(Grid3 g, const float* hi, const float* v, float scale_x, float scale_y,
                       float scale_z, float* out, hipStream_t st) {
  const size_t n = g.n();
  if (n == 0) return hipSuccess;
  if (n >= (size_t(1) << 31) || g.nx < 2 || g.ny < 2 || g.nz < 2) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n + kWarpThreads - 1) / kWarpThreads);
  hipLaunchKernelGGL(k_warp, dim3(blocks), dim3(kWarpThreads), 0, st, hi, v, v + n, v + 2 * n,
                     out, g.nx, g.ny, g.nz, (unsigned)n, scale_x, scale_y, scale_z);
  return hipGetLastError();
}

}  // namespace rfa
