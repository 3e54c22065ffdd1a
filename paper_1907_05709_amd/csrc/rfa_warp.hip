// rfa_warp.hip -- breathing-motion view of the temperature image.
//
// The simulated temperature is shown in the breathing phase given by a
// surrogate signal beta(t) by pulling it back through the inverse motion
// field (Eq. (eq:breathing)): T_view(x) = T(x + beta v(x)).  z is the fastest
// index, so a wave covers 64 consecutive z voxels and, the motion being
// smooth, its corner gathers fall on a few contiguous cache lines of four
// source rows.  Bytes that must move per voxel: the three displacement
// components, one output, and the source image once (20 bytes); the 2 x 2
// corner re-reads are served by the caches.
//
// Launch shape (measured on 256^3 at 0.5 mm with a 12 mm field): each
// thread takes kVx voxels adjacent in x, which share source rows and put
// four independent gather chains in flight (55 us against 83 us for one
// voxel per thread); the two z corners of a row are one 8-byte load (a
// multi-dword load needs only 4-byte alignment); the displacement is read
// with the ordinary cache policy, so the part of it that stays in the
// last-level cache between frames is reused (non-temporal reads cost 25 %),
// and the output is stored non-temporally (write-back stores cost 35 %).
#include "rfa_warp.h"
#include "rfa_tile_common.h"

namespace rfa {
namespace {

constexpr int kWarpThreads = 256;
constexpr int kVx = 4;

// One displacement field: x, y, z component planes (metres) and the factors
// that turn them into voxels (surrogate / spacing per axis).
struct WarpField {
  const float* x;
  const float* y;
  const float* z;
  float cx, cy, cz;
};

// Two consecutive floats, 4-byte aligned.
typedef float pair_f32 __attribute__((ext_vector_type(2), aligned(4)));

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

// (1 - t) a + t b as two FMAs: exactly a at t = 0 and exactly b at t = 1, so
// positions on a voxel centre (integer shifts, positions clamped to a wall)
// return that voxel's value unrounded.
__device__ __forceinline__ float lerp(float a, float b, float t) {
  return __builtin_fmaf(t, b, __builtin_fmaf(-t, a, a));
}

// Positions s_a = a.c_a * a_a (+ b.c_b * b_a with a second field), in voxels.
template <bool kTwo>
__global__ __launch_bounds__(kWarpThreads) void k_warp(const float* __restrict__ hi, WarpField a,
                                                       WarpField b, float* __restrict__ out,
                                                       int nx, int ny, int nz,
                                                       unsigned n_threads) {
  const int wg = tile::remap_xcd(blockIdx.x, gridDim.x);
  const unsigned q = (unsigned)wg * kWarpThreads + threadIdx.x;
  if (q >= n_threads) return;
  const unsigned row = q / (unsigned)nz;
  const int z = (int)(q - row * (unsigned)nz);
  const int xg = (int)(row / (unsigned)ny);  // group of kVx x planes
  const int y = (int)(row - (unsigned)xg * (unsigned)ny);
  const unsigned sy = (unsigned)nz, sx = (unsigned)ny * (unsigned)nz;
  const unsigned yz = (unsigned)y * sy + (unsigned)z;

  // planes past nx (last group) repeat plane nx - 1 and are not stored
  float ux[kVx], uy[kVx], uz[kVx];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const unsigned o = (unsigned)min(xg * kVx + j, nx - 1) * sx + yz;
    ux[j] = a.cx * a.x[o];
    uy[j] = a.cy * a.y[o];
    uz[j] = a.cz * a.z[o];
    if constexpr (kTwo) {
      ux[j] = __builtin_fmaf(b.cx, b.x[o], ux[j]);
      uy[j] = __builtin_fmaf(b.cy, b.y[o], uy[j]);
      uz[j] = __builtin_fmaf(b.cz, b.z[o], uz[j]);
    }
  }
  float r[kVx];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    int kx, ky, kz;
    float fx, fy, fz;
    locate(ux[j], min(xg * kVx + j, nx - 1), nx, kx, fx);
    locate(uy[j], y, ny, ky, fy);
    locate(uz[j], z, nz, kz, fz);
    const float* p = hi + ((unsigned)kx * sx + (unsigned)ky * sy + (unsigned)kz);
    const pair_f32 c00 = *(const pair_f32*)p;
    const pair_f32 c01 = *(const pair_f32*)(p + sy);
    const pair_f32 c10 = *(const pair_f32*)(p + sx);
    const pair_f32 c11 = *(const pair_f32*)(p + sx + sy);
    const float e00 = lerp(c00.x, c00.y, fz), e01 = lerp(c01.x, c01.y, fz);
    const float e10 = lerp(c10.x, c10.y, fz), e11 = lerp(c11.x, c11.y, fz);
    r[j] = lerp(lerp(e00, e01, fy), lerp(e10, e11, fy), fx);
  }
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const int x = xg * kVx + j;
    if (x < nx) __builtin_nontemporal_store(37.0f + r[j], out + ((unsigned)x * sx + yz));
  }
}

}  // namespace

hipError_t launch_warp(Grid3 g, const float* hi, const float* v, const float (&scale)[3],
                       const float* v2, const float (&scale2)[3], float* out, hipStream_t st) {
  const size_t n = g.n();
  if (n == 0) return hipSuccess;
  if (n >= (size_t(1) << 31) || g.nx < 2 || g.ny < 2 || g.nz < 2) return hipErrorInvalidValue;
  const size_t threads = (size_t)((g.nx + kVx - 1) / kVx) * g.ny * g.nz;
  const unsigned blocks = (unsigned)((threads + kWarpThreads - 1) / kWarpThreads);
  const WarpField a{v, v + n, v + 2 * n, scale[0], scale[1], scale[2]};
  if (v2) {
    const WarpField b{v2, v2 + n, v2 + 2 * n, scale2[0], scale2[1], scale2[2]};
    hipLaunchKernelGGL(k_warp<true>, dim3(blocks), dim3(kWarpThreads), 0, st, hi, a, b, out,
                       g.nx, g.ny, g.nz, (unsigned)threads);
  } else {
    hipLaunchKernelGGL(k_warp<false>, dim3(blocks), dim3(kWarpThreads), 0, st, hi, a, a, out,
                       g.nx, g.ny, g.nz, (unsigned)threads);
  }
  return hipGetLastError();
}

}  // namespace rfa
