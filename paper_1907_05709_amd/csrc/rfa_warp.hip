// rfa_warp.hip -- breathing-motion view of the temperature image.
//
// The simulated temperature is shown in the breathing phase given by a
// surrogate signal beta(t) by pulling it back through the inverse motion
// field (Eq. (eq:breathing)): T_view(x) = T(x + beta v(x)).  z is the fastest
// index, so a wave covers 64 consecutive z voxels and, the motion being
// smooth, its corner gathers fall on a few contiguous cache lines of four
// source rows.  Bytes that must move per voxel: the three displacement
// components, one output, and the float-float source state once (24 bytes);
// the 2 x 2 corner re-reads are served by the caches.
//
// Accuracy (the view is within 1e-4 K of the FP64 interpolant of the state):
//  * sample positions are formed in FP64 (the displacement in voxels is up
//    to tens of voxels, where an FP32 product would misplace the sample by
//    ~1e-6 voxel, i.e. ~1e-4 K on the steepest slopes next to the needle);
//    only the fraction within the cell, in [0, 1], is rounded to float;
//  * the eight corners are read as float-float (hi + lo) and interpolated
//    as excess over the hi word of the corner nearest to the sample, so the
//    lerps act on local differences (a few K) instead of the full 900 K;
//  * 37 + that hi word is split exactly (TwoSum) and the output rounded
//    once.  A sample on a voxel centre (fractions 0 or 1: integer shifts,
//    positions clamped to a wall) is that voxel's float-float state rounded
//    once: the lerps return their end values exactly and the nearest corner
//    is the voxel itself.
//
// Launch shape (measured on 256^3 at 0.5 mm with a 12 mm field): each
// thread takes kVx voxels adjacent in x, which share source rows and put
// four independent gather chains in flight (one voxel per thread is ~1.5x
// slower); the two z corners of a row are one 8-byte load (a multi-dword
// load needs only 4-byte alignment); the displacement is read with the
// ordinary cache policy, so the part of it that stays in the last-level
// cache between frames is reused (non-temporal reads cost 25 %), and the
// output is stored non-temporally (write-back stores cost 35 %).
#include "rfa_warp.h"
#include "rfa_tile_common.h"

namespace rfa {
namespace {

constexpr int kWarpThreads = 256;
constexpr int kVx = 4;

// One displacement field: x, y, z component planes (metres) and the factors
// that turn them into voxels (surrogate / spacing per axis, FP64).
struct WarpField {
  const float* x;
  const float* y;
  const float* z;
  double cx, cy, cz;
};

// Two consecutive floats, 4-byte aligned.
typedef float pair_f32 __attribute__((ext_vector_type(2), aligned(4)));

// Split the position i + s (voxels, FP64) into a base index k in [0, n - 2]
// and a fraction f in [0, 1], positions beyond the walls taken at the wall.
// s - floor(s) is exact in FP64; f is its one rounding to float.  A
// non-finite s lands on a wall, so every gather stays inside the grid.
__device__ __forceinline__ void locate(double s, int i, int n, int& k, float& f) {
  const double lim = (double)n;
  if (!(s >= -lim)) s = -lim;  // also NaN
  if (!(s <= lim)) s = lim;
  const double fl = floor(s);
  f = (float)(s - fl);
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

// Excess of the float-float corner (h, l) over the base b, rounded once
// (h - b is exact for neighbouring values within a factor of two; 0 for
// the base corner itself, whose excess is then exactly l).
__device__ __forceinline__ float rel(float h, float l, float b) { return (h - b) + l; }

// Positions s_a = a.c_a * a_a (+ b.c_b * b_a with a second field), in voxels.
template <bool kTwo>
__global__ __launch_bounds__(kWarpThreads) void k_warp(const float* __restrict__ hi,
                                                       const float* __restrict__ lo,
                                                       WarpField a, WarpField b,
                                                       float* __restrict__ out, int nx, int ny,
                                                       int nz, unsigned n_threads) {
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
  double ux[kVx], uy[kVx], uz[kVx];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const unsigned o = (unsigned)min(xg * kVx + j, nx - 1) * sx + yz;
    ux[j] = a.cx * (double)a.x[o];
    uy[j] = a.cy * (double)a.y[o];
    uz[j] = a.cz * (double)a.z[o];
    if constexpr (kTwo) {
      ux[j] = __builtin_fma(b.cx, (double)b.x[o], ux[j]);
      uy[j] = __builtin_fma(b.cy, (double)b.y[o], uy[j]);
      uz[j] = __builtin_fma(b.cz, (double)b.z[o], uz[j]);
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
    const unsigned c = (unsigned)kx * sx + (unsigned)ky * sy + (unsigned)kz;
    const pair_f32 h00 = *(const pair_f32*)(hi + c);
    const pair_f32 h01 = *(const pair_f32*)(hi + c + sy);
    const pair_f32 h10 = *(const pair_f32*)(hi + c + sx);
    const pair_f32 h11 = *(const pair_f32*)(hi + c + sx + sy);
    const pair_f32 l00 = *(const pair_f32*)(lo + c);
    const pair_f32 l01 = *(const pair_f32*)(lo + c + sy);
    const pair_f32 l10 = *(const pair_f32*)(lo + c + sx);
    const pair_f32 l11 = *(const pair_f32*)(lo + c + sx + sy);
    // hi word of the corner nearest to the sample (ties to the lower one)
    const bool cz = fz >= 0.5f, cy = fy >= 0.5f, cx = fx >= 0.5f;
    const float by0 = cy ? (cz ? h01.y : h01.x) : (cz ? h00.y : h00.x);
    const float by1 = cy ? (cz ? h11.y : h11.x) : (cz ? h10.y : h10.x);
    const float b0 = cx ? by1 : by0;
    const float e00 = lerp(rel(h00.x, l00.x, b0), rel(h00.y, l00.y, b0), fz);
    const float e01 = lerp(rel(h01.x, l01.x, b0), rel(h01.y, l01.y, b0), fz);
    const float e10 = lerp(rel(h10.x, l10.x, b0), rel(h10.y, l10.y, b0), fz);
    const float e11 = lerp(rel(h11.x, l11.x, b0), rel(h11.y, l11.y, b0), fz);
    const float d = lerp(lerp(e00, e01, fy), lerp(e10, e11, fy), fx);
    // 37 + b0 split exactly into s + e, then the one rounding s + (e + d)
    const float s = 37.0f + b0;
    const float bv = s - 37.0f;
    const float e = (37.0f - (s - bv)) + (b0 - bv);
    r[j] = s + (e + d);
  }
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const int x = xg * kVx + j;
    if (x < nx) __builtin_nontemporal_store(r[j], out + ((unsigned)x * sx + yz));
  }
}

}  // namespace

hipError_t launch_warp(Grid3 g, const float* hi, const float* lo, const float* v,
                       const double (&scale)[3], const float* v2, const double (&scale2)[3],
                       float* out, hipStream_t st) {
  const size_t n = g.n();
  if (n == 0) return hipSuccess;
  if (n >= (size_t(1) << 31) || g.nx < 2 || g.ny < 2 || g.nz < 2) return hipErrorInvalidValue;
  const size_t threads = (size_t)((g.nx + kVx - 1) / kVx) * g.ny * g.nz;
  const unsigned blocks = (unsigned)((threads + kWarpThreads - 1) / kWarpThreads);
  const WarpField a{v, v + n, v + 2 * n, scale[0], scale[1], scale[2]};
  if (v2) {
    const WarpField b{v2, v2 + n, v2 + 2 * n, scale2[0], scale2[1], scale2[2]};
    hipLaunchKernelGGL(k_warp<true>, dim3(blocks), dim3(kWarpThreads), 0, st, hi, lo, a, b,
                       out, g.nx, g.ny, g.nz, (unsigned)threads);
  } else {
    hipLaunchKernelGGL(k_warp<false>, dim3(blocks), dim3(kWarpThreads), 0, st, hi, lo, a, a,
                       out, g.nx, g.ny, g.nz, (unsigned)threads);
  }
  return hipGetLastError();
}

}  // namespace rfa
