// rfa_warp.hip -- breathing-motion view of the temperature image.
//
// The simulated temperature is shown in the breathing phase given by a
// surrogate signal beta(t) by pulling it back through the inverse motion
// field (Eq. (eq:breathing)): T_view(x) = T(x + beta v(x)).  z is the fastest
// index, so a wave covers 64 consecutive z voxels and, the motion being
// smooth, its corner gathers fall on a few contiguous cache lines of four
// source rows.  Bytes that must move per voxel: the three displacement
// components, one output and the state's hi word once (20 bytes; lo words
// only where they matter, see kLoAll); the 2 x 2 corner re-reads are served
// by the caches.  What bounds the kernel is the gathers themselves: each
// corner gather instruction costs about the same whatever its width or
// whether its lanes are masked out by offset, so the kernel issues as few
// as the accuracy allows.
//
// Accuracy (the view is within 1e-4 K of the FP64 interpolant of the state):
//  * sample positions are float-float: the displacement in voxels is up to
//    tens of voxels, where one FP32 product would misplace the sample by
//    ~1e-6 voxel, i.e. ~1e-4 K on the steepest slopes next to the needle.
//    The FP64 factor c = surrogate / spacing is split into c_hi + c_lo
//    (floats); c_hi v is formed exactly as p + fma(c_hi, v, -p) and c_lo v
//    added to the error word, which leaves the position within ~2^-47 of
//    c v.  The cell index is the floor of that pair and only the fraction
//    within the cell, in [0, 1], is rounded to float (at most twice where
//    the error word carries the sum across a cell boundary);
//  * the eight corners are interpolated as excess over the hi word of the
//    corner nearest to the sample, so the lerps act on local differences (a
//    few K) instead of the full 900 K.  Their lo words are read where they
//    matter at this tolerance: in cells with a corner at or above 1024 degC
//    and for samples on a voxel centre (see kLoAll); elsewhere they move the
//    view by less than half an ulp of the hi word;
//  * 37 + that hi word is split exactly (TwoSum) and the output rounded
//    once.  A sample on a voxel centre (fractions 0 or 1: integer shifts,
//    positions clamped to a wall) is that voxel's float-float state rounded
//    once: the lerps return their end values exactly and the nearest corner
//    is the voxel itself.
//
// Launch shape (measured on 256^3 at 0.5 mm with a 12 mm field): a
// work-group takes a tile of 64 z by 4 y rows and each thread kVx voxels
// adjacent in x, which share source rows and put four independent gather
// chains in flight (one voxel per thread is ~1.5x slower); the two z
// corners of a row are one 8-byte load (a multi-dword load needs only
// 4-byte alignment); the displacement is read with the
// ordinary cache policy, so the part of it that stays in the last-level
// cache between frames is reused (non-temporal reads cost 25 %), and the
// output is stored non-temporally (write-back stores cost 35 %).
#include "rfa_warp.h"
#include "rfa_tile_common.h"

namespace rfa {
namespace {

constexpr int kWarpThreads = 256;
constexpr int kVx = 4;
// Excess temperature (K) from which a cell reads its corners' lo words.
// Below it (T < 1024 degC) the lo words, each at most ulp(hi) / 2 <= 3.1e-5
// K, move the interpolant by at most that much, and the output's rounding
// adds at most as much again: 6.1e-5 K together.  Above it the output's
// rounding alone reaches 6.1e-5 K, so hotter cells keep every lo word.
constexpr float kLoAll = 987.0f;

// One displacement field: x, y, z component planes (metres) and the factors
// that turn them into voxels (surrogate / spacing per axis) as float-float
// pairs.
struct WarpField {
  const float* x;
  const float* y;
  const float* z;
  float ch[3], cl[3];
};

// Two consecutive floats, 4-byte aligned.
typedef float pair_f32 __attribute__((ext_vector_type(2), aligned(4)));

// c v as p + e: p = c_hi v rounded, e = its exact error plus c_lo v.
__device__ __forceinline__ void scaled(float v, float ch, float cl, float& p, float& e) {
  p = ch * v;
  e = __builtin_fmaf(ch, v, -p) + cl * v;
}

// (pa + ea) + (pb + eb) as p + e: pa + pb split exactly (TwoSum), the error
// words added to the remainder.  With pb = +-0 and eb = 0 it returns
// (pa, ea) bit for bit.
__device__ __forceinline__ void add_ff(float pa, float ea, float pb, float eb, float& p,
                                       float& e) {
  p = pa + pb;
  const float bb = p - pa;
  const float r = (pa - (p - bb)) + (pb - bb);
  e = (r + ea) + eb;
}

// Split the position i + (p + e) (voxels) into a base index k in [0, n - 2]
// and a fraction f in [0, 1], positions beyond the walls taken at the wall.
// p is clamped to [-n, n] (a NaN to -n; the error word is dropped there),
// fl = floor(p) and t = p - fl are exact, and t + e lies in [-1, 2), so its
// floor g moves the cell by at most one and f = (t + e) - g.  Where t + e
// rounds to 1, the sample is the next cell's corner with weight 0, the same
// value as weight 1 on this cell's far corner.  Branch-free.
__device__ __forceinline__ void locate(float p, float e, int i, int n, int& k, float& f) {
  const float lim = (float)n;
  e = fabsf(p) < lim ? e : 0.0f;
  p = fminf(fmaxf(p, -lim), lim);
  const float fl = floorf(p);
  const float in = (p - fl) + e;
  const float g = floorf(in);
  const int kk = i + (int)(fl + g);
  k = min(max(kk, 0), n - 2);
  f = kk < 0 ? 0.0f : (kk > n - 2 ? 1.0f : in - g);
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

// Positions s_a = c_a v_a (+ c2_a v2_a with a second field), in voxels.
// A work-group covers 64 z (one wave row, lane = z) by 4 y rows by kVx x
// planes; the tile index is uniform, so no per-lane division is needed.
// kBuf: every offset fits a 32-bit buffer descriptor (n < 2^29), so the
// eight corner gathers share one vector offset and take the row and plane
// strides as scalar offsets; y and z indices are below 2^24 (24-bit
// multiplies).
template <bool kTwo, bool kBuf>
__global__ __launch_bounds__(kWarpThreads) void k_warp(const float* __restrict__ hi,
                                                       const float* __restrict__ lo,
                                                       WarpField a, WarpField b,
                                                       float* __restrict__ out, int nx, int ny,
                                                       int nz, int tiles_z, int tiles_y,
                                                       int nwg) {
  const int wg = tile::remap_xcd(blockIdx.x, nwg);
  const int tz = wg % tiles_z;
  const int rest = wg / tiles_z;
  const int ty = rest % tiles_y;
  const int xg = rest / tiles_y;  // group of kVx x planes
  const int z = tz * 64 + (int)(threadIdx.x & 63);
  const int y = ty * 4 + (int)(threadIdx.x >> 6);
  if (z >= nz || y >= ny) return;  // no barrier follows
  const unsigned sy = (unsigned)nz, sx = (unsigned)ny * (unsigned)nz;
  auto mul = [](unsigned u, unsigned w) { return kBuf ? __umul24(u, w) : u * w; };
  const unsigned yz = mul((unsigned)y, sy) + (unsigned)z;
  const unsigned n = sx * (unsigned)nx;
  __amdgpu_buffer_rsrc_t rh, rl, rax, ray, raz, rbx, rby, rbz, ro;
  if constexpr (kBuf) {
    const size_t bytes = (size_t)n * 4;
    rh = tile::make_rsrc(hi, bytes);
    rl = tile::make_rsrc(lo, bytes);
    rax = tile::make_rsrc(a.x, bytes);
    ray = tile::make_rsrc(a.y, bytes);
    raz = tile::make_rsrc(a.z, bytes);
    rbx = tile::make_rsrc(b.x, bytes);
    rby = tile::make_rsrc(b.y, bytes);
    rbz = tile::make_rsrc(b.z, bytes);
    ro = tile::make_rsrc(out, bytes);
  }
  // component w of a displacement at voxel o
  auto disp = [&](const float* w, __amdgpu_buffer_rsrc_t r, unsigned o) {
    if constexpr (kBuf)
      return tile::ld_f32(r, o * 4u, 0);
    else
      return w[o];
  };
  const int so1 = (int)(sy * 4u), so2 = (int)(sx * 4u), so3 = (int)((sx + sy) * 4u);
  auto corners = [&](const float* base, __amdgpu_buffer_rsrc_t r, unsigned c, pair_f32& c00,
                     pair_f32& c01, pair_f32& c10, pair_f32& c11) {
    if constexpr (kBuf) {
      const int vo = (int)(c * 4u);
      c00 = __builtin_bit_cast(pair_f32, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0));
      c01 = __builtin_bit_cast(pair_f32, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so1, 0));
      c10 = __builtin_bit_cast(pair_f32, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so2, 0));
      c11 = __builtin_bit_cast(pair_f32, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so3, 0));
    } else {
      const float* q = base + c;
      c00 = *(const pair_f32*)q;
      c01 = *(const pair_f32*)(q + sy);
      c10 = *(const pair_f32*)(q + sx);
      c11 = *(const pair_f32*)(q + sx + sy);
    }
  };

  // planes past nx (last group) repeat plane nx - 1 and are not stored
  float px[kVx], py[kVx], pz[kVx], ex[kVx], ey[kVx], ez[kVx];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const unsigned o = (unsigned)min(xg * kVx + j, nx - 1) * sx + yz;
    scaled(disp(a.x, rax, o), a.ch[0], a.cl[0], px[j], ex[j]);
    scaled(disp(a.y, ray, o), a.ch[1], a.cl[1], py[j], ey[j]);
    scaled(disp(a.z, raz, o), a.ch[2], a.cl[2], pz[j], ez[j]);
    if constexpr (kTwo) {
      float pb, eb;
      scaled(disp(b.x, rbx, o), b.ch[0], b.cl[0], pb, eb);
      add_ff(px[j], ex[j], pb, eb, px[j], ex[j]);
      scaled(disp(b.y, rby, o), b.ch[1], b.cl[1], pb, eb);
      add_ff(py[j], ey[j], pb, eb, py[j], ey[j]);
      scaled(disp(b.z, rbz, o), b.ch[2], b.cl[2], pb, eb);
      add_ff(pz[j], ez[j], pb, eb, pz[j], ez[j]);
    }
  }
  // Phase 1: cell, fractions and the four hi pairs of every voxel, all
  // gathers issued before any use.
  unsigned cc[kVx];
  float fx[kVx], fy[kVx], fz[kVx];
  pair_f32 h[kVx][4];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    int kx, ky, kz;
    locate(px[j], ex[j], min(xg * kVx + j, nx - 1), nx, kx, fx[j]);
    locate(py[j], ey[j], y, ny, ky, fy[j]);
    locate(pz[j], ez[j], z, nz, kz, fz[j]);
    cc[j] = (unsigned)kx * sx + mul((unsigned)ky, sy) + (unsigned)kz;
    corners(hi, rh, cc[j], h[j][0], h[j][1], h[j][2], h[j][3]);
  }
  // A sample on a voxel centre (every fraction 0 or 1) also reads that
  // voxel's lo word (the nearest corner's): the interpolant there is
  // exactly its excess, so the view is the state rounded once.  Known from
  // the fractions alone, so these loads fly with the hi gathers; a branch,
  // taken only by waves that hold such a sample.
  bool ctr[kVx];
  bool any_ctr = false;
  float lb[kVx];
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    auto edge = [](float f) { return f == 0.0f || f == 1.0f; };
    ctr[j] = edge(fx[j]) && edge(fy[j]) && edge(fz[j]);
    any_ctr = any_ctr || ctr[j];
    lb[j] = 0.0f;
  }
  if (any_ctr) {
#pragma unroll
    for (int j = 0; j < kVx; ++j) {
      const unsigned cb = cc[j] + (fz[j] >= 0.5f ? 1u : 0u) + (fy[j] >= 0.5f ? sy : 0u) +
                          (fx[j] >= 0.5f ? sx : 0u);
      if constexpr (kBuf)
        lb[j] = tile::ld_f32(rl, ctr[j] ? cb * 4u : tile::kOob, 0);
      else
        lb[j] = ctr[j] ? lo[cb] : 0.0f;
    }
  }
  // Trilinear interpolation of the corner excesses (h - b0) + l over the hi
  // word b0 of the corner nearest to the sample (ties to the lower one),
  // then 37 + b0 split exactly into s + e and the one rounding s + (e + d).
  auto base = [&](int j) {
    const bool cz = fz[j] >= 0.5f, cy = fy[j] >= 0.5f, cx = fx[j] >= 0.5f;
    const float by0 = cy ? (cz ? h[j][1].y : h[j][1].x) : (cz ? h[j][0].y : h[j][0].x);
    const float by1 = cy ? (cz ? h[j][3].y : h[j][3].x) : (cz ? h[j][2].y : h[j][2].x);
    return cx ? by1 : by0;
  };
  auto finish = [](float b0, float d) {
    const float s = 37.0f + b0;
    const float bv = s - 37.0f;
    const float e = (37.0f - (s - bv)) + (b0 - bv);
    return s + (e + d);
  };
  auto view = [&](int j, const pair_f32 (&l)[4]) {
    const pair_f32 h00 = h[j][0], h01 = h[j][1], h10 = h[j][2], h11 = h[j][3];
    const float gz = fz[j], gy = fy[j], gx = fx[j];
    const float b0 = base(j);
    const float e00 = lerp(rel(h00.x, l[0].x, b0), rel(h00.y, l[0].y, b0), gz);
    const float e01 = lerp(rel(h01.x, l[1].x, b0), rel(h01.y, l[1].y, b0), gz);
    const float e10 = lerp(rel(h10.x, l[2].x, b0), rel(h10.y, l[2].y, b0), gz);
    const float e11 = lerp(rel(h11.x, l[3].x, b0), rel(h11.y, l[3].y, b0), gz);
    return finish(b0, lerp(lerp(e00, e01, gy), lerp(e10, e11, gy), gx));
  };
  // Phase 2: every voxel from the hi words (and a centre's own lo word).
  float r[kVx];
  bool hot[kVx];
  bool any_hot = false;
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const pair_f32 zero[4] = {};
    r[j] = ctr[j] ? finish(base(j), lb[j]) : view(j, zero);
    float m = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) m = fmaxf(m, fmaxf(fabsf(h[j][q].x), fabsf(h[j][q].y)));
    hot[j] = m >= kLoAll;
    any_hot = any_hot || hot[j];
  }
  // Phase 3: cells with a corner at or above kLoAll read their eight lo
  // words and are redone (a branch, taken only by waves that hold such a
  // cell: gathers masked out by offset cost as much as real ones).
  if (any_hot) {
#pragma unroll
    for (int j = 0; j < kVx; ++j) {
      pair_f32 l[4];
      if constexpr (kBuf) {
        corners(lo, rl, hot[j] ? cc[j] : tile::kOob / 4u, l[0], l[1], l[2], l[3]);
      } else {
        l[0] = l[1] = l[2] = l[3] = pair_f32{0.0f, 0.0f};
        if (hot[j]) corners(lo, rl, cc[j], l[0], l[1], l[2], l[3]);
      }
      r[j] = hot[j] ? view(j, l) : r[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kVx; ++j) {
    const int x = xg * kVx + j;
    if constexpr (kBuf) {
      tile::st_f32<tile::kStoreStream>(r[j], ro, x < nx ? ((unsigned)x * sx + yz) * 4u : tile::kOob,
                                       0);
    } else {
      if (x < nx) __builtin_nontemporal_store(r[j], out + ((unsigned)x * sx + yz));
    }
  }
}

}  // namespace

hipError_t launch_warp(Grid3 g, const float* hi, const float* lo, const float* v,
                       const double (&scale)[3], const float* v2, const double (&scale2)[3],
                       float* out, hipStream_t st) {
  const size_t n = g.n();
  if (n == 0) return hipSuccess;
  if (n >= (size_t(1) << 31) || g.nx < 2 || g.ny < 2 || g.nz < 2) return hipErrorInvalidValue;
  auto field = [&](const float* w, const double(&c)[3]) {
    WarpField f{w, w + n, w + 2 * n, {}, {}};
    for (int a = 0; a < 3; ++a) {
      f.ch[a] = (float)c[a];
      f.cl[a] = (float)(c[a] - (double)f.ch[a]);
    }
    return f;
  };
  const int tiles_z = (g.nz + 63) / 64, tiles_y = (g.ny + 3) / 4;
  const size_t nwg = (size_t)tiles_z * tiles_y * ((g.nx + kVx - 1) / kVx);
  if (nwg > 0x7fffffffu) return hipErrorInvalidValue;
  const bool buf = n * 4 <= 0x7fffffffu && g.ny < (1 << 24) && g.nz < (1 << 24);
  const WarpField a = field(v, scale);
  const WarpField b = v2 ? field(v2, scale2) : a;
  const dim3 grid((unsigned)nwg), block(kWarpThreads);
  const int nw = (int)nwg;
  if (v2 && buf)
    hipLaunchKernelGGL((k_warp<true, true>), grid, block, 0, st, hi, lo, a, b, out, g.nx, g.ny,
                       g.nz, tiles_z, tiles_y, nw);
  else if (v2)
    hipLaunchKernelGGL((k_warp<true, false>), grid, block, 0, st, hi, lo, a, b, out, g.nx,
                       g.ny, g.nz, tiles_z, tiles_y, nw);
  else if (buf)
    hipLaunchKernelGGL((k_warp<false, true>), grid, block, 0, st, hi, lo, a, b, out, g.nx,
                       g.ny, g.nz, tiles_z, tiles_y, nw);
  else
    hipLaunchKernelGGL((k_warp<false, false>), grid, block, 0, st, hi, lo, a, b, out, g.nx,
                       g.ny, g.nz, tiles_z, tiles_y, nw);
  return hipGetLastError();
}

}  // namespace rfa
