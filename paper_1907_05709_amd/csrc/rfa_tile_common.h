// rfa_tile_common.h -- device helpers shared by the tiled step kernels
// (internal): buffer-descriptor access, XCD-aware work-group order, table
// staging and the work-group partial-sum epilogue.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfa_device.h"

namespace rfa {
namespace tile {

constexpr int kRsrcWord3 = 0x00020000;  // gfx9 buffer descriptor word 3 (32-bit data format)
// A vector offset at or beyond a descriptor's record count makes a buffer
// load return 0 and a buffer store do nothing; descriptors here never span
// 2^31 bytes, so this offset (plus any in-range scalar offset) is always
// out of range.  Used to predicate stores without a branch.
constexpr unsigned kOob = 0x80000000u;
// Cache policies of the kernels' stores (cache-policy bits of gfx950 buffer
// instructions), chosen by measurement per schedule.  kStoreThrough (sc1)
// writes through to the device-coherent level, so little dirty data is left
// in the per-XCD L2s to write back when a short launch ends: best for one
// grid whose working set stays in the last-level cache between launches.
// kStoreStream (nt) marks the data as streaming: best when the working set
// exceeds that cache.  kStoreBack (no bits) is the ordinary write-back
// policy, best for the longer launches of cache-sized batch groups.
constexpr int kStoreThrough = 16;
constexpr int kStoreStream = 2;
constexpr int kStoreBack = 0;

// Hardware places work-group w on XCD w % 8.  Give XCD k the contiguous range
// of logical tiles [base_k, base_k + count_k), so tiles sharing halo rows
// meet in one XCD's L2.
__device__ __forceinline__ int remap_xcd(int wg, int nwg) {
  constexpr int kXcd = 8;
  const int per = nwg / kXcd;
  const int rem = nwg % kXcd;
  const int xcd = wg % kXcd;
  const int slot = wg / kXcd;
  const int base = xcd * per + (xcd < rem ? xcd : rem);
  return base + slot;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, size_t bytes) {
  const int n = bytes > 0x7fffffffu ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, kRsrcWord3);
}

// 32-bit buffer loads/stores move raw bits: reinterpret, never convert.
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
}
template <int AUX = kStoreThrough>
__device__ __forceinline__ void st_f32(float v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                       int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, soff, AUX);
}
__device__ __forceinline__ unsigned ld_u8(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return (unsigned)__builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, soff, 0);
}
template <int AUX = kStoreThrough>
__device__ __forceinline__ void st_u8(unsigned v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                      int soff) {
  __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, (int)voff, soff, AUX);
}

// Stage the coefficient tables of the nc classes in use into LDS.
__device__ __forceinline__ void stage_tables(float2* cf, float4* cls, const Tables* tab, int nc,
                                             int nthreads) {
  const int per_axis = nc * nc;
  const float2* src = &tab->cf[0][0];
  for (int t = threadIdx.x; t < 3 * per_axis; t += nthreads) {
    const int ax = t / per_axis, r = t - ax * per_axis;
    const int a = r / nc, c = r - a * nc;
    const int i = ax * kMaxClasses * kMaxClasses + a * kMaxClasses + c;
    cf[i] = src[i];
  }
  if ((int)threadIdx.x < nc) cls[threadIdx.x] = tab->cls[threadIdx.x];
}

// Work-group sum of the threads' partials in fixed order (waves, then wave
// index) into out[0..2]; red is LDS scratch of 3 x n_waves floats.
__device__ __forceinline__ void write_partials(const Partial& acc, float* red, int n_waves,
                                               float* out) {
  const int lane = threadIdx.x & 63;
  const int wy = threadIdx.x >> 6;
  const float pe = wave_sum(acc.perf);
  const float bn = wave_sum(acc.bnd);
  const unsigned mo = wave_sum_u(acc.mono);
  if (lane == 0) {
    red[wy] = pe;
    red[n_waves + wy] = bn;
    red[2 * n_waves + wy] = (float)mo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int w = 0; w < n_waves; ++w) {
      a0 += red[w];
      a1 += red[n_waves + w];
      a2 += red[2 * n_waves + w];
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
  }
}

}  // namespace tile
}  // namespace rfa
