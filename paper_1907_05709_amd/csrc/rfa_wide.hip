// rfa_wide.hip -- one-step kernel with ZV consecutive z voxels per lane.
//
// Same schedule as the 2.5-D tiled kernel (a work-group of TY wavefronts
// marches a tile along x, y and z neighbours from a double-buffered LDS
// plane, x neighbours from registers, loads issued two planes ahead into a
// ring of four register sets), but each
// lane owns ZV (2 or 4) consecutive voxels along z, so a wave row spans
// 64 * ZV voxels: every global access is a ZV-wide vector (dwordx2/x4, the
// class bytes as one 16/32-bit word), a tile row of 256 voxels needs no z
// halo inside grids up to 256 wide, and per voxel the kernel issues ZV times
// fewer memory instructions.  Requires nz % ZV == 0 (rows stay aligned).
//
// Halo of the LDS plane: wave 0 loads the row below the tile, wave 1 the
// row above (one vector per lane), wave 2 the aligned vectors that hold the
// z neighbours left and right of each tile row (lanes 0 .. 2 TY - 1).  All
// other lanes issue the same loads with an out-of-range buffer offset
// (returns zero, no memory traffic) and store into a scratch vector, so all
// waves run one instruction stream.  As in the tiled kernel, planes past
// the chunk's end are computed as held voxels and every store that must not
// happen gets an out-of-range offset: no branch surrounds a memory
// instruction.
//
// The source increment is read only where a lane's voxels carry the source
// flag (kSource: s != 0, set with s; elsewhere s is exactly 0): its load is
// issued one plane after the plane's other loads, predicated on the class
// bytes they brought, still a plane before its use.
//
// The per-voxel arithmetic is voxel_step() of rfa_device.h, so results are
// bitwise those of the other step kernels.
//
// TONLY (temperature only): without damage-coupled perfusion the new
// temperature depends on neither the damage integral nor the latch bit, so
// a launch that must reproduce only the temperature (the adjoint's segment
// recompute) skips the damage integral's load and store and the class-byte
// store: 21 instead of 29 bytes per voxel-step with a perfusion field, the
// temperature bitwise that of a full step.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rfa_tile_common.h"
#include "rfa_tiled.h"

namespace rfa {

namespace {

using namespace tile;

template <int ZV>
struct Vec;
template <>
struct Vec<2> {
  typedef float f __attribute__((ext_vector_type(2)));
  typedef unsigned u __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<4> {
  typedef float f __attribute__((ext_vector_type(4)));
  typedef unsigned u __attribute__((ext_vector_type(4)));
};

template <int ZV>
__device__ __forceinline__ typename Vec<ZV>::f ldv(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                   int soff) {
  if constexpr (ZV == 4)
    return __builtin_bit_cast(typename Vec<4>::f,
                              __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, soff, 0));
  else
    return __builtin_bit_cast(typename Vec<2>::f,
                              __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
}
// A buffer store of more than 64 bits reads its data registers some cycles
// after issue, and a VALU write to them in that window corrupts the stored
// value.  The compiler pads that window with wait states only when the
// store's scalar offset is an immediate (it assumes a register scalar offset
// covers it, which does not hold under load on gfx950), so the 128-bit
// store takes its whole offset in the vector register and a zero immediate.
template <int ZV, int AUX>
__device__ __forceinline__ void stv(typename Vec<ZV>::f v, __amdgpu_buffer_rsrc_t r,
                                   unsigned voff) {
  if constexpr (ZV == 4)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(typename Vec<4>::u, v), r,
                                           (int)voff, 0, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(typename Vec<2>::u, v), r,
                                          (int)voff, 0, AUX);
}
// ZV class bytes as one word
template <int ZV>
__device__ __forceinline__ unsigned ldb(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (ZV == 4)
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0);
  else
    return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, soff, 0);
}
template <int ZV, int AUX>
__device__ __forceinline__ void stb(unsigned v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                   int soff) {
  if constexpr (ZV == 4)
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, soff, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)voff, soff, AUX);
}
__device__ __forceinline__ unsigned byte_of(unsigned w, int k) { return (w >> (8 * k)) & 0xFFu; }

template <int ZV>
using LabWord = typename std::conditional<ZV == 4, unsigned, unsigned short>::type;

constexpr int kAheadW = 2;  // planes loaded ahead of the computed one
constexpr int kRingW = 4;   // register ring (unroll factor; even, so slot & 1 = LDS buffer)

template <int ZV>
struct PlaneW {
  typename Vec<ZV>::f h, l, s, om, pf;  // own voxels: state, source, damage, perfusion
  typename Vec<ZV>::f hh, hl;           // halo vector (rows or z neighbours)
  unsigned b, hb;                       // class bytes of own / halo vector
};

template <int ZV, int TY>
struct WideSmem {
  static constexpr int ZW = 64 * ZV;        // voxels along z per tile row
  static constexpr int RW = ZW + 2 * ZV;    // LDS row: left halo vector, ZW voxels, right one
  static constexpr int ROWS = TY + 2;
  static constexpr int CELLS = ROWS * RW;   // plus one scratch vector
  float2 cf[3 * kMaxClasses * kMaxClasses];
  float4 cls[kMaxClasses];
  float th[2][CELLS + ZV];
  float tl[2][CELLS + ZV];
  uint8_t tb[2][CELLS + ZV];
  float red[3 * TY];
};

}  // namespace

// Two voxels per lane fit 128 VGPRs (four waves per SIMD); with a perfusion
// field (and its damage coupling) they would spill there and run three
// waves per SIMD instead; four voxels per lane keep the compiler's choice
// (two waves per SIMD).
template <int ZV, int TY, bool PERF, int AUX, bool TONLY>
__global__ __launch_bounds__(64 * TY, ZV == 2 ? (PERF ? 3 : 4) : 1) void k_step_wide(StepBuffers b, StepConst K, int nx,
                                                       int ny, int nz, int xc, int tiles_z,
                                                       int tiles_y, int nwg) {
  static_assert(TY >= 3, "waves 0-2 load the halo");
  using VF = typename Vec<ZV>::f;
  using S = WideSmem<ZV, TY>;
  constexpr int ZW = S::ZW, RW = S::RW, CELLS = S::CELLS;
  __shared__ S sm;
  stage_tables(sm.cf, sm.cls, b.tab, b.n_classes, 64 * TY);

  const int wg = remap_xcd(blockIdx.x, nwg);
  const int tz = wg % tiles_z;
  const int ty = (wg / tiles_z) % tiles_y;
  const int tx = wg / (tiles_z * tiles_y);
  const int lane = threadIdx.x & 63;
  const int wy = threadIdx.x >> 6;
  const int z0 = tz * ZW, y0 = ty * TY;
  const int zq = z0 + ZV * lane;  // first voxel of this lane
  const int y = y0 + wy;
  const bool inside = zq < nz && y < ny;
  const int x0 = tx * xc;
  const int x1 = min(x0 + xc, nx);
  const int xb = max(x0 - 1, 0);
  const unsigned psz = (unsigned)(ny * nz);
  const unsigned col = inside ? (unsigned)(y * nz + zq) : 0u;

  __amdgpu_buffer_rsrc_t r_hi, r_lo, r_lab, r_src, r_om, r_pf, r_hio, r_loo;
  {
    const size_t off = (size_t)xb * psz;
    const size_t rest = (size_t)(nx - xb) * psz;
    r_hi = make_rsrc(b.hi_in + off, rest * 4);
    r_lo = make_rsrc(b.lo_in + off, rest * 4);
    r_lab = make_rsrc(b.lab + off, rest);
    r_src = make_rsrc(b.src + off, rest * 4);
    r_om = make_rsrc(b.omega + off, rest * 4);
    r_pf = make_rsrc(PERF ? b.perf + off : b.src + off, rest * 4);
    r_hio = make_rsrc(b.hi_out + off, rest * 4);
    r_loo = make_rsrc(b.lo_out + off, rest * 4);
  }

  // Halo vector of this lane: LDS cell and grid offset (kOob: none).
  int hcell = CELLS;
  unsigned hoff = kOob;
  {
    int hy = -1, hz = -1;
    if (wy == 0) {
      hy = y0 - 1; hz = zq; hcell = ZV + ZV * lane;
    } else if (wy == 1) {
      hy = y0 + TY; hz = zq; hcell = (TY + 1) * RW + ZV + ZV * lane;
    } else if (wy == 2 && lane < TY) {
      hy = y0 + lane; hz = z0 - ZV; hcell = (lane + 1) * RW;
    } else if (wy == 2 && lane < 2 * TY) {
      hy = y0 + lane - TY; hz = z0 + ZW; hcell = (lane - TY + 1) * RW + ZV + ZW;
    }
    if (hy >= 0 && hy < ny && hz >= 0 && hz < nz)
      hoff = (unsigned)(hy * nz + hz);
    else
      hcell = CELLS;  // scratch vector; the cell it stands for feeds held voxels only
  }
  const unsigned hoff4 = hoff == kOob ? kOob : hoff * 4;

  auto load = [&](int x, PlaneW<ZV>& q) {
    const int xo = min(x, nx - 1) - xb;  // uniform
    const int xf = min(x, x1 - 1) - xb;  // uniform
    const int so4 = xo * (int)psz * 4, so1 = xo * (int)psz;
    const int sf4 = xf * (int)psz * 4, sf1 = xf * (int)psz;
    q.h = ldv<ZV>(r_hi, col * 4, so4);
    q.l = ldv<ZV>(r_lo, col * 4, so4);
    q.b = ldb<ZV>(r_lab, col, so1);
    if constexpr (TONLY)
      q.om = VF{};
    else
      q.om = ldv<ZV>(r_om, col * 4, sf4);
    if constexpr (PERF) q.pf = ldv<ZV>(r_pf, col * 4, sf4);
    q.hh = ldv<ZV>(r_hi, hoff4, sf4);
    q.hl = ldv<ZV>(r_lo, hoff4, sf4);
    q.hb = ldb<ZV>(r_lab, hoff == kOob ? kOob : hoff, sf1);
  };
  // source increments of plane x, on lanes whose voxels are flagged (the
  // class bytes of plane x are in q.b; below x1 they are plane x's own)
  constexpr unsigned kSrcWord = ZV == 4 ? kSource * 0x01010101u : kSource * 0x0101u;
  auto load_s = [&](int x, PlaneW<ZV>& q) {
    const int xf = min(x, x1 - 1) - xb;  // uniform
    q.s = ldv<ZV>(r_src, (q.b & kSrcWord) ? col * 4 : kOob, xf * (int)psz * 4);
  };

  // x-1 neighbours (own voxels) of the plane being computed
  VF hm, lm;
  unsigned bm;
  {
    const int so = (max(x0 - 1, 0) - xb) * (int)psz;
    hm = ldv<ZV>(r_hi, col * 4, so * 4);
    lm = ldv<ZV>(r_lo, col * 4, so * 4);
    bm = ldb<ZV>(r_lab, col, so);
  }
  PlaneW<ZV> q[kRingW];
#pragma unroll
  for (int k = 0; k < kAheadW; ++k) load(x0 + k, q[k]);
#pragma unroll
  for (int k = 0; k < kAheadW - 1; ++k) load_s(x0 + k, q[k]);

  Partial acc{0.0f, 0.0f, 0u};
  const int me = (wy + 1) * RW + ZV + ZV * lane;  // first own LDS cell
  const unsigned st4 = inside ? col * 4 : kOob;
  const unsigned st1 = inside ? col : kOob;

  // One plane; SL = ring slot of plane x, BUF = its LDS buffer (compile time).
  auto plane_step = [&](auto SL_, int x) {
    constexpr int SL = decltype(SL_)::value;
    constexpr int BUF = SL & 1;
    constexpr int SN = (SL + 1) % kRingW;        // plane x + 1
    constexpr int SA = (SL + kAheadW) % kRingW;  // receives plane x + kAheadW
    constexpr int SS = (SL + kAheadW - 1) % kRingW;  // plane x + kAheadW - 1
    using LW = LabWord<ZV>;
    load(x + kAheadW, q[SA]);
    load_s(x + kAheadW - 1, q[SS]);
    const PlaneW<ZV>& P = q[SL];
    *reinterpret_cast<VF*>(&sm.th[BUF][me]) = P.h;
    *reinterpret_cast<VF*>(&sm.tl[BUF][me]) = P.l;
    *reinterpret_cast<LW*>(&sm.tb[BUF][me]) = (LW)P.b;
    *reinterpret_cast<VF*>(&sm.th[BUF][hcell]) = P.hh;
    *reinterpret_cast<VF*>(&sm.tl[BUF][hcell]) = P.hl;
    *reinterpret_cast<LW*>(&sm.tb[BUF][hcell]) = (LW)P.hb;
    __syncthreads();
    const VF hym = *reinterpret_cast<const VF*>(&sm.th[BUF][me - RW]);
    const VF lym = *reinterpret_cast<const VF*>(&sm.tl[BUF][me - RW]);
    const VF hyp = *reinterpret_cast<const VF*>(&sm.th[BUF][me + RW]);
    const VF lyp = *reinterpret_cast<const VF*>(&sm.tl[BUF][me + RW]);
    const unsigned bym = *reinterpret_cast<const LW*>(&sm.tb[BUF][me - RW]);
    const unsigned byp = *reinterpret_cast<const LW*>(&sm.tb[BUF][me + RW]);
    const float hzm = sm.th[BUF][me - 1], lzm = sm.tl[BUF][me - 1];
    const float hzp = sm.th[BUF][me + ZV], lzp = sm.tl[BUF][me + ZV];
    const unsigned bzm = sm.tb[BUF][me - 1], bzp = sm.tb[BUF][me + ZV];
    const PlaneW<ZV>& N = q[SN];
    const bool valid = x < x1;  // uniform
    // past the chunk every voxel is computed as held: no contributions
    const unsigned held_all = valid ? 0u : kHeld * (ZV == 4 ? 0x01010101u : 0x0101u);
    const unsigned pb = P.b | held_all;
    VF nh, nl, om = P.om;
    unsigned nlab = 0u;
#pragma unroll
    for (int k = 0; k < ZV; ++k) {
      const unsigned lab = byte_of(pb, k);
      const float zmh = k > 0 ? P.h[k > 0 ? k - 1 : 0] : hzm;
      const float zml = k > 0 ? P.l[k > 0 ? k - 1 : 0] : lzm;
      const unsigned zmb = k > 0 ? byte_of(P.b, k > 0 ? k - 1 : 0) : bzm;
      const float zph = k < ZV - 1 ? P.h[k < ZV - 1 ? k + 1 : 0] : hzp;
      const float zpl = k < ZV - 1 ? P.l[k < ZV - 1 ? k + 1 : 0] : lzp;
      const unsigned zpb = k < ZV - 1 ? byte_of(P.b, k < ZV - 1 ? k + 1 : 0) : bzp;
      const float pf = PERF ? P.pf[k] : 1.0f;
      float h2, l2, o = om[k];
      unsigned lb2;
      voxel_step<ZV == 4>(P.h[k], P.l[k], lab, hm[k], lm[k], byte_of(bm, k), N.h[k], N.l[k],
                 byte_of(N.b, k), hym[k], lym[k], byte_of(bym, k), hyp[k], lyp[k],
                 byte_of(byp, k), zmh, zml, zmb, zph, zpl, zpb, P.s[k], pf, o, sm.cf, sm.cls,
                 K, h2, l2, lb2, acc, PERF);
      nh[k] = h2;
      nl[k] = l2;
      om[k] = o;
      nlab |= lb2 << (8 * k);  // lab plus the latch bit: one byte
    }
    {
      const int so = (min(x, x1 - 1) - xb) * (int)psz;  // uniform
      // st4 = kOob plus a plane offset below 2^31 stays out of range
      const unsigned v4 = valid ? st4 + 4u * (unsigned)so : kOob;
      stv<ZV, AUX>(nh, r_hio, v4);
      stv<ZV, AUX>(nl, r_loo, v4);
      if constexpr (!TONLY) {
        stv<ZV, AUX>(om, r_om, v4);
        // past the chunk the computed bytes carry the held flag: never stored
        stb<ZV, AUX>(nlab, r_lab, (valid && nlab != P.b) ? st1 : kOob, so);
      }
    }
    hm = P.h;
    lm = P.l;
    bm = P.b;
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  static_assert(kRingW == 4, "unrolled for a ring of four planes");
  for (int x = x0; x < x1; x += kRingW) {
    plane_step(I0{}, x);
    plane_step(I1{}, x + 1);
    plane_step(I2{}, x + 2);
    plane_step(I3{}, x + 3);
  }

  if (b.partials) write_partials(acc, sm.red, TY, b.partials + (size_t)wg * 3);
}

TiledShape wide_shape(Grid3 g, int zv, int ty, int xc) {
  TiledShape s;
  s.ty = ty;
  s.xc = xc;
  s.tiles_z = (g.nz + 64 * zv - 1) / (64 * zv);
  s.tiles_y = (g.ny + ty - 1) / ty;
  s.chunks_x = (g.nx + xc - 1) / xc;
  s.nwg = s.tiles_z * s.tiles_y * s.chunks_x;
  return s;
}

bool wide_fits(Grid3 g, int zv, int xc) {
  // rows must start on a ZV-voxel boundary; planes x0 - 1 .. x0 + xc are
  // addressed by signed 32-bit byte offsets
  return (zv == 2 || zv == 4) && g.nz % zv == 0 &&
         (double)(xc + 2) * g.ny * g.nz * 4.0 < 2147483647.0;
}

template <int ZV, int TY, int AUX, bool TONLY>
static hipError_t launch_wide_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                                 const StepConst& K, hipStream_t st) {
  dim3 grid(s.nwg), block(64 * TY);
  if (b.perf)
    hipLaunchKernelGGL((k_step_wide<ZV, TY, true, AUX, TONLY>), grid, block, 0, st, b, K, g.nx,
                       g.ny, g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  else
    hipLaunchKernelGGL((k_step_wide<ZV, TY, false, AUX, TONLY>), grid, block, 0, st, b, K, g.nx,
                       g.ny, g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  return hipGetLastError();
}

template <int ZV, int TY, bool TONLY>
static hipError_t launch_wide_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                                 const StepConst& K, int store, hipStream_t st) {
  switch (store) {
    case kPolicyThrough: return launch_wide_ty<ZV, TY, kStoreThrough, TONLY>(s, g, b, K, st);
    case kPolicyStream: return launch_wide_ty<ZV, TY, kStoreStream, TONLY>(s, g, b, K, st);
    default: return launch_wide_ty<ZV, TY, kStoreBack, TONLY>(s, g, b, K, st);
  }
}

template <bool TONLY>
static hipError_t launch_wide(int zv, const TiledShape& s, Grid3 g, const StepBuffers& b,
                              const StepConst& K, int store, hipStream_t st) {
  if (!wide_fits(g, zv, s.xc)) return hipErrorInvalidValue;
  if (zv == 4 && s.ty == 4) return launch_wide_ty<4, 4, TONLY>(s, g, b, K, store, st);
  if (zv == 4 && s.ty == 8) return launch_wide_ty<4, 8, TONLY>(s, g, b, K, store, st);
  if (zv == 2 && s.ty == 4) return launch_wide_ty<2, 4, TONLY>(s, g, b, K, store, st);
  if (zv == 2 && s.ty == 8) return launch_wide_ty<2, 8, TONLY>(s, g, b, K, store, st);
  return hipErrorInvalidValue;
}

hipError_t launch_step_wide(int zv, const TiledShape& s, Grid3 g, const StepBuffers& b,
                            const StepConst& K, int store, hipStream_t st) {
  return launch_wide<false>(zv, s, g, b, K, store, st);
}

hipError_t launch_step_wide_temperature(int zv, const TiledShape& s, Grid3 g,
                                        const StepBuffers& b, const StepConst& K, int store,
                                        hipStream_t st) {
  return launch_wide<true>(zv, s, g, b, K, store, st);
}

}  // namespace rfa
