// rfa_tiled2.hip -- temporal blocking: two explicit steps per launch.
//
// A work-group of TY wavefronts covers a footprint of 64 (z, one voxel per
// lane) by TY (y, one row per wave) voxel columns and marches along x over
// a chunk of xc planes.  At plane j it computes the first step (n -> n+1)
// on the whole footprint and, one plane behind, the second step
// (n+1 -> n+2) of plane j - 1 on the footprint's interior of 62 x (TY - 2)
// columns: the voxels it owns and stores.  The first step's values on the
// footprint's rim and on the plane either side of the chunk are computed by
// the neighbouring work-groups too (overlapped halo), so only the state
// after two steps goes back to memory: temperature, class bytes, source and
// damage integral cross HBM once per two steps.
//
// LDS holds, double-buffered by plane, the step-n plane with a one-voxel
// halo ring (neighbours of the first step) and the step-(n+1) plane over
// the footprint (neighbours of the second step).  The two write sets of a
// plane are published by one barrier:
//   iteration j:  write step-n plane j and step-(n+1) plane j-1;  barrier;
//                 first step of plane j;  second step of plane j-1.
// A buffer written in iteration j was last read in iteration j-2, and
// every wave has passed the barrier of iteration j-1 since.
//
// Both steps are voxel_step() of rfa_device.h in the same operation order
// as the one-step kernels, so one launch here leaves the state bitwise
// equal to two one-step launches.  The first step at a position outside the
// grid (clamped onto the held (0, 0) column) or next to an unwritten LDS
// cell only ever feeds a held voxel or a voxel that is not stored.
// Concurrent work-groups write only the voxels they own; the values they
// read from other work-groups' voxels (damage integral, latch bit) only
// reach outputs that are not stored.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rfa_tile_common.h"
#include "rfa_tiled.h"

namespace rfa {

namespace {

using namespace tile;

constexpr int kAhead2 = 2;  // planes loaded ahead of the first step
constexpr int kRing2 = 4;   // register ring: planes j-1 (second step), j, j+1, j+2
constexpr int kInnerZ = 62;

struct Plane2 {
  float h, l;       // own column state at step n
  unsigned b;       // own column label byte
  float hh, hl;     // halo element state
  unsigned hb;      // halo element label byte
  float s, om, pf;  // own voxel: source increment, damage integral, perfusion factor
};

template <int TY>
struct Tile2Smem {
  static constexpr int W = 66;            // 64 lanes + z halo
  static constexpr int ROWS = TY + 2;     // TY rows + y halo
  static constexpr int CELLS = ROWS * W;  // plus one scratch cell for threads without halo
  float2 cf[3 * kMaxClasses * kMaxClasses];
  float4 cls[kMaxClasses];
  float2 t0[2][CELLS + 1];  // step n, footprint + halo ring
  uint8_t b0[2][CELLS + 1];
  float2 t1[2][CELLS];      // step n+1, footprint cells
  uint8_t b1[2][CELLS];
  float red[3 * TY];
};

}  // namespace

template <int TY, bool PERF, int AUX>
__global__ __launch_bounds__(64 * TY) void k_step_tiled2(StepBuffers b, StepConst K, int nx,
                                                         int ny, int nz, int xc, int tiles_z,
                                                         int tiles_y, int nwg) {
  static_assert(TY >= 4, "the owned interior needs rows");
  constexpr int W = Tile2Smem<TY>::W;
  constexpr int CELLS = Tile2Smem<TY>::CELLS;
  __shared__ Tile2Smem<TY> sm;
  stage_tables(sm.cf, sm.cls, b.tab, b.n_classes, 64 * TY);

  const int wg = remap_xcd(blockIdx.x, nwg);
  const int tz = wg % tiles_z;
  const int ty = (wg / tiles_z) % tiles_y;
  const int tx = wg / (tiles_z * tiles_y);
  const int lane = threadIdx.x & 63;
  const int wy = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  const int z0 = tz * kInnerZ - 1;  // footprint origin
  const int y0 = ty * (TY - 2) - 1;
  const int z = z0 + lane;
  const int y = y0 + wy;
  const bool in_grid = z >= 0 && z < nz && y >= 0 && y < ny;
  const bool owner = in_grid && lane >= 1 && lane <= kInnerZ && wy >= 1 && wy <= TY - 2;
  const int wy_u = __builtin_amdgcn_readfirstlane(wy);
  const bool inner_row = wy_u >= 1 && wy_u <= TY - 2;  // uniform per wave
  const int x0 = tx * xc;
  const int x1 = min(x0 + xc, nx);
  const int xb = max(x0 - 2, 0);          // first plane the descriptors cover
  const int xs_hi = min(x1 + 1, nx - 1);  // last plane of state reads
  const int xf_lo = max(x0 - 1, 0);       // planes of first-step inputs
  const int xf_hi = min(x1, nx - 1);
  const unsigned psz = (unsigned)(ny * nz);
  const unsigned col = in_grid ? (unsigned)(y * nz + z) : 0u;

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

  // Halo element of the step-n plane owned by this thread (at most one).
  int hcell = CELLS, hy = -1, hz = -1;
  {
    int hrow = 0, hcol = 0;
    if (tid < 64) {
      hrow = 0; hcol = tid + 1; hy = y0 - 1; hz = z0 + tid;
    } else if (tid < 128) {
      hrow = TY + 1; hcol = tid - 64 + 1; hy = y0 + TY; hz = z0 + tid - 64;
    } else if (tid < 128 + TY) {
      hrow = tid - 128 + 1; hcol = 0; hy = y0 + tid - 128; hz = z0 - 1;
    } else if (tid < 128 + 2 * TY) {
      hrow = tid - 128 - TY + 1; hcol = 65; hy = y0 + tid - 128 - TY; hz = z0 + 64;
    }
    if (hy >= 0 && hy < ny && hz >= 0 && hz < nz) hcell = hrow * W + hcol;
  }
  const unsigned hoff = hcell < CELLS ? (unsigned)(hy * nz + hz) : col;

  auto load = [&](int x, Plane2& q) {
    const int xs = min(max(x, 0), xs_hi) - xb;      // uniform
    const int xf = min(max(x, xf_lo), xf_hi) - xb;  // uniform
    const int ss4 = xs * (int)psz * 4, ss1 = xs * (int)psz;
    const int sf4 = xf * (int)psz * 4, sf1 = xf * (int)psz;
    q.h = ld_f32(r_hi, col * 4, ss4);
    q.l = ld_f32(r_lo, col * 4, ss4);
    q.b = ld_u8(r_lab, col, ss1);
    q.s = ld_f32(r_src, col * 4, sf4);
    q.om = ld_f32(r_om, col * 4, sf4);
    q.pf = PERF ? ld_f32(r_pf, col * 4, sf4) : 1.0f;
    q.hh = ld_f32(r_hi, hoff * 4, sf4);
    q.hl = ld_f32(r_lo, hoff * 4, sf4);
    q.hb = ld_u8(r_lab, hoff, sf1);
  };

  // step-n own column at plane j - 1 (x- neighbour of the first step)
  float hm, lm;
  unsigned bm;
  {
    const int ss = (max(x0 - 2, 0) - xb) * (int)psz;
    hm = ld_f32(r_hi, col * 4, ss * 4);
    lm = ld_f32(r_lo, col * 4, ss * 4);
    bm = ld_u8(r_lab, col, ss);
  }
  Plane2 q[kRing2];
  load(x0 - 1, q[0]);
  load(x0, q[1]);
  // step-(n+1) own column at planes j - 1 (p) and j - 2 (pp)
  float h1p = 0.f, l1p = 0.f, om1p = 0.f, h1pp = 0.f, l1pp = 0.f;
  unsigned b1p = 0u, b1pp = 0u;

  Partial acc{0.0f, 0.0f, 0u};
  const int me = (wy + 1) * W + lane + 1;

  // Plane j; S = its ring slot, BUF = its LDS buffer (both compile time).
  auto iter = [&](auto S_, auto BUF_, int j) {
    constexpr int S = decltype(S_)::value;
    constexpr int BUF = decltype(BUF_)::value;
    constexpr int SN = (S + 1) % kRing2;        // plane j + 1
    constexpr int SP = (S + kRing2 - 1) % kRing2;  // plane j - 1
    constexpr int SL = (S + kAhead2) % kRing2;  // receives plane j + 2
    load(j + kAhead2, q[SL]);
    const Plane2& P = q[S];
    sm.t0[BUF][me] = make_float2(P.h, P.l);
    sm.b0[BUF][me] = (uint8_t)P.b;
    sm.t0[BUF][hcell] = make_float2(P.hh, P.hl);
    sm.b0[BUF][hcell] = (uint8_t)P.hb;
    sm.t1[1 - BUF][me] = make_float2(h1p, l1p);
    sm.b1[1 - BUF][me] = (uint8_t)b1p;
    __syncthreads();

    // first step, plane j, whole footprint
    float h1, l1, om1 = P.om;
    unsigned b1;
    {
      const float2 ym = sm.t0[BUF][me - W], yp = sm.t0[BUF][me + W];
      const float2 zm = sm.t0[BUF][me - 1], zp = sm.t0[BUF][me + 1];
      const unsigned bym = sm.b0[BUF][me - W], byp = sm.b0[BUF][me + W];
      const unsigned bzm = sm.b0[BUF][me - 1], bzp = sm.b0[BUF][me + 1];
      const Plane2& N = q[SN];
      Partial p1{0.0f, 0.0f, 0u};
      voxel_step(P.h, P.l, P.b, hm, lm, bm, N.h, N.l, N.b, ym.x, ym.y, bym, yp.x, yp.y, byp,
                 zm.x, zm.y, bzm, zp.x, zp.y, bzp, P.s, P.pf, om1, sm.cf, sm.cls, K, h1, l1, b1,
                 p1, PERF);
      const bool own1 = owner && j >= x0 && j < x1;
      acc.perf += own1 ? p1.perf : 0.0f;
      acc.bnd += own1 ? p1.bnd : 0.0f;
      acc.mono += own1 ? p1.mono : 0u;
    }

    // second step, plane j - 1, stored by the owners while it lies in the
    // chunk (every pass issues the same memory instructions; see below).
    // The footprint's first and last rows own nothing: their waves skip the
    // arithmetic (a wave-uniform branch around LDS reads and VALU only).
    {
      const bool keep = owner && j > x0 && j <= x1;
      const Plane2& Q = q[SP];
      float h2 = h1p, l2 = l1p, om2 = om1p;
      unsigned b2 = b1p;
      Partial p2{0.0f, 0.0f, 0u};
      if (inner_row) {
        const float2 ym = sm.t1[1 - BUF][me - W], yp = sm.t1[1 - BUF][me + W];
        const float2 zm = sm.t1[1 - BUF][me - 1], zp = sm.t1[1 - BUF][me + 1];
        const unsigned bym = sm.b1[1 - BUF][me - W], byp = sm.b1[1 - BUF][me + W];
        const unsigned bzm = sm.b1[1 - BUF][me - 1], bzp = sm.b1[1 - BUF][me + 1];
        voxel_step(h1p, l1p, b1p, h1pp, l1pp, b1pp, h1, l1, b1, ym.x, ym.y, bym, yp.x, yp.y,
                   byp, zm.x, zm.y, bzm, zp.x, zp.y, bzp, Q.s, Q.pf, om2, sm.cf, sm.cls, K, h2,
                   l2, b2, p2, PERF);
      }
      const int so = (min(max(j - 1, x0), x1 - 1) - xb) * (int)psz;  // uniform
      const unsigned v4 = keep ? col * 4 : kOob;
      st_f32<AUX>(h2, r_hio, v4, so * 4);
      st_f32<AUX>(l2, r_loo, v4, so * 4);
      st_f32<AUX>(om2, r_om, v4, so * 4);
      st_u8<AUX>(b2, r_lab, (keep && b2 != Q.b) ? col : kOob, so);
      acc.perf += keep ? p2.perf : 0.0f;
      acc.bnd += keep ? p2.bnd : 0.0f;
      acc.mono += keep ? p2.mono : 0u;
    }
    h1pp = h1p;
    l1pp = l1p;
    b1pp = b1p;
    h1p = h1;
    l1p = l1;
    b1p = b1;
    om1p = om1;
    hm = P.h;
    lm = P.l;
    bm = P.b;
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  static_assert(kRing2 == 4, "unrolled for a ring of four planes");
  // Planes x0 - 1 .. x1: plane x0 - 1 + k uses ring slot k % 4 and LDS buffer
  // k & 1.  Every pass runs all four planes and issues the same loads and
  // stores: stores outside the chunk or by non-owners get an out-of-range
  // buffer offset (dropped by the hardware), so no branch surrounds a memory
  // instruction and the compiler's wait counts stay exact.
  for (int j = x0 - 1; j <= x1; j += kRing2) {
    iter(I0{}, I0{}, j);
    iter(I1{}, I1{}, j + 1);
    iter(I2{}, I0{}, j + 2);
    iter(I3{}, I1{}, j + 3);
  }

  if (b.partials) write_partials(acc, sm.red, TY, b.partials + (size_t)wg * 3);
}

TiledShape tiled2_shape(Grid3 g, int ty, int xc) {
  TiledShape s;
  s.ty = ty;
  s.xc = xc;
  s.tiles_z = (g.nz + kInnerZ - 1) / kInnerZ;
  s.tiles_y = (g.ny + (ty - 2) - 1) / (ty - 2);
  s.chunks_x = (g.nx + xc - 1) / xc;
  s.nwg = s.tiles_z * s.tiles_y * s.chunks_x;
  return s;
}

bool tiled2_fits(Grid3 g, int xc) {
  // planes x0 - 2 .. x0 + xc + 1 are addressed by signed 32-bit byte offsets
  return (double)(xc + 4) * g.ny * g.nz * 4.0 < 2147483647.0;
}

template <int TY, int AUX>
static hipError_t launch2_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                             const StepConst& K, hipStream_t st) {
  dim3 grid(s.nwg), block(64 * TY);
  if (b.perf)
    hipLaunchKernelGGL((k_step_tiled2<TY, true, AUX>), grid, block, 0, st, b, K, g.nx, g.ny,
                       g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  else
    hipLaunchKernelGGL((k_step_tiled2<TY, false, AUX>), grid, block, 0, st, b, K, g.nx, g.ny,
                       g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  return hipGetLastError();
}

template <int TY>
static hipError_t launch2_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                             const StepConst& K, int store, hipStream_t st) {
  switch (store) {
    case kPolicyThrough: return launch2_ty<TY, kStoreThrough>(s, g, b, K, st);
    case kPolicyStream: return launch2_ty<TY, kStoreStream>(s, g, b, K, st);
    default: return launch2_ty<TY, kStoreBack>(s, g, b, K, st);
  }
}

hipError_t launch_step_tiled2(const TiledShape& s, Grid3 g, const StepBuffers& b,
                              const StepConst& K, int store, hipStream_t st) {
  if (!tiled2_fits(g, s.xc)) return hipErrorInvalidValue;
  switch (s.ty) {
    case 8: return launch2_ty<8>(s, g, b, K, store, st);
    case 16: return launch2_ty<16>(s, g, b, K, store, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rfa
