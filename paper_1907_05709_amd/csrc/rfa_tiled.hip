// rfa_tiled.hip -- the production step kernel: 2.5-D tiles marching along x.
//
// A work-group of TY wavefronts owns a tile of 64 (z, one voxel per lane)
// by TY (y, one row per wave) voxel columns and marches along x over a
// chunk of xc planes.  The y and z neighbours of plane x come from a
// double-buffered LDS copy of the plane with a one-voxel halo; the x
// neighbours from registers.  Each voxel's state is read from HBM once per
// step, plus the halo ring of the tile.
//
// Latency hiding: the loads of plane x + AHEAD (own column, halo element,
// damage integral) are issued while plane x is computed, into a ring of
// kSlots register sets (AHEAD = 3 in the single-grid kernel; 2 in the batch
// kernel, whose 64 registers let eight waves per SIMD hide the rest, +5 %
// on the planning sweep); the source increment of plane x + AHEAD - 1 is
// loaded with them, only for voxels whose class byte (then in registers)
// carries the source flag (s is exactly 0 elsewhere).  The x loop is unrolled kSlots times
// so every ring index is a compile-time constant (no register moves).  One
// barrier per plane.  Every pass of the unrolled loop computes all kSlots
// planes and issues the same loads and stores, whatever the chunk length:
// planes past the chunk's end are computed as held voxels and their stores
// (like those of lanes outside the grid, and unchanged latch bytes) get an
// out-of-range buffer offset, which the hardware drops.  With no branch
// around a memory instruction, the compiler's wait counts stay exact and a
// plane waits only for its own loads, not for the ones in flight behind it.
//
// Addressing: every array is accessed through a buffer descriptor whose
// base is the first plane the work-group touches; a lane adds a fixed
// 32-bit byte offset (its column) and the plane enters as a uniform scalar
// offset, so loads and stores cost no vector address arithmetic.  Lanes
// whose column lies outside the grid read the grid's (0, 0) column, which
// is on the held outer layer, and store nothing.
//
// Work-group ids are remapped so consecutive tiles on one XCD are spatial
// neighbours and share their halo rows in that XCD's L2.
//
// The per-voxel arithmetic is voxel_step() of rfa_device.h, identical to
// the reference kernel, so both produce bitwise-equal states.  A held
// voxel's result does not depend on its neighbours, so held and free voxels
// share one instruction stream.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rfa_tile_common.h"
#include "rfa_tiled.h"

namespace rfa {

namespace {

using namespace tile;

constexpr int kAhead = 3;  // planes in flight ahead of the computed one (at most)
constexpr int kSlots = 4;  // register ring size

// Registers of one plane for one thread.
struct Plane {
  float h, l;       // own column state
  unsigned b;       // own column label byte
  float hh, hl;     // halo element state
  unsigned hb;      // halo element label byte
  float s, om, pf;  // own voxel: source increment, damage integral, perfusion factor
};

// Buffer descriptors of the arrays, based at plane xb of the grid.
struct Rsrc {
  __amdgpu_buffer_rsrc_t hi_in, lo_in, lab, src, om, perf, hi_out, lo_out;
};

struct TileCtx {
  Rsrc r;
  int xb;            // first plane covered by the descriptors
  int nx, x1;
  unsigned psz;      // plane size, voxels
  unsigned col;      // own column offset (voxels) in a plane
  unsigned hoff;     // halo element offset (voxels) in a plane
};

__device__ __forceinline__ void load_plane(const TileCtx& c, int x, bool perf, Plane& q) {
  const int xo = min(x, c.nx - 1) - c.xb;   // uniform
  const int xf = min(x, c.x1 - 1) - c.xb;   // uniform
  const int so4 = xo * (int)c.psz * 4, so1 = xo * (int)c.psz;
  const int sf4 = xf * (int)c.psz * 4, sf1 = xf * (int)c.psz;
  q.h = ld_f32(c.r.hi_in, c.col * 4, so4);
  q.l = ld_f32(c.r.lo_in, c.col * 4, so4);
  q.b = ld_u8(c.r.lab, c.col, so1);
  q.om = ld_f32(c.r.om, c.col * 4, sf4);
  q.pf = perf ? ld_f32(c.r.perf, c.col * 4, sf4) : 1.0f;
  q.hh = ld_f32(c.r.hi_in, c.hoff * 4, sf4);
  q.hl = ld_f32(c.r.lo_in, c.hoff * 4, sf4);
  q.hb = ld_u8(c.r.lab, c.hoff, sf1);
}

// Source increment of plane x for a voxel whose class byte (already in q.b)
// carries the source flag; elsewhere s is exactly 0 and is not read.
__device__ __forceinline__ void load_src(const TileCtx& c, int x, Plane& q) {
  const int sf4 = (min(x, c.x1 - 1) - c.xb) * (int)c.psz * 4;  // uniform
  q.s = ld_f32(c.r.src, (q.b & kSource) ? c.col * 4 : kOob, sf4);
}



// LDS working set of one work-group (2.5-D tile: 64 z by TY rows).
template <int TY>
struct TileSmem {
  static constexpr int W = 66;            // 64 lanes + z halo
  static constexpr int ROWS = TY + 2;     // TY rows + y halo
  static constexpr int CELLS = ROWS * W;  // plus one scratch cell for threads without halo
  float2 cf[3 * kMaxClasses * kMaxClasses];
  float4 cls[kMaxClasses];
  float2 ts[2][CELLS + 1];
  uint8_t bs[2][CELLS + 1];
  float red[3][TY];
};

// LDS working set of a flat work-group: T = 64 NW consecutive voxels of a
// plane in (y, z) order, plus nz voxels before and after them (the y
// neighbours); grids up to nz = T / 2.
template <int NW>
struct FlatSmem {
  static constexpr int T = 64 * NW;
  static constexpr int MAX_NZ = T / 2;
  static constexpr int CELLS = T + 2 * MAX_NZ;  // plus one scratch cell
  float2 cf[3 * kMaxClasses * kMaxClasses];
  float4 cls[kMaxClasses];
  float2 ts[2][CELLS + 1];
  uint8_t bs[2][CELLS + 1];
  float red[3][NW];
};

// Where one thread sits in its work-group's LDS plane.
struct LanePlace {
  unsigned col;   // own column offset (voxels) in a plane; 0 outside the grid
  bool inside;    // own column inside the grid
  int me;         // own LDS cell
  int ys;         // LDS distance of the y neighbours (z neighbours: 1)
  int hcell;      // LDS cell this thread fills with a halo element, or the scratch cell
  unsigned hoff;  // plane offset (voxels) of the element it loads for hcell, in range
};

// 2.5-D tile (tz, ty): 64 z voxels (one per lane) by TY rows (one per wave);
// halo rows y0-1 / y0+TY and columns z0-1 / z0+64.  Halo elements outside
// the grid go to the scratch cell: the cells they stand for feed held
// voxels only.
template <int TY>
__device__ __forceinline__ LanePlace tile_place(int ny, int nz, int tz, int ty) {
  constexpr int W = TileSmem<TY>::W;
  constexpr int CELLS = TileSmem<TY>::CELLS;
  const int lane = threadIdx.x & 63;
  const int wy = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  const int z = tz * 64 + lane;
  const int y = ty * TY + wy;
  LanePlace p;
  p.inside = z < nz && y < ny;
  p.col = p.inside ? (unsigned)(y * nz + z) : 0u;
  p.me = (wy + 1) * W + lane + 1;
  p.ys = W;
  int hcell = CELLS, hy = -1, hz = -1;
  {
    const int y0 = ty * TY, z0 = tz * 64;
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
  p.hcell = hcell;
  p.hoff = hcell < CELLS ? (unsigned)(hy * nz + hz) : p.col;
  return p;
}

// Flat segment t of a plane: voxels [t T, t T + T) in (y, z) order, one per
// thread.  z neighbours are the adjacent cells (at a row's ends both the
// voxel and the cell belong to the held outer layer), y neighbours nz cells
// away; the nz voxels before and after the segment are the halo, loaded by
// threads 0 .. 2 nz - 1 (nz <= T / 2).  Halo cells outside the plane are
// filled from the thread's own column: finite values that feed held
// voxels only.  Only a plane's last segment has idle lanes.
template <int NW>
__device__ __forceinline__ LanePlace flat_place(int ny, int nz, int t) {
  constexpr int T = FlatSmem<NW>::T;
  constexpr int CELLS = FlatSmem<NW>::CELLS;
  const int i = threadIdx.x;
  const int np = ny * nz;
  const int f0 = t * T, f = f0 + i;
  LanePlace p;
  p.inside = f < np;
  p.col = p.inside ? (unsigned)f : 0u;
  p.me = nz + i;
  p.ys = nz;
  int h = -1;
  p.hcell = CELLS;
  if (i < nz) {
    p.hcell = i; h = f0 - nz + i;
  } else if (i < 2 * nz) {
    p.hcell = nz + T + (i - nz); h = f0 + T + (i - nz);
  }
  p.hoff = (h >= 0 && h < np) ? (unsigned)h : p.col;
  return p;
}

// March one work-group's placement over the x-chunk [tx*xc, tx*xc + xc) of
// one grid.  ts / bs: the two LDS plane buffers (cells cells apart).  Tables
// must be staged (a barrier inside the march orders them).  The
// work-group's partial sums are written to partials[wg_slot * 3] if
// partials is not null.
template <int NT, int AUX, int AHEAD = kAhead>
__device__ __forceinline__ void march(float2* ts, uint8_t* bs, int cells, float* red,
                                      const float2* cf, const float4* cls,
                                      const StepBuffers& b, const StepConst& K, bool perf,
                                      int nx, int ny, int nz, int xc, int tx,
                                      const LanePlace& lp, float* partials, int wg_slot) {
  const int x0 = tx * xc;
  TileCtx c;
  c.nx = nx;
  c.x1 = min(x0 + xc, nx);
  c.xb = max(x0 - 1, 0);
  c.psz = (unsigned)(ny * nz);
  c.col = lp.col;
  c.hoff = lp.hoff;
  {
    const size_t off = (size_t)c.xb * c.psz;
    const size_t rest = (size_t)(nx - c.xb) * c.psz;
    c.r.hi_in = make_rsrc(b.hi_in + off, rest * 4);
    c.r.lo_in = make_rsrc(b.lo_in + off, rest * 4);
    c.r.lab = make_rsrc(b.lab + off, rest);
    c.r.src = make_rsrc(b.src + off, rest * 4);
    c.r.om = make_rsrc(b.omega + off, rest * 4);
    c.r.perf = make_rsrc(perf ? b.perf + off : b.src + off, rest * 4);
    c.r.hi_out = make_rsrc(b.hi_out + off, rest * 4);
    c.r.lo_out = make_rsrc(b.lo_out + off, rest * 4);
  }

  // x-1 neighbour of the plane being computed (own column)
  float hm, lm;
  unsigned bm;
  {
    const int so = (max(x0 - 1, 0) - c.xb) * (int)c.psz;
    hm = ld_f32(c.r.hi_in, c.col * 4, so * 4);
    lm = ld_f32(c.r.lo_in, c.col * 4, so * 4);
    bm = ld_u8(c.r.lab, c.col, so);
  }
  static_assert(AHEAD >= 1 && AHEAD < kSlots && AHEAD <= kAhead, "ring depth");
  Plane q[kSlots];
#pragma unroll
  for (int k = 0; k < AHEAD; ++k) load_plane(c, x0 + k, perf, q[k]);
#pragma unroll
  for (int k = 0; k < AHEAD - 1; ++k) load_src(c, x0 + k, q[k]);

  Partial acc{0.0f, 0.0f, 0u};
  const int me = lp.me, ys = lp.ys, hcell = lp.hcell;
  const unsigned st4 = lp.inside ? c.col * 4 : kOob;  // store offsets (out of range: dropped)
  const unsigned st1 = lp.inside ? c.col : kOob;

  // One plane; S = ring slot of plane x (compile time), BUF = LDS buffer.
  auto plane_step = [&](auto S_, auto BUF_, int x) {
    constexpr int S = decltype(S_)::value;
    constexpr int BUF = decltype(BUF_)::value;
    constexpr int SN = (S + 1) % kSlots;       // plane x+1
    constexpr int SL = (S + AHEAD) % kSlots;      // slot receiving plane x+AHEAD
    constexpr int SS = (S + AHEAD - 1) % kSlots;  // plane x+AHEAD-1: its source
    load_plane(c, x + AHEAD, perf, q[SL]);
    load_src(c, x + AHEAD - 1, q[SS]);
    const Plane& P = q[S];
    float2* t2 = ts + BUF * cells;
    uint8_t* t1 = bs + BUF * cells;
    t2[me] = make_float2(P.h, P.l);
    t1[me] = (uint8_t)P.b;
    t2[hcell] = make_float2(P.hh, P.hl);
    t1[hcell] = (uint8_t)P.hb;
    __syncthreads();
    const float2 ym = t2[me - ys], yp = t2[me + ys];
    const float2 zm = t2[me - 1], zp = t2[me + 1];
    const unsigned bym = t1[me - ys], byp = t1[me + ys];
    const unsigned bzm = t1[me - 1], bzp = t1[me + 1];
    const Plane& N = q[SN];
    float nh, nl, om = P.om;
    unsigned nlab;
    const bool valid = x < c.x1;                        // uniform
    const unsigned lab = P.b | (valid ? 0u : kHeld);   // past the chunk: no contributions
    voxel_step(P.h, P.l, lab, hm, lm, bm, N.h, N.l, N.b, ym.x, ym.y, bym, yp.x, yp.y, byp,
               zm.x, zm.y, bzm, zp.x, zp.y, bzp, P.s, P.pf, om, cf, cls, K, nh, nl, nlab,
               acc, perf);
    {
      const int so = (min(x, c.x1 - 1) - c.xb) * (int)c.psz;  // uniform
      const unsigned v4 = valid ? st4 : kOob;
      st_f32<AUX>(nh, c.r.hi_out, v4, so * 4);
      st_f32<AUX>(nl, c.r.lo_out, v4, so * 4);
      st_f32<AUX>(om, c.r.om, v4, so * 4);
      st_u8<AUX>(nlab, c.r.lab, (valid && nlab != P.b) ? st1 : kOob, so);
    }
    hm = P.h;
    lm = P.l;
    bm = P.b;
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  static_assert(kSlots == 4, "unrolled for a ring of four planes");
  // kSlots is even, so plane x uses LDS buffer (x - x0) & 1 = slot & 1.
  for (int x = x0; x < c.x1; x += kSlots) {
    plane_step(I0{}, I0{}, x);
    plane_step(I1{}, I1{}, x + 1);
    plane_step(I2{}, I0{}, x + 2);
    plane_step(I3{}, I1{}, x + 3);
  }

  if (partials) write_partials(acc, red, NT, partials + (size_t)wg_slot * 3);
}

}  // namespace

template <int TY, bool PERF, int AUX>
__global__ __launch_bounds__(64 * TY) void k_step_tiled(StepBuffers b, StepConst K, int nx,
                                                        int ny, int nz, int xc, int tiles_z,
                                                        int tiles_y, int nwg) {
  __shared__ TileSmem<TY> sm;
  stage_tables(sm.cf, sm.cls, b.tab, b.n_classes, 64 * TY);
  const int wg = remap_xcd(blockIdx.x, nwg);
  const int tz = wg % tiles_z;
  const int ty = (wg / tiles_z) % tiles_y;
  const int tx = wg / (tiles_z * tiles_y);
  const LanePlace lp = tile_place<TY>(ny, nz, tz, ty);
  march<TY, AUX>(&sm.ts[0][0], &sm.bs[0][0], TileSmem<TY>::CELLS + 1, &sm.red[0][0], sm.cf,
                 sm.cls, b, K, PERF, nx, ny, nz, xc, tx, lp, b.partials, wg);
}

// Batched step over the work list of all instances (items grouped by
// instance).  LOOP: a persistent grid walks the list round-robin; otherwise
// one work-group per item, in XCD-aware order, at eight waves per SIMD (64
// registers with a ring two planes deep, no spills).  FLAT: items are flat plane
// segments of 64 TY voxels (item tz = segment), else 2.5-D tiles.  Each
// item stages its instance's tables before its march.  parity selects the
// ping-pong image.
template <int TY, bool PERF, bool LOOP, bool FLAT>
__global__ __launch_bounds__(64 * TY, PERF || LOOP ? 1 : 8) void k_step_batch(const BatchInstance* inst,
                                                        const BatchItem* items, int first_item,
                                                        int n_items, int parity,
                                                        float* partials) {
  using Smem = typename std::conditional<FLAT, FlatSmem<TY>, TileSmem<TY>>::type;
  __shared__ Smem sm;
  // Work item and instance fields are the same for the whole work-group;
  // say so (readfirstlane), so descriptors and constants live in scalar
  // registers as in the single-grid kernel.
  auto ui = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
  auto uf = [](float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
  };
  auto up = [](auto* p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffull));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<decltype(p)>(((unsigned long long)hi << 32) | lo);
  };
  auto one = [&](int it) {
    const BatchItem w = items[it];
    const BatchInstance& I = inst[ui(w.inst)];
    StepBuffers b;
    b.hi_in = up(I.hi[parity]);
    b.lo_in = up(I.lo[parity]);
    b.hi_out = up(I.hi[1 - parity]);
    b.lo_out = up(I.lo[1 - parity]);
    b.lab = up(I.lab);
    b.src = up(I.src);
    b.omega = up(I.om);
    b.perf = up(I.perf);
    b.tab = up(I.tab);
    b.partials = nullptr;
    b.n_classes = ui(I.n_classes);
    StepConst K;
    K.dtka = uf(I.K.dtka);
    K.c2 = uf(I.K.c2);
    K.tak = uf(I.K.tak);
    K.clamp2 = uf(I.K.clamp2);
    K.cap = uf(I.K.cap);
    K.thr = uf(I.K.thr);
    K.decay2 = uf(I.K.decay2);
    stage_tables(sm.cf, sm.cls, b.tab, b.n_classes, 64 * TY);
    const int ny = ui(I.ny), nz = ui(I.nz);
    LanePlace lp;
    if constexpr (FLAT)
      lp = flat_place<TY>(ny, nz, ui(w.tz));
    else
      lp = tile_place<TY>(ny, nz, ui(w.tz), ui(w.ty));
    // groups of a batch are sized to stay in the last-level cache
    march<TY, kStoreBack, 2>(&sm.ts[0][0], &sm.bs[0][0], Smem::CELLS + 1, &sm.red[0][0],
                             sm.cf, sm.cls, b, K, PERF, ui(I.nx), ny, nz, ui(I.xc), ui(w.tx),
                             lp, partials, it);
  };
  if (LOOP) {
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
      one(first_item + k);
      __syncthreads();  // the next item restages the tables
    }
  } else {
    one(first_item + remap_xcd(blockIdx.x, n_items));
  }
}

template <int TY, bool PERF, bool FLAT>
static hipError_t launch_batch_ty(const BatchInstance* inst, const BatchItem* items,
                                  int first_item, int n_items, int n_wg, int parity,
                                  float* partials, hipStream_t st) {
  if (n_wg > 0)
    hipLaunchKernelGGL((k_step_batch<TY, PERF, true, FLAT>), dim3(n_wg), dim3(64 * TY), 0, st,
                       inst, items, first_item, n_items, parity, partials);
  else
    hipLaunchKernelGGL((k_step_batch<TY, PERF, false, FLAT>), dim3(n_items), dim3(64 * TY), 0,
                       st, inst, items, first_item, n_items, parity, partials);
  return hipGetLastError();
}

template <int TY, bool FLAT>
static hipError_t launch_batch_ty(bool perf, const BatchInstance* inst, const BatchItem* items,
                                  int first_item, int n_items, int n_wg, int parity,
                                  float* partials, hipStream_t st) {
  return perf ? launch_batch_ty<TY, true, FLAT>(inst, items, first_item, n_items, n_wg,
                                                parity, partials, st)
              : launch_batch_ty<TY, false, FLAT>(inst, items, first_item, n_items, n_wg,
                                                 parity, partials, st);
}

int flat_max_nz(int ty) { return ty == 16 ? FlatSmem<16>::MAX_NZ : FlatSmem<8>::MAX_NZ; }

TiledShape flat_shape(Grid3 g, int ty, int xc) {
  TiledShape s;
  s.ty = ty;
  s.xc = xc;
  s.tiles_z = (g.ny * g.nz + 64 * ty - 1) / (64 * ty);  // segments of a plane
  s.tiles_y = 1;
  s.chunks_x = (g.nx + xc - 1) / xc;
  s.nwg = s.tiles_z * s.chunks_x;
  return s;
}

TiledShape tiled_shape(Grid3 g, int ty, int xc) {
  TiledShape s;
  s.ty = ty;
  s.xc = xc;
  s.tiles_z = (g.nz + 63) / 64;
  s.tiles_y = (g.ny + ty - 1) / ty;
  s.chunks_x = (g.nx + xc - 1) / xc;
  s.nwg = s.tiles_z * s.tiles_y * s.chunks_x;
  return s;
}

bool tiled_fits(Grid3 g, int xc) {
  // scalar plane offsets are signed 32-bit byte offsets from the chunk base
  return (double)(xc + kAhead + 2) * g.ny * g.nz * 4.0 < 2147483647.0;
}

template <int TY, int AUX>
static hipError_t launch_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                            const StepConst& K, hipStream_t st) {
  dim3 grid(s.nwg), block(64 * TY);
  if (b.perf)
    hipLaunchKernelGGL((k_step_tiled<TY, true, AUX>), grid, block, 0, st, b, K, g.nx, g.ny,
                       g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  else
    hipLaunchKernelGGL((k_step_tiled<TY, false, AUX>), grid, block, 0, st, b, K, g.nx, g.ny,
                       g.nz, s.xc, s.tiles_z, s.tiles_y, s.nwg);
  return hipGetLastError();
}

template <int TY>
static hipError_t launch_ty(const TiledShape& s, Grid3 g, const StepBuffers& b,
                            const StepConst& K, int store, hipStream_t st) {
  switch (store) {
    case kPolicyThrough: return launch_ty<TY, kStoreThrough>(s, g, b, K, st);
    case kPolicyStream: return launch_ty<TY, kStoreStream>(s, g, b, K, st);
    default: return launch_ty<TY, kStoreBack>(s, g, b, K, st);
  }
}

hipError_t launch_step_batch(int ty, bool flat, bool perf, const BatchInstance* inst,
                             const BatchItem* items, int first_item, int n_items, int n_wg,
                             int parity, float* partials, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (!flat && ty == 4)
    return launch_batch_ty<4, false>(perf, inst, items, first_item, n_items, n_wg, parity,
                                     partials, st);
  if (!flat && ty == 8)
    return launch_batch_ty<8, false>(perf, inst, items, first_item, n_items, n_wg, parity,
                                     partials, st);
  if (flat && ty == 8)
    return launch_batch_ty<8, true>(perf, inst, items, first_item, n_items, n_wg, parity,
                                    partials, st);
  if (flat && ty == 16)
    return launch_batch_ty<16, true>(perf, inst, items, first_item, n_items, n_wg, parity,
                                     partials, st);
  return hipErrorInvalidValue;
}

hipError_t launch_step_tiled(const TiledShape& s, Grid3 g, const StepBuffers& b,
                             const StepConst& K, int store, hipStream_t st) {
  if (!tiled_fits(g, s.xc)) return hipErrorInvalidValue;
  switch (s.ty) {
    case 4: return launch_ty<4>(s, g, b, K, store, st);
    case 8: return launch_ty<8>(s, g, b, K, store, st);
    case 16: return launch_ty<16>(s, g, b, K, store, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rfa
