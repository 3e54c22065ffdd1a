// rfa_adjoint.hip -- discrete adjoint of the explicit stepper and the
// perfusion-correction field.
//
// Forward step of a free voxel p (excess temperature theta, class l):
//   theta'_p = theta_p + sum_faces C(l_p, l_q)(theta_q - theta_p)
//              - B_l f_p theta_p + Qs_l + s_p
//   Omega'_p = Omega_p + dt k_a exp(c theta_p / (T_aK + theta_p))    (tissue)
// held voxels keep their value.  For a loss L(Omega^N) with w = dL/dOmega^N
// the adjoint lambda^n = dL/dtheta^n obeys, for free q,
//   lambda^n_q = (1 - sum_faces C(l_q, l_p) - B_l f_q) lambda^{n+1}_q
//              + sum_{free p ~ q} C(l_p, l_q) lambda^{n+1}_p
//              + w_q dt d rate/d theta (theta^n_q)
// and lambda = 0 on held voxels (nothing depends on their value).  Along the
// way dL/ds_p = sum_n lambda^{n+1}_p and dL/df_p = sum_n lambda^{n+1}_p
// (-B_l theta^n_p) are accumulated (s: source increment, f: perfusion
// multiplier).  The exponent cap of the damage rate has zero derivative.
//
// The coefficient tables are the forward's (float-float); the adjoint runs
// in FP32 (gradients are checked to 1e-3 relative).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "rfa_adjoint.h"
#include "rfa_tile_common.h"
#include "rfa_tiled.h"

#include <type_traits>

namespace rfa {

namespace {

__device__ double block_sum_256(double v, double* sh) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Knot span and local coordinate of voxel i of n along an axis carried by
// m control points (uniform cubic B-spline spanning the grid).
__device__ __forceinline__ void span_of(int i, int n, int m, int& s, double& t) {
  const double u = n > 1 ? (double)i * (double)(m - 3) / (double)(n - 1) : 0.0;
  int k = (int)floor(u);
  k = k > m - 4 ? m - 4 : (k < 0 ? 0 : k);
  s = k;
  t = u - k;
}

__device__ __forceinline__ void basis(double t, double* b) {
  const double s = 1.0 - t;
  b[0] = s * s * s / 6.0;
  b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  b[3] = t * t * t / 6.0;
}

}  // namespace

// f = exp(sum_j B_j(x) c_j) on every voxel.
__global__ void k_bspline_eval(const float* ctrl, int m, int nx, int ny, int nz, float* f) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(p % nz), j = (int)((p / nz) % ny), i = (int)(p / ((size_t)nz * ny));
    int si, sj, sk;
    double ti, tj, tk, bi[4], bj[4], bk[4];
    span_of(i, nx, m, si, ti);
    span_of(j, ny, m, sj, tj);
    span_of(k, nz, m, sk, tk);
    basis(ti, bi);
    basis(tj, bj);
    basis(tk, bk);
    double v = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c)
          v += bi[a] * bj[b] * bk[c] * (double)ctrl[((size_t)(si + a) * m + (sj + b)) * m + (sk + c)];
    f[p] = (float)exp(v);
  }
}

hipError_t launch_bspline_eval(Grid3 g, const float* ctrl, int m, float* f, hipStream_t st) {
  hipLaunchKernelGGL(k_bspline_eval, dim3(2048), dim3(256), 0, st, ctrl, m, g.nx, g.ny, g.nz, f);
  return hipGetLastError();
}

// One factor of the separable B-spline transpose: contract the middle axis
// (n voxels) of a [N0][n][N2] array against the m basis functions of that
// axis, out[o0][c][o2] = sum_{i in support(c)} in[o0][i][o2] B_c(i), summed
// in increasing i.  vfirst[s] = first voxel of knot span s (s = 0 .. m-3).
// With in == nullptr the input is gf * f (FP64 products of the two fields).
__global__ __launch_bounds__(256) void k_bspline_contract(const double* in, const float* gf,
                                                          const float* f, long long N0, int n,
                                                          int N2, int m, const int* vfirst,
                                                          double* out) {
  const long long total = N0 * m * N2;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int o2 = (int)(e % N2);
    const long long r = e / N2;
    const int c = (int)(r % m);
    const long long o0 = r / m;
    const int s0 = c - 3 < 0 ? 0 : c - 3;
    const int s1 = c > m - 4 ? m - 4 : c;
    const int lo = vfirst[s0], hi = vfirst[s1 + 1];
    double acc = 0.0;
    for (int i = lo; i < hi; ++i) {
      int sp;
      double t, bb[4];
      span_of(i, n, m, sp, t);
      basis(t, bb);
      const size_t idx = ((size_t)o0 * n + i) * N2 + o2;
      const double v = in ? in[idx] : (double)gf[idx] * (double)f[idx];
      acc += v * bb[c - sp];
    }
    out[e] = acc;
  }
}

hipError_t launch_bspline_grad(Grid3 g, const float* gf, const float* f, int m,
                               const int* vfirst_x, const int* vfirst_y, const int* vfirst_z,
                               double* scratch, double* gctrl, hipStream_t st) {
  // gctrl[a][b][c] = sum_p gf_p f_p Bx_a(i) By_b(j) Bz_c(k): z, then y, then x
  double* t1 = scratch;                               // [nx][ny][m]
  double* t2 = scratch + (size_t)g.nx * g.ny * m;     // [nx][m][m]
  auto blocks = [](long long total) {
    return (unsigned)std::min<long long>((total + 255) / 256, 8192);
  };
  const long long n1 = (long long)g.nx * g.ny * m, n2 = (long long)g.nx * m * m,
                  n3 = (long long)m * m * m;
  hipLaunchKernelGGL(k_bspline_contract, dim3(blocks(n1)), dim3(256), 0, st, nullptr, gf, f,
                     (long long)g.nx * g.ny, g.nz, 1, m, vfirst_z, t1);
  hipLaunchKernelGGL(k_bspline_contract, dim3(blocks(n2)), dim3(256), 0, st, t1, nullptr,
                     nullptr, (long long)g.nx, g.ny, m, m, vfirst_y, t2);
  hipLaunchKernelGGL(k_bspline_contract, dim3(blocks(n3)), dim3(256), 0, st, t2, nullptr,
                     nullptr, 1LL, g.nx, m * m, m, vfirst_x, gctrl);
  return hipGetLastError();
}

size_t bspline_grad_scratch(Grid3 g, int m) {
  return (size_t)g.nx * g.ny * m + (size_t)g.nx * m * m;
}

// w' = w on tissue voxels whose damage integral stayed below the cap, else 0.
__global__ void k_adjoint_weight(const float* w, const float* om, const uint8_t* lab, float cap,
                                 float* wa, size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x)
    wa[p] = ((lab[p] & kTissue) && om[p] < cap) ? w[p] : 0.0f;
}

hipError_t launch_adjoint_weight(Grid3 g, const float* w, const float* om, const uint8_t* lab,
                                 float cap, float* wa, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_weight, dim3(2048), dim3(256), 0, st, w, om, lab, cap, wa, g.n());
  return hipGetLastError();
}

// The face coefficients of one class pair along one axis, each float-float
// table entry rounded to float: x = C(q, p) (q's own row), y = C(p, q).
// Table entries in bytes: row of a class = its masked label << 4, entry =
// the other class's masked label (the label keeps the class times 8).
__device__ __forceinline__ float2 pair_from_table(const float2* __restrict__ cf, int axis,
                                                  unsigned cq, unsigned cp) {
  const char* t = reinterpret_cast<const char*>(cf + axis * kMaxClasses * kMaxClasses);
  const float2 a = *reinterpret_cast<const float2*>(t + ((cq << 4) | cp));
  const float2 b = *reinterpret_cast<const float2*>(t + ((cp << 4) | cq));
  return make_float2(a.x + a.y, b.x + b.y);
}

// Pair table: pc[axis][a][c] = pair_from_table(cf, axis, a, c), built once
// per work-group so the per-voxel update reads one entry per face.
__device__ __forceinline__ void stage_pairs(float2* pc, float4* cls, const Tables* tab,
                                            int nthreads) {
  constexpr int per_axis = kMaxClasses * kMaxClasses;
  for (int t = threadIdx.x; t < 3 * per_axis; t += nthreads) {
    const int ax = t / per_axis, r = t - ax * per_axis;
    const unsigned a = (unsigned)(r / kMaxClasses), c = (unsigned)(r % kMaxClasses);
    pc[t] = pair_from_table(&tab->cf[0][0], ax, a << kClassShift, c << kClassShift);
  }
  if ((int)threadIdx.x < kMaxClasses) cls[threadIdx.x] = tab->cls[threadIdx.x];
}

// Pair-table lookup in the same byte-offset form.
__device__ __forceinline__ float2 pair_from_pairs(const float2* __restrict__ pc, int axis,
                                                  unsigned cq, unsigned cp) {
  const char* t = reinterpret_cast<const char*>(pc + axis * kMaxClasses * kMaxClasses);
  return *reinterpret_cast<const float2*>(t + ((cq << 4) | cp));
}

// Adjoint update of one voxel q: lam_out = (M^T lam_in)_q + w_q dt rate'(theta^n_q),
// and the accumulations sacc += lam_in_q, facc += lam_in_q (-B theta^n_q), for
// a free voxel; a held voxel gets lam_out = 0 and accumulates nothing
// (returns false).  Neighbours in the order x-, x+, y-, y+, z-, z+; pair(axis,
// cq, cp) gives {C(q, p), C(p, q)} for masked labels, from the forward's
// tables or from the pair table (the same floats either way); cls points at
// the class table.  Branch-free: a held voxel's neighbour values may be
// arbitrary (the tiled kernel leaves halo cells outside the grid unwritten)
// and reach nothing but selects on the held flags.
template <class Pair>
__device__ __forceinline__ bool adjoint_voxel(float lam, float th, unsigned lq, float pf,
                                              float w, const float (&nlam)[6],
                                              const unsigned (&nlab)[6], Pair pair,
                                              const float4* __restrict__ cls,
                                              const StepConst& K, float& lam_out,
                                              float& sacc, float& facc) {
  const bool held = (lq & kHeld) != 0u;
  const float4 cl = cls[class_of(lq)];
  const float B = (cl.x + cl.y) * pf;
  const unsigned cq = lq & kClassMask;
  float diag = 1.0f - B;
  float off = 0.0f;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const unsigned lp = nlab[f];
    const float2 c = pair(f >> 1, cq, lp & kClassMask);
    diag -= c.x;                                        // C(q, p): q's own row
    const float o = __builtin_fmaf(c.y, nlam[f], off);  // C(p, q)
    off = (lp & kHeld) ? off : o;
  }
  // damage-rate derivative at theta^n, the rate evaluated as the forward
  // step evaluates it (zero off tissue and where the exponent is capped)
  const float r = __builtin_amdgcn_rcpf(K.tak + th);
  const float x = K.c2 * th * r;
  const float rate = K.dtka * __builtin_amdgcn_exp2f(fminf(x, K.clamp2));
  const float dr0 = rate * (K.c2 * 0.69314718f) * K.tak * (r * r);
  const float dr = ((lq & kTissue) != 0u && x < K.clamp2) ? dr0 : 0.0f;
  const float lo = __builtin_fmaf(diag, lam, off) + w * dr;
  lam_out = held ? 0.0f : lo;
  sacc = held ? sacc : sacc + lam;
  facc = held ? facc : __builtin_fmaf(-cl.x - cl.y, th * lam, facc);
  return !held;
}

// Reference adjoint step, one thread per voxel.
__global__ __launch_bounds__(256) void k_adjoint_step(AdjointBuffers a, StepConst K, int nx,
                                                      int ny, int nz) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int i = blockIdx.z;
  if (k >= nz || j >= ny) return;
  const size_t sx = (size_t)ny * nz, sy = nz;
  const size_t q = (size_t)i * sx + (size_t)j * sy + k;
  const unsigned lq = a.lab[q];
  if (lq & kHeld) {
    a.lam_out[q] = 0.0f;
    return;
  }
  const size_t nb[6] = {q - sx, q + sx, q - sy, q + sy, q - 1, q + 1};
  float nlam[6];
  unsigned nlab[6];
  for (int f = 0; f < 6; ++f) {
    nlam[f] = a.lam_in[nb[f]];
    nlab[f] = a.lab[nb[f]];
  }
  const bool on_src = a.sacc_all || (lq & kSource) != 0u;
  float lo, sa = on_src ? a.sacc[q] : 0.0f, fa = a.facc[q];
  const float2* cf = &a.tab->cf[0][0];
  adjoint_voxel(a.lam_in[q], a.theta[q], lq, a.perf ? a.perf[q] : 1.0f, a.w[q], nlam, nlab,
                [cf](int ax, unsigned cq, unsigned cp) { return pair_from_table(cf, ax, cq, cp); },
                a.tab->cls, K, lo, sa, fa);
  a.lam_out[q] = lo;
  if (on_src) a.sacc[q] = sa;
  a.facc[q] = fa;
}

namespace {

constexpr int kAdjAhead = 3;             // planes in flight ahead of the computed one
constexpr int kAdjRing = kAdjAhead + 1;  // register ring (unroll factor)

struct AdjPlane {
  float lam;      // own lambda^{n+1}
  unsigned b;     // own class byte
  float hl;       // halo element lambda
  unsigned hb;    // halo element class byte
  float th, w, pf, sa, fa;
};

template <int TY>
struct AdjSmem {
  static constexpr int W = 66;
  static constexpr int ROWS = TY + 2;
  static constexpr int CELLS = ROWS * W;
  float2 pc[3 * kMaxClasses * kMaxClasses];  // pair table
  float4 cls[kMaxClasses];
  float lam[2][CELLS + 1];
  uint8_t lab[2][CELLS + 1];
};

}  // namespace

// Adjoint step with the production step kernel's schedule: a work-group of
// TY waves owns a 64 (z) x TY (y) tile and marches along x; y and z
// neighbours of lambda and the class byte come from a double-buffered LDS
// plane with a one-voxel halo, x neighbours from registers, loads are
// issued kAdjAhead planes ahead into a register ring, and stores that must
// not happen (outside the grid, past the chunk, accumulators of held
// voxels) get an out-of-range buffer offset instead of a branch.  The
// per-voxel arithmetic is adjoint_voxel(), as in the reference kernel.
template <int TY, bool PERF>
__global__ __launch_bounds__(64 * TY) void k_adjoint_tiled(AdjointBuffers a, StepConst K,
                                                           int nx, int ny, int nz, int xc,
                                                           int tiles_z, int tiles_y, int nwg) {
  using namespace tile;
  constexpr int W = AdjSmem<TY>::W;
  constexpr int CELLS = AdjSmem<TY>::CELLS;
  __shared__ AdjSmem<TY> sm;
  stage_pairs(sm.pc, sm.cls, a.tab, 64 * TY);
  const int wg = remap_xcd(blockIdx.x, nwg);
  const int tz = wg % tiles_z;
  const int ty = (wg / tiles_z) % tiles_y;
  const int tx = wg / (tiles_z * tiles_y);
  const int lane = threadIdx.x & 63;
  const int wy = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  const int z = tz * 64 + lane;
  const int y = ty * TY + wy;
  const int x0 = tx * xc;
  const int x1 = min(x0 + xc, nx);
  const bool inside = z < nz && y < ny;
  const int xb = max(x0 - 1, 0);
  const unsigned psz = (unsigned)(ny * nz);
  const unsigned col = inside ? (unsigned)(y * nz + z) : 0u;

  __amdgpu_buffer_rsrc_t r_lam, r_lab, r_th, r_w, r_pf, r_sa, r_fa, r_out;
  {
    const size_t off = (size_t)xb * psz;
    const size_t rest = (size_t)(nx - xb) * psz;
    r_lam = make_rsrc(a.lam_in + off, rest * 4);
    r_lab = make_rsrc(a.lab + off, rest);
    r_th = make_rsrc(a.theta + off, rest * 4);
    r_w = make_rsrc(a.w + off, rest * 4);
    r_pf = make_rsrc(PERF ? a.perf + off : a.w + off, rest * 4);
    r_sa = make_rsrc(a.sacc + off, rest * 4);
    r_fa = make_rsrc(a.facc + off, rest * 4);
    r_out = make_rsrc(a.lam_out + off, rest * 4);
  }

  // halo element of this thread (rows y0-1 / y0+TY, columns z0-1 / z0+64)
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
  const unsigned hoff = hcell < CELLS ? (unsigned)(hy * nz + hz) : col;

  auto load = [&](int x, AdjPlane& q) {
    const int xo = min(x, nx - 1) - xb;  // uniform
    const int xf = min(x, x1 - 1) - xb;  // uniform
    const int so4 = xo * (int)psz * 4, so1 = xo * (int)psz;
    const int sf4 = xf * (int)psz * 4, sf1 = xf * (int)psz;
    q.lam = ld_f32(r_lam, col * 4, so4);
    q.b = ld_u8(r_lab, col, so1);
    q.hl = ld_f32(r_lam, hoff * 4, sf4);
    q.hb = ld_u8(r_lab, hoff, sf1);
    q.th = ld_f32(r_th, col * 4, sf4);
    q.w = ld_f32(r_w, col * 4, sf4);
    q.pf = PERF ? ld_f32(r_pf, col * 4, sf4) : 1.0f;
    q.fa = ld_f32(r_fa, col * 4, sf4);
  };
  // the source accumulator of plane x on the source's support, issued one
  // plane after the plane's other loads (it needs their class byte)
  const bool sacc_all = a.sacc_all;
  auto load_sa = [&](int x, AdjPlane& q) {
    const int sf4 = (min(x, x1 - 1) - xb) * (int)psz * 4;  // uniform
    q.sa = ld_f32(r_sa, (sacc_all || (q.b & kSource)) ? col * 4 : kOob, sf4);
  };

  float lm;  // lambda of the x-1 neighbour (own column)
  unsigned bm;
  {
    const int so = (max(x0 - 1, 0) - xb) * (int)psz;
    lm = ld_f32(r_lam, col * 4, so * 4);
    bm = ld_u8(r_lab, col, so);
  }
  AdjPlane q[kAdjRing];
#pragma unroll
  for (int k = 0; k < kAdjAhead; ++k) load(x0 + k, q[k]);
#pragma unroll
  for (int k = 0; k < kAdjAhead - 1; ++k) load_sa(x0 + k, q[k]);
  const int me = (wy + 1) * W + lane + 1;
  const unsigned st4 = inside ? col * 4 : kOob;

  auto plane = [&](auto S_, int x) {
    constexpr int S = decltype(S_)::value;
    constexpr int BUF = S & 1;
    constexpr int SN = (S + 1) % kAdjRing;
    constexpr int SA = (S + kAdjAhead) % kAdjRing;
    constexpr int SS = (S + kAdjAhead - 1) % kAdjRing;
    load(x + kAdjAhead, q[SA]);
    load_sa(x + kAdjAhead - 1, q[SS]);
    const AdjPlane& P = q[S];
    sm.lam[BUF][me] = P.lam;
    sm.lab[BUF][me] = (uint8_t)P.b;
    sm.lam[BUF][hcell] = P.hl;
    sm.lab[BUF][hcell] = (uint8_t)P.hb;
    __syncthreads();
    const AdjPlane& N = q[SN];
    const float nlam[6] = {lm, N.lam, sm.lam[BUF][me - W], sm.lam[BUF][me + W],
                           sm.lam[BUF][me - 1], sm.lam[BUF][me + 1]};
    const unsigned nlab[6] = {bm, N.b, sm.lab[BUF][me - W], sm.lab[BUF][me + W],
                              sm.lab[BUF][me - 1], sm.lab[BUF][me + 1]};
    const bool valid = x < x1;  // uniform
    float lo, sa = P.sa, fa = P.fa;
    const float2* pc = sm.pc;
    const bool free = adjoint_voxel(
        P.lam, P.th, P.b, P.pf, P.w, nlam, nlab,
        [pc](int ax, unsigned cq, unsigned cp) { return pair_from_pairs(pc, ax, cq, cp); },
        sm.cls, K, lo, sa, fa);
    const int so = (min(x, x1 - 1) - xb) * (int)psz * 4;  // uniform
    const unsigned v = valid ? st4 : kOob;
    st_f32(lo, r_out, v, so);
    st_f32(sa, r_sa, (free && (sacc_all || (P.b & kSource))) ? v : kOob, so);
    st_f32(fa, r_fa, free ? v : kOob, so);
    lm = P.lam;
    bm = P.b;
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  static_assert(kAdjRing == 4, "unrolled for a ring of four planes");
  for (int x = x0; x < x1; x += kAdjRing) {
    plane(I0{}, x);
    plane(I1{}, x + 1);
    plane(I2{}, x + 2);
    plane(I3{}, x + 3);
  }
}

hipError_t launch_adjoint_step(Grid3 g, const AdjointBuffers& a, const StepConst& K,
                               hipStream_t st) {
  dim3 grid((g.nz + 63) / 64, (g.ny + 3) / 4, g.nx), block(64, 4);
  hipLaunchKernelGGL(k_adjoint_step, grid, block, 0, st, a, K, g.nx, g.ny, g.nz);
  return hipGetLastError();
}

bool adjoint_tiled_fits(Grid3 g, int xc) {
  return (double)(xc + kAdjAhead + 2) * g.ny * g.nz * 4.0 < 2147483647.0;
}

hipError_t launch_adjoint_tiled(Grid3 g, int ty, int xc, const AdjointBuffers& a,
                                const StepConst& K, hipStream_t st) {
  if (!adjoint_tiled_fits(g, xc)) return hipErrorInvalidValue;
  const TiledShape s = tiled_shape(g, ty, xc);
  const dim3 grid(s.nwg);
  if (ty == 4) {
    if (a.perf)
      hipLaunchKernelGGL((k_adjoint_tiled<4, true>), grid, dim3(256), 0, st, a, K, g.nx, g.ny,
                         g.nz, xc, s.tiles_z, s.tiles_y, s.nwg);
    else
      hipLaunchKernelGGL((k_adjoint_tiled<4, false>), grid, dim3(256), 0, st, a, K, g.nx, g.ny,
                         g.nz, xc, s.tiles_z, s.tiles_y, s.nwg);
  } else if (ty == 8) {
    if (a.perf)
      hipLaunchKernelGGL((k_adjoint_tiled<8, true>), grid, dim3(512), 0, st, a, K, g.nx, g.ny,
                         g.nz, xc, s.tiles_z, s.tiles_y, s.nwg);
    else
      hipLaunchKernelGGL((k_adjoint_tiled<8, false>), grid, dim3(512), 0, st, a, K, g.nx, g.ny,
                         g.nz, xc, s.tiles_z, s.tiles_y, s.nwg);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Per-tine sums sum_p g_t(p) v_p with v_p = sacc_p dt / (rho c)_p on free
// voxels (grid.y = tine); partial[t][block].
__global__ __launch_bounds__(256) void k_source_dot(const uint8_t* lab, const Chord* chords,
                                                    const int* tine_first, double sigma,
                                                    const float* sacc, const ClassParams* cp,
                                                    double dt, int nx, int ny, int nz,
                                                    double dx, double dy, double dz,
                                                    double* partial) {
  __shared__ double sh[4];
  const int t = blockIdx.y;
  const int c0 = tine_first[t], c1 = tine_first[t + 1];
  const size_t n = (size_t)nx * ny * nz;
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    if (v & kHeld) continue;
    const double sv = (double)sacc[p] * dt / cp->rc[class_of(v)];
    if (sv == 0.0) continue;
    const int k = (int)(p % nz);
    const int j = (int)((p / nz) % ny);
    const int i = (int)(p / ((size_t)nz * ny));
    const double x = (2.0 * i - (nx - 1)) * dx / 2.0;
    const double y = (2.0 * j - (ny - 1)) * dy / 2.0;
    const double z = (2.0 * k - (nz - 1)) * dz / 2.0;
    double g = 0.0;
    for (int c = c0; c < c1; ++c) g += chord_density(chords[c], x, y, z, sigma);
    acc += g * sv;
  }
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)t * gridDim.x + blockIdx.x] = acc;
}

// The same sums from stored per-tine densities u[t][n] (same traversal and
// order, so identical results).
__global__ __launch_bounds__(256) void k_source_dot_fields(const uint8_t* lab, const double* u,
                                                           const float* sacc,
                                                           const ClassParams* cp, double dt,
                                                           size_t n, double* partial) {
  __shared__ double sh[4];
  const int t = blockIdx.y;
  const double* ut = u + (size_t)t * n;
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    if (v & kHeld) continue;
    const double sv = (double)sacc[p] * dt / cp->rc[class_of(v)];
    if (sv == 0.0) continue;
    acc += ut[p] * sv;
  }
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)t * gridDim.x + blockIdx.x] = acc;
}

hipError_t launch_source_dot_fields(Grid3 g, const uint8_t* lab, const double* u, int n_tines,
                                    const float* sacc, const ClassParams* cp_dev, double dt,
                                    double* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_source_dot_fields, dim3(nblk, n_tines), dim3(256), 0, st, lab, u, sacc,
                     cp_dev, dt, g.n(), partial);
  return hipGetLastError();
}

hipError_t launch_source_dot(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                             const Chord* chords, const int* tine_first, int n_tines,
                             double sigma, const float* sacc, const ClassParams* cp_dev,
                             double dt, double* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_source_dot, dim3(nblk, n_tines), dim3(256), 0, st, lab, chords,
                     tine_first, sigma, sacc, cp_dev, dt, g.nx, g.ny, g.nz, dx, dy, dz, partial);
  return hipGetLastError();
}

}  // namespace rfa
