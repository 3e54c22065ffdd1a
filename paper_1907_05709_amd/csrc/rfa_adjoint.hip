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

#include "rfa_adjoint.h"

namespace rfa {

namespace {

__device__ __forceinline__ float coef(const Tables* T, int axis, unsigned a, unsigned b) {
  const float2 c = T->cf[axis][(a & kClassMask) * kMaxClasses + (b & kClassMask)];
  return c.x + c.y;
}

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

// gctrl[j] = sum_p gf_p f_p B_j(x_p): one block per control point gathers
// over the voxels of its support box (fixed order, deterministic).
__global__ __launch_bounds__(256) void k_bspline_grad(const float* gf, const float* f, int m,
                                                      int nx, int ny, int nz,
                                                      const int* vfirst_x,
                                                      const int* vfirst_y,
                                                      const int* vfirst_z, double* gctrl) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  const int ja = j / (m * m), jb = (j / m) % m, jc = j % m;
  // voxels whose span s satisfies s <= j <= s + 3, i.e. s in [j-3, j]
  auto range = [&](int jj, const int* vf, int& lo, int& hi) {
    const int s0 = jj - 3 < 0 ? 0 : jj - 3;
    const int s1 = jj > m - 4 ? m - 4 : jj;
    lo = vf[s0];
    hi = vf[s1 + 1];
  };
  int x0, x1, y0, y1, z0, z1;
  range(ja, vfirst_x, x0, x1);
  range(jb, vfirst_y, y0, y1);
  range(jc, vfirst_z, z0, z1);
  const int ex = x1 - x0, ey = y1 - y0, ez = z1 - z0;
  const long long cnt = (long long)ex * ey * ez;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < cnt; e += 256) {
    const int k = z0 + (int)(e % ez), jy = y0 + (int)((e / ez) % ey), i = x0 + (int)(e / ((long long)ez * ey));
    int si, sj, sk;
    double ti, tj, tk, bi[4], bj[4], bk[4];
    span_of(i, nx, m, si, ti);
    span_of(jy, ny, m, sj, tj);
    span_of(k, nz, m, sk, tk);
    const int a = ja - si, b = jb - sj, c = jc - sk;
    if (a < 0 || a > 3 || b < 0 || b > 3 || c < 0 || c > 3) continue;
    basis(ti, bi);
    basis(tj, bj);
    basis(tk, bk);
    const size_t p = ((size_t)i * ny + jy) * nz + k;
    acc += (double)gf[p] * (double)f[p] * bi[a] * bj[b] * bk[c];
  }
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) gctrl[j] = acc;
}

hipError_t launch_bspline_grad(Grid3 g, const float* gf, const float* f, int m,
                               const int* vfirst_x, const int* vfirst_y, const int* vfirst_z,
                               double* gctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_bspline_grad, dim3(m * m * m), dim3(256), 0, st, gf, f, m, g.nx, g.ny,
                     g.nz, vfirst_x, vfirst_y, vfirst_z, gctrl);
  return hipGetLastError();
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

// One adjoint step: lam_out = M^T lam_in + w' dt rate'(theta^n); accumulates
// dL/ds (sacc += lam_in) and dL/df (facc += lam_in (-B theta^n)) on free voxels.
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
  const Tables* T = a.tab;
  const float lam = a.lam_in[q];
  const float th = a.theta[q];
  const float pf = a.perf ? a.perf[q] : 1.0f;
  const float4 cl = T->cls[lq & kClassMask];
  const float B = (cl.x + cl.y) * pf;
  const size_t nb[6] = {q - sx, q + sx, q - sy, q + sy, q - 1, q + 1};
  float diag = 1.0f - B;
  float off = 0.0f;
  for (int f = 0; f < 6; ++f) {
    const unsigned lp = a.lab[nb[f]];
    diag -= coef(T, f >> 1, lq, lp);                  // q's own row
    if (!(lp & kHeld)) off = __builtin_fmaf(coef(T, f >> 1, lp, lq), a.lam_in[nb[f]], off);
  }
  // damage-rate derivative at theta^n (zero where the exponent is capped)
  float dr = 0.0f;
  if (lq & kTissue) {
    const float tk = K.tak + th;
    const float x = K.c2 * th / tk;
    if (x < K.clamp2) {
      const float rate = K.dtka * __builtin_amdgcn_exp2f(x);
      dr = rate * (K.c2 * 0.69314718f) * K.tak / (tk * tk);
    }
  }
  a.lam_out[q] = __builtin_fmaf(diag, lam, off) + a.w[q] * dr;
  a.sacc[q] += lam;
  a.facc[q] = __builtin_fmaf(-cl.x - cl.y, th * lam, a.facc[q]);
}

hipError_t launch_adjoint_step(Grid3 g, const AdjointBuffers& a, const StepConst& K,
                               hipStream_t st) {
  dim3 grid((g.nz + 63) / 64, (g.ny + 3) / 4, g.nx), block(64, 4);
  hipLaunchKernelGGL(k_adjoint_step, grid, block, 0, st, a, K, g.nx, g.ny, g.nz);
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
    const double sv = (double)sacc[p] * dt / cp->rc[v & kClassMask];
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

hipError_t launch_source_dot(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                             const Chord* chords, const int* tine_first, int n_tines,
                             double sigma, const float* sacc, const ClassParams* cp_dev,
                             double dt, double* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_source_dot, dim3(nblk, n_tines), dim3(256), 0, st, lab, chords,
                     tine_first, sigma, sacc, cp_dev, dt, g.nx, g.ny, g.nz, dx, dy, dz, partial);
  return hipGetLastError();
}

}  // namespace rfa
