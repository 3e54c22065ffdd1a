// rfa_kernels.hip -- setup, reference-step and reduction kernels (gfx950).
//
// All reductions are deterministic: fixed work assignment, fixed-order
// tree sums, no floating-point atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rfa_kernels.h"

namespace rfa {

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

__device__ __forceinline__ size_t vidx(int i, int j, int k, int ny, int nz) {
  return ((size_t)i * ny + j) * nz + k;
}

// Block sum of a double over kRedThreads threads; result valid on thread 0.
__device__ double block_sum_d(double v, double* sh) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

__device__ double wave_min_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ double wave_max_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ double block_min_d(double v, double* sh) {
  v = wave_min_d(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = INFINITY;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) r = fmin(r, sh[i]);
  __syncthreads();
  return r;
}
__device__ double block_max_d(double v, double* sh) {
  v = wave_max_d(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = -INFINITY;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;
}

}  // namespace

// ===========================================================================
// Reference step: one thread per voxel, block 64 (z) x 4 (y), grid over
// (z tiles, y tiles, x).  Neighbours are read straight from global memory.
// ===========================================================================
template <bool PERF>
__global__ __launch_bounds__(256) void k_step_naive(StepBuffers b, StepConst K, int nx, int ny,
                                                    int nz) {
  __shared__ float2 cf[3 * kMaxClasses * kMaxClasses];
  __shared__ float4 cls[kMaxClasses];
  __shared__ float red[3][4];
  const int tid = threadIdx.y * 64 + threadIdx.x;
  {
    const float2* src = &b.tab->cf[0][0];
    for (int t = tid; t < 3 * kMaxClasses * kMaxClasses; t += 256) cf[t] = src[t];
    if (tid < kMaxClasses) cls[tid] = b.tab->cls[tid];
  }
  __syncthreads();
  const int k = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int i = blockIdx.z;
  Partial acc{0.0f, 0.0f, 0u};
  if (k < nz && j < ny) {
    const size_t p = vidx(i, j, k, ny, nz);
    const unsigned lab = b.lab[p];
    const float hi = b.hi_in[p], lo = b.lo_in[p];
    float om = b.omega[p];
    const float s = b.src[p];
    const float pf = PERF ? b.perf[p] : 1.0f;
    // Held voxels (possibly on the outer layer) read no neighbours.
    const bool held = (lab & kHeld) != 0u;
    const size_t sx = (size_t)ny * nz, sy = (size_t)nz;
    const size_t pxm = held ? p : p - sx, pxp = held ? p : p + sx;
    const size_t pym = held ? p : p - sy, pyp = held ? p : p + sy;
    const size_t pzm = held ? p : p - 1, pzp = held ? p : p + 1;
    float nh, nl;
    unsigned nlab;
    voxel_step(hi, lo, lab,
               b.hi_in[pxm], b.lo_in[pxm], b.lab[pxm], b.hi_in[pxp], b.lo_in[pxp], b.lab[pxp],
               b.hi_in[pym], b.lo_in[pym], b.lab[pym], b.hi_in[pyp], b.lo_in[pyp], b.lab[pyp],
               b.hi_in[pzm], b.lo_in[pzm], b.lab[pzm], b.hi_in[pzp], b.lo_in[pzp], b.lab[pzp],
               s, pf, om, cf, cls, K, nh, nl, nlab, acc, PERF);
    b.hi_out[p] = nh;
    b.lo_out[p] = nl;
    b.omega[p] = om;
    if (nlab != lab) b.lab[p] = (uint8_t)nlab;
  }
  if (b.partials) {
    const float pe = wave_sum(acc.perf);
    const float bn = wave_sum(acc.bnd);
    const unsigned mo = wave_sum_u(acc.mono);
    if (threadIdx.x == 0) {
      red[0][threadIdx.y] = pe;
      red[1][threadIdx.y] = bn;
      red[2][threadIdx.y] = (float)mo;
    }
    __syncthreads();
    if (tid == 0) {
      const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
      float* out = b.partials + wg * 3;
      out[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      out[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      out[2] = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    }
  }
}

int naive_wg_count(Grid3 g) { return ((g.nz + 63) / 64) * ((g.ny + 3) / 4) * g.nx; }

hipError_t launch_step_naive(Grid3 g, const StepBuffers& b, const StepConst& K,
                             hipStream_t st) {
  dim3 grid((g.nz + 63) / 64, (g.ny + 3) / 4, g.nx), block(64, 4);
  if (b.perf)
    hipLaunchKernelGGL(k_step_naive<true>, grid, block, 0, st, b, K, g.nx, g.ny, g.nz);
  else
    hipLaunchKernelGGL(k_step_naive<false>, grid, block, 0, st, b, K, g.nx, g.ny, g.nz);
  return hipGetLastError();
}

// ===========================================================================
// Diagnostic partial sums: one block, slots in order, work-groups strided.
// ===========================================================================
// One block of 1024 threads: each thread sums a fixed strided subset of the
// flat [n_slots * nwg] entries of each component, then a fixed tree.
__global__ __launch_bounds__(1024) void k_reduce_partials(const float* partials, int n_slots,
                                                          int nwg, double* acc) {
  __shared__ double sh[3][16];
  const size_t n = (size_t)n_slots * nwg;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  // Each thread sums elements threadIdx.x + 1024 k in increasing k; the
  // loads of eight consecutive k are issued before their adds, so a
  // launch costs a few memory latencies instead of one per element.
  constexpr int kU = 8;
  size_t e = threadIdx.x;
  for (; e + (kU - 1) * 1024 < n; e += kU * 1024) {
    float q[kU][3];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const float* p = partials + (e + (size_t)k * 1024) * 3;
      q[k][0] = p[0];
      q[k][1] = p[1];
      q[k][2] = p[2];
    }
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      v0 += (double)q[k][0];
      v1 += (double)q[k][1];
      v2 += (double)q[k][2];
    }
  }
  for (; e < n; e += 1024) {
    const float* p = partials + e * 3;
    v0 += (double)p[0];
    v1 += (double)p[1];
    v2 += (double)p[2];
  }
  v0 = wave_sum_d(v0);
  v1 = wave_sum_d(v1);
  v2 = wave_sum_d(v2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = v0;
    sh[1][w] = v1;
    sh[2][w] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += sh[threadIdx.x][i];
    acc[threadIdx.x] += t;
  }
}

hipError_t launch_reduce_partials(const float* partials, int n_slots, int nwg, double* acc,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, st, partials, n_slots, nwg,
                     acc);
  return hipGetLastError();
}

// Batched diagnostics in two fixed-order passes: block (i, s) sums the
// partials of instance i's items in step slot s into slot_acc[i][s][.]
// (its threads stride over the items, then wave and work-group sums), and
// block i of the second pass adds its n_slots slot sums (one lane each, a
// wave sum) to acc[3 i .. 3 i + 2].  Every instance and slot gets its own
// work-group, so the pass is as wide as the batch.
__global__ __launch_bounds__(256) void k_reduce_batch_slots(const float* partials, int n_items,
                                                            const int* first, int inst0,
                                                            int slot_stride, double* slot_acc) {
  __shared__ double sh[3][4];
  const int i = inst0 + blockIdx.x, s = blockIdx.y;
  const int a = first[2 * i], cnt = first[2 * i + 1] - first[2 * i];
  const float* p = partials + ((size_t)s * n_items + a) * 3;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int k = threadIdx.x; k < cnt; k += 256) {
    v0 += (double)p[3 * k];
    v1 += (double)p[3 * k + 1];
    v2 += (double)p[3 * k + 2];
  }
  v0 = wave_sum_d(v0);
  v1 = wave_sum_d(v1);
  v2 = wave_sum_d(v2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = v0;
    sh[1][w] = v1;
    sh[2][w] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3)
    slot_acc[((size_t)i * slot_stride + s) * 3 + threadIdx.x] =
        (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
}

__global__ __launch_bounds__(64) void k_reduce_batch_final(const double* slot_acc, int n_slots,
                                                           int inst0, int slot_stride,
                                                           double* acc) {
  const int i = inst0 + blockIdx.x, s = threadIdx.x;
  const double* q = slot_acc + ((size_t)i * slot_stride + s) * 3;
  const bool on = s < n_slots;
  const double v0 = wave_sum_d(on ? q[0] : 0.0);
  const double v1 = wave_sum_d(on ? q[1] : 0.0);
  const double v2 = wave_sum_d(on ? q[2] : 0.0);
  if (s == 0) {
    acc[3 * i] += v0;
    acc[3 * i + 1] += v1;
    acc[3 * i + 2] += v2;
  }
}

hipError_t launch_reduce_batch(const float* partials, int n_slots, int n_items,
                               const int* first, int inst0, int n_inst, double* slot_acc,
                               int slot_stride, double* acc, hipStream_t st) {
  if (n_inst <= 0 || n_slots <= 0) return hipSuccess;
  if (n_slots > slot_stride || slot_stride > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_batch_slots, dim3(n_inst, n_slots), dim3(256), 0, st, partials,
                     n_items, first, inst0, slot_stride, slot_acc);
  hipLaunchKernelGGL(k_reduce_batch_final, dim3(n_inst), dim3(64), 0, st, slot_acc, n_slots,
                     inst0, slot_stride, acc);
  return hipGetLastError();
}

// ===========================================================================
// Setup kernels
// ===========================================================================
__global__ void k_build_labels(const uint8_t* user, uint8_t* lab, const ClassParams* cp,
                               unsigned* bad, int nx, int ny, int nz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned u = user[p];
    const int k = (int)(p % nz);
    const int j = (int)((p / nz) % ny);
    const int i = (int)(p / ((size_t)nz * ny));
    if ((int)u >= cp->n) {
      atomicAdd(bad, 1u);
      lab[p] = 0;
      continue;
    }
    unsigned v = u << kClassShift;
    if (cp->tissue[u]) v |= kTissue;
    const bool outer = i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1;
    if (cp->fixed[u] || outer) v |= kHeld;
    lab[p] = (uint8_t)v;
  }
}

hipError_t launch_build_labels(Grid3 g, const uint8_t* user, uint8_t* lab,
                               const ClassParams* cp_dev, unsigned* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_build_labels, dim3(2048), dim3(256), 0, st, user, lab, cp_dev, bad, g.nx,
                     g.ny, g.nz);
  return hipGetLastError();
}

__device__ __forceinline__ void split_theta(double th, float& hi, float& lo) {
  hi = (float)th;
  lo = (float)(th - (double)hi);
}

__device__ __forceinline__ bool reaches(float hi, float lo, float thr) {
  return hi > thr || (hi == thr && lo >= 0.0f);
}

__global__ void k_reset_state(uint8_t* lab, float* hi, float* lo, float* om, const ClassParams* cp,
                              float thr, size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    unsigned v = lab[p] & ~kLatch;
    const unsigned c = class_of(v);
    const double th = cp->fixed[c] ? cp->t_fixed[c] - 37.0 : 0.0;
    float h, l;
    split_theta(th, h, l);
    hi[p] = h;
    lo[p] = l;
    om[p] = 0.0f;
    if ((v & kTissue) && reaches(h, l, thr)) v |= kLatch;
    lab[p] = (uint8_t)v;
  }
}

hipError_t launch_reset_state(Grid3 g, uint8_t* lab, float* hi, float* lo, float* om,
                              const ClassParams* cp_dev, float thr, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_state, dim3(2048), dim3(256), 0, st, lab, hi, lo, om, cp_dev, thr,
                     g.n());
  return hipGetLastError();
}

// ---- stability bound -------------------------------------------------------
__device__ __forceinline__ double face_k(const ClassParams* cp, unsigned a, unsigned b) {
  const double ka = cp->k[a], kb = cp->k[b];
  return (ka + kb) == 0.0 ? 0.0 : 2.0 * ka * kb / (ka + kb);
}

__global__ __launch_bounds__(kRedThreads) void k_dt_bound(const uint8_t* lab, const float* perf,
                                                          const ClassParams* cp, double ix,
                                                          double iy, double iz, int nx, int ny,
                                                          int nz, double* partial) {
  __shared__ double sh[kRedThreads / 64];
  const size_t n = (size_t)nx * ny * nz;
  double best = INFINITY;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    if (v & kHeld) continue;
    const unsigned c = class_of(v);
    const size_t sx = (size_t)ny * nz, sy = nz;
    double s = cp->h[c] * (perf ? (double)perf[p] : 1.0);
    s += (face_k(cp, c, class_of(lab[p - sx])) + face_k(cp, c, class_of(lab[p + sx]))) * ix;
    s += (face_k(cp, c, class_of(lab[p - sy])) + face_k(cp, c, class_of(lab[p + sy]))) * iy;
    s += (face_k(cp, c, class_of(lab[p - 1])) + face_k(cp, c, class_of(lab[p + 1]))) * iz;
    const double d = s > 0.0 ? cp->rc[c] / s : INFINITY;
    best = fmin(best, d);
  }
  best = block_min_d(best, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = best;
}

__global__ __launch_bounds__(kRedThreads) void k_min_partials(const double* partial, int n,
                                                              double* out) {
  __shared__ double sh[kRedThreads / 64];
  double v = INFINITY;
  for (int i = threadIdx.x; i < n; i += kRedThreads) v = fmin(v, partial[i]);
  v = block_min_d(v, sh);
  if (threadIdx.x == 0) *out = v;
}

hipError_t launch_dt_bound(Grid3 g, const uint8_t* lab, const float* perf,
                           const ClassParams* cp_dev, double inv_d2x, double inv_d2y,
                           double inv_d2z, double* partial, int* nblk_out, double* result,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_dt_bound, dim3(kRedBlocks), dim3(kRedThreads), 0, st, lab, perf, cp_dev,
                     inv_d2x, inv_d2y, inv_d2z, g.nx, g.ny, g.nz, partial);
  hipLaunchKernelGGL(k_min_partials, dim3(1), dim3(kRedThreads), 0, st, partial, kRedBlocks,
                     result);
  if (nblk_out) *nblk_out = kRedBlocks;
  return hipGetLastError();
}

// ---- RF source (FP64) --------------------------------------------------------
__device__ __forceinline__ double tine_density(const Chord* chords, int first, int last, double x,
                                               double y, double z, double sigma) {
  double g = 0.0;
  for (int c = first; c < last; ++c) g += chord_density(chords[c], x, y, z, sigma);
  return g;
}

// grid.x: voxel blocks (grid-stride), grid.y: tine.  partial[tine][block].
__global__ __launch_bounds__(kRedThreads) void k_source_sums(const uint8_t* lab,
                                                             const Chord* chords,
                                                             const int* tine_first, double sigma,
                                                             int nx, int ny, int nz, double dx,
                                                             double dy, double dz,
                                                             double* partial) {
  __shared__ double sh[kRedThreads / 64];
  const int t = blockIdx.y;
  const int c0 = tine_first[t], c1 = tine_first[t + 1];
  const size_t n = (size_t)nx * ny * nz;
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    if (lab[p] & kHeld) continue;
    const int k = (int)(p % nz);
    const int j = (int)((p / nz) % ny);
    const int i = (int)(p / ((size_t)nz * ny));
    const double x = (2.0 * i - (nx - 1)) * dx / 2.0;
    const double y = (2.0 * j - (ny - 1)) * dy / 2.0;
    const double z = (2.0 * k - (nz - 1)) * dz / 2.0;
    acc += tine_density(chords, c0, c1, x, y, z, sigma);
  }
  acc = block_sum_d(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)t * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(kRedThreads) void k_sum_rows(const double* partial, int ncol,
                                                          double scale, double* out) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0.0;
  const double* row = partial + (size_t)blockIdx.x * ncol;
  for (int i = threadIdx.x; i < ncol; i += kRedThreads) v += row[i];
  v = block_sum_d(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v * scale;
}

hipError_t launch_source_sums(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                              const Chord* chords, const int* tine_first, int n_tines,
                              double sigma, double* partial, int* nblk_out, double* sums,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_source_sums, dim3(kRedBlocks, n_tines), dim3(kRedThreads), 0, st, lab,
                     chords, tine_first, sigma, g.nx, g.ny, g.nz, dx, dy, dz, partial);
  hipLaunchKernelGGL(k_sum_rows, dim3(n_tines), dim3(kRedThreads), 0, st, partial, kRedBlocks,
                     dx * dy * dz, sums);
  if (nblk_out) *nblk_out = kRedBlocks;
  return hipGetLastError();
}

// u[t][p] = g_t(p), the unnormalised density of tine t, on free voxels and
// 0 on held ones (kept so that new tine powers only recombine the fields).
__global__ void k_source_fields(const uint8_t* lab, const Chord* chords, const int* tine_first,
                                int n_tines, double sigma, double* u, int nx, int ny, int nz,
                                double dx, double dy, double dz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    if (lab[p] & kHeld) {
      for (int t = 0; t < n_tines; ++t) u[(size_t)t * n + p] = 0.0;
      continue;
    }
    const int k = (int)(p % nz);
    const int j = (int)((p / nz) % ny);
    const int i = (int)(p / ((size_t)nz * ny));
    const double x = (2.0 * i - (nx - 1)) * dx / 2.0;
    const double y = (2.0 * j - (ny - 1)) * dy / 2.0;
    const double z = (2.0 * k - (nz - 1)) * dz / 2.0;
    for (int t = 0; t < n_tines; ++t)
      u[(size_t)t * n + p] = tine_density(chords, tine_first[t], tine_first[t + 1], x, y, z, sigma);
  }
}

// Per-tine integrals from stored fields: the traversal and summation order
// of k_source_sums, so the results are identical.
__global__ __launch_bounds__(kRedThreads) void k_field_sums(const uint8_t* lab, const double* u,
                                                            size_t n, double* partial) {
  __shared__ double sh[kRedThreads / 64];
  const int t = blockIdx.y;
  const double* ut = u + (size_t)t * n;
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    if (lab[p] & kHeld) continue;
    acc += ut[p];
  }
  acc = block_sum_d(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)t * gridDim.x + blockIdx.x] = acc;
}

// q[p] = sum_t scale[t] u_t(p) on free voxels, in the order of k_source_write.
__global__ void k_source_combine(const uint8_t* lab, const double* u, int n_tines,
                                 const double* scale, double* q, size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (!(lab[p] & kHeld))
      for (int t = 0; t < n_tines; ++t) v += scale[t] * u[(size_t)t * n + p];
    q[p] = v;
  }
}

hipError_t launch_source_fields(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                                const Chord* chords, const int* tine_first, int n_tines,
                                double sigma, double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_source_fields, dim3(4096), dim3(256), 0, st, lab, chords, tine_first,
                     n_tines, sigma, u, g.nx, g.ny, g.nz, dx, dy, dz);
  return hipGetLastError();
}

hipError_t launch_field_sums(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                             const double* u, int n_tines, double* partial, double* sums,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_field_sums, dim3(kRedBlocks, n_tines), dim3(kRedThreads), 0, st, lab, u,
                     g.n(), partial);
  hipLaunchKernelGGL(k_sum_rows, dim3(n_tines), dim3(kRedThreads), 0, st, partial, kRedBlocks,
                     dx * dy * dz, sums);
  return hipGetLastError();
}

hipError_t launch_source_combine(Grid3 g, const uint8_t* lab, const double* u, int n_tines,
                                 const double* scale, double* q, hipStream_t st) {
  hipLaunchKernelGGL(k_source_combine, dim3(4096), dim3(256), 0, st, lab, u, n_tines, scale, q,
                     g.n());
  return hipGetLastError();
}

// q[p] = sum_t scale[t] * g_t(p) on free voxels (scale = power / integral).
__global__ void k_source_write(const uint8_t* lab, const Chord* chords, const int* tine_first,
                               int n_tines, double sigma, const double* scale, double* q, int nx,
                               int ny, int nz, double dx, double dy, double dz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (!(lab[p] & kHeld)) {
      const int k = (int)(p % nz);
      const int j = (int)((p / nz) % ny);
      const int i = (int)(p / ((size_t)nz * ny));
      const double x = (2.0 * i - (nx - 1)) * dx / 2.0;
      const double y = (2.0 * j - (ny - 1)) * dy / 2.0;
      const double z = (2.0 * k - (nz - 1)) * dz / 2.0;
      for (int t = 0; t < n_tines; ++t)
        v += scale[t] * tine_density(chords, tine_first[t], tine_first[t + 1], x, y, z, sigma);
    }
    q[p] = v;
  }
}

hipError_t launch_source_write(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                               const Chord* chords, const int* tine_first, int n_tines,
                               double sigma, const double* scale, double* q,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_source_write, dim3(4096), dim3(256), 0, st, lab, chords, tine_first,
                     n_tines, sigma, scale, q, g.nx, g.ny, g.nz, dx, dy, dz);
  return hipGetLastError();
}

// s = dt q / (rho c) (0 on held voxels), and the label's source flag set
// exactly where s != 0: the step kernels read s only on flagged voxels (the
// RF source beyond its Gaussian cut-off is exactly zero, so most of the grid
// needs no source bytes).
__global__ void k_source_increment(uint8_t* lab, const double* q, const ClassParams* cp,
                                   double dt, float* s, size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    const float sv = (v & kHeld) ? 0.0f : (float)(dt * q[p] / cp->rc[class_of(v)]);
    s[p] = sv;
    const unsigned nv = sv != 0.0f ? (v | kSource) : (v & ~kSource);
    if (nv != v) lab[p] = (uint8_t)nv;
  }
}

// Voxels whose label carries the flag bit(s) `flag`, added into *count.
__global__ __launch_bounds__(256) void k_count_flag(const uint8_t* lab, unsigned flag, size_t n,
                                                    unsigned long long* count) {
  unsigned c = 0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x)
    c += (lab[p] & flag) ? 1u : 0u;
  c = wave_sum_u(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

hipError_t launch_count_flag(Grid3 g, const uint8_t* lab, unsigned flag,
                             unsigned long long* count, hipStream_t st) {
  hipLaunchKernelGGL(k_count_flag, dim3(1024), dim3(256), 0, st, lab, flag, g.n(), count);
  return hipGetLastError();
}

hipError_t launch_source_increment(Grid3 g, uint8_t* lab, const double* q,
                                   const ClassParams* cp_dev, double dt, float* s,
                                   hipStream_t st) {
  hipLaunchKernelGGL(k_source_increment, dim3(2048), dim3(256), 0, st, lab, q, cp_dev, dt, s,
                     g.n());
  return hipGetLastError();
}

// ---- state reductions ------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_state_reduce(const uint8_t* lab, const float* hi,
                                                              const float* lo,
                                                              const ClassParams* cp, double vol,
                                                              size_t n, double* partial) {
  __shared__ double sh[kRedThreads / 64];
  double e = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const double th = (double)hi[p] + (double)lo[p];
    if (!isfinite(th)) {
      bad += 1.0;
      continue;
    }
    const unsigned v = lab[p];
    if (!(v & kHeld)) e += cp->rc[class_of(v)] * th;
    mn = fmin(mn, th);
    mx = fmax(mx, th);
  }
  e = block_sum_d(e, sh);
  mn = block_min_d(mn, sh);
  mx = block_max_d(mx, sh);
  bad = block_sum_d(bad, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 4 + 0] = e * vol;
    partial[blockIdx.x * 4 + 1] = mn;
    partial[blockIdx.x * 4 + 2] = mx;
    partial[blockIdx.x * 4 + 3] = bad;
  }
}

__global__ __launch_bounds__(kRedThreads) void k_state_finish(const double* partial, int nb,
                                                              double* out4) {
  __shared__ double sh[kRedThreads / 64];
  double e = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) {
    e += partial[b * 4 + 0];
    mn = fmin(mn, partial[b * 4 + 1]);
    mx = fmax(mx, partial[b * 4 + 2]);
    bad += partial[b * 4 + 3];
  }
  e = block_sum_d(e, sh);
  mn = block_min_d(mn, sh);
  mx = block_max_d(mx, sh);
  bad = block_sum_d(bad, sh);
  if (threadIdx.x == 0) {
    out4[0] = e;
    out4[1] = mn + 37.0;
    out4[2] = mx + 37.0;
    out4[3] = bad;
  }
}

hipError_t launch_state_reduce(Grid3 g, const uint8_t* lab, const float* hi, const float* lo,
                               const ClassParams* cp_dev, double vol, double* partial,
                               double* out4, hipStream_t st) {
  hipLaunchKernelGGL(k_state_reduce, dim3(kRedBlocks), dim3(kRedThreads), 0, st, lab, hi, lo,
                     cp_dev, vol, g.n(), partial);
  hipLaunchKernelGGL(k_state_finish, dim3(1), dim3(kRedThreads), 0, st, partial, kRedBlocks,
                     out4);
  return hipGetLastError();
}

// ---- damage outputs ----------------------------------------------------------
__global__ __launch_bounds__(256) void k_damage(const uint8_t* lab, const float* om, uint8_t* mask,
                                                unsigned long long* counts, size_t n) {
  __shared__ unsigned cnt[kMaxClasses][2];
  if (threadIdx.x < 2 * kMaxClasses) (&cnt[0][0])[threadIdx.x] = 0u;
  __syncthreads();
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    const bool tis = (v & kTissue) != 0u;
    const unsigned b0 = (tis && (v & kLatch)) ? 1u : 0u;
    const unsigned b1 = (tis && om[p] >= 1.0f) ? 2u : 0u;
    if (mask) mask[p] = (uint8_t)(b0 | b1);
    if (b0) atomicAdd(&cnt[class_of(v)][0], 1u);
    if (b1) atomicAdd(&cnt[class_of(v)][1], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMaxClasses) {
    const unsigned c = (&cnt[0][0])[threadIdx.x];
    if (c) atomicAdd(&counts[threadIdx.x], (unsigned long long)c);
  }
}

hipError_t launch_damage(Grid3 g, const uint8_t* lab, const float* om, uint8_t* mask,
                         unsigned long long* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_damage, dim3(2048), dim3(256), 0, st, lab, om, mask, counts, g.n());
  return hipGetLastError();
}

// Counters to zero with a kernel rather than a memset, so that a caller may
// capture the launch in a graph.
__global__ __launch_bounds__(64) void k_zero_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += 64) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

// Streaming probe of the step kernels' byte mix without the stencil: per
// voxel read theta hi and lo, the class byte and Omega, write theta hi, lo
// and Omega (25 B), four voxels per thread as 16-byte accesses.  The
// arithmetic only keeps every load live.
__global__ __launch_bounds__(256) void k_stream_mix(const float4* __restrict__ hi,
                                                    const float4* __restrict__ lo,
                                                    const unsigned* __restrict__ lab,
                                                    const float4* __restrict__ om,
                                                    float4* __restrict__ hi_o,
                                                    float4* __restrict__ lo_o,
                                                    float4* __restrict__ om_o, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float s = (float)(lab[i] & 0xffu) * 1e-30f;
    const float4 h = hi[i], l = lo[i], o = om[i];
    hi_o[i] = make_float4(h.x + s, h.y + s, h.z + s, h.w + s);
    lo_o[i] = make_float4(l.x - s, l.y - s, l.z - s, l.w - s);
    om_o[i] = make_float4(o.x + s, o.y + s, o.z + s, o.w + s);
  }
}

hipError_t launch_stream_mix(const float4* const (&in)[3], const unsigned* lab,
                             float4* const (&out)[3], size_t n4, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_mix, dim3((unsigned)blocks), dim3(256), 0, st, in[0], in[1], lab,
                     in[2], out[0], out[1], out[2], n4);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ a,
                                              float4* __restrict__ b, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Streaming copy with non-temporal hints, four 16-byte vectors per thread
// per pass.
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_nt(const float4* __restrict__ a4,
                                                 float4* __restrict__ b4, size_t n4) {
  const v4f* a = reinterpret_cast<const v4f*>(a4);
  v4f* b = reinterpret_cast<v4f*>(b4);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const v4f v0 = __builtin_nontemporal_load(a + i);
    const v4f v1 = __builtin_nontemporal_load(a + i + stride);
    const v4f v2 = __builtin_nontemporal_load(a + i + 2 * stride);
    const v4f v3 = __builtin_nontemporal_load(a + i + 3 * stride);
    __builtin_nontemporal_store(v0, b + i);
    __builtin_nontemporal_store(v1, b + i + stride);
    __builtin_nontemporal_store(v2, b + i + 2 * stride);
    __builtin_nontemporal_store(v3, b + i + 3 * stride);
  }
  for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

hipError_t launch_copy(const float4* a, float4* b, size_t n4, int max_blocks, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n4 + 255) / 256, (size_t)max_blocks);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, a, b, n4);
  return hipGetLastError();
}

hipError_t launch_copy_nt(const float4* a, float4* b, size_t n4, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n4 + 1023) / 1024, 256 * 8);
  hipLaunchKernelGGL(k_copy_nt, dim3((unsigned)blocks), dim3(256), 0, st, a, b, n4);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_free_counts(const uint8_t* lab,
                                                     unsigned long long* counts, size_t n) {
  __shared__ unsigned cnt[kMaxClasses];
  if (threadIdx.x < kMaxClasses) cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    const unsigned v = lab[p];
    if (!(v & kHeld)) atomicAdd(&cnt[class_of(v)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kMaxClasses && cnt[threadIdx.x])
    atomicAdd(&counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

hipError_t launch_free_counts(Grid3 g, const uint8_t* lab, unsigned long long* counts,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_free_counts, dim3(2048), dim3(256), 0, st, lab, counts, g.n());
  return hipGetLastError();
}

__global__ void k_temperature_out(const float* hi, const float* lo, double* t, size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x)
    t[p] = 37.0 + ((double)hi[p] + (double)lo[p]);
}

hipError_t launch_temperature_out(Grid3 g, const float* hi, const float* lo, double* t,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_temperature_out, dim3(2048), dim3(256), 0, st, hi, lo, t, g.n());
  return hipGetLastError();
}

__global__ void k_temperature_in(const double* t, float* hi, float* lo, uint8_t* lab, float thr,
                                 size_t n) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    float h, l;
    split_theta(t[p] - 37.0, h, l);
    hi[p] = h;
    lo[p] = l;
    const unsigned v = lab[p];
    if ((v & kTissue) && reaches(h, l, thr)) lab[p] = (uint8_t)(v | kLatch);
  }
}

hipError_t launch_temperature_in(Grid3 g, const double* t, float* hi, float* lo, uint8_t* lab,
                                 float thr, hipStream_t st) {
  hipLaunchKernelGGL(k_temperature_in, dim3(2048), dim3(256), 0, st, t, hi, lo, lab, thr, g.n());
  return hipGetLastError();
}

}  // namespace rfa
