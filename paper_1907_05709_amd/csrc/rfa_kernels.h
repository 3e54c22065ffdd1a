// rfa_kernels.h -- host-side launchers of the device kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfa_device.h"

namespace rfa {

struct Grid3 {
  int nx, ny, nz;
  size_t n() const { return (size_t)nx * ny * nz; }
};

// Class parameters in FP64 for setup kernels.
struct ClassParams {
  double k[kMaxClasses];
  double rc[kMaxClasses];   // rho c
  double h[kMaxClasses];
  double t_fixed[kMaxClasses];
  int fixed[kMaxClasses];
  int tissue[kMaxClasses];
  int n;
};

// One chord of a needle tine.
struct Chord {
  double mx, my, mz;   // midpoint, m
  double ux, uy, uz;   // unit direction
  double half;         // half length, m
  int tine;
  int pad;
};

// Density of one chord (uniform unit line density smeared by an isotropic
// Gaussian of standard deviation sigma) at point (x, y, z), 1/m^2.  Chords
// farther than 9 sigma contribute below 1e-17 of the peak and are skipped.
__device__ __forceinline__ double chord_density(const Chord& c, double x, double y, double z,
                                                double sigma) {
  const double rx = x - c.mx, ry = y - c.my, rz = z - c.mz;
  const double s = rx * c.ux + ry * c.uy + rz * c.uz;
  const double r2 = rx * rx + ry * ry + rz * rz;
  double dp2 = r2 - s * s;
  dp2 = dp2 < 0.0 ? 0.0 : dp2;
  const double cut = 9.0 * sigma;
  if (dp2 > cut * cut || fabs(s) > c.half + cut) return 0.0;
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  const double radial = exp(-dp2 * inv2s2) * inv2s2 * (1.0 / M_PI);
  const double w = 1.0 / (M_SQRT2 * sigma);
  const double axial = 0.5 * (erf((c.half - s) * w) + erf((c.half + s) * w));
  return radial * axial;
}

struct StepBuffers {
  const float* hi_in;
  const float* lo_in;
  float* hi_out;
  float* lo_out;
  uint8_t* lab;
  const float* src;
  float* omega;
  const float* perf;     // may be null
  const Tables* tab;
  float* partials;       // [nwg * 3] for this step, may be null
  int n_classes;         // classes in use (table rows staged into LDS)
};

// ---- stepping ------------------------------------------------------------
// One step, one thread per voxel (reference kernel).  Returns work-groups
// per launch (the partials stride).
int naive_wg_count(Grid3 g);
hipError_t launch_step_naive(Grid3 g, const StepBuffers& b, const StepConst& K,
                             hipStream_t st);

// Sum step partials [n_slots][nwg][3] in fixed order into acc[3] (double,
// accumulated): acc += {perf, bnd, mono}.
hipError_t launch_reduce_partials(const float* partials, int n_slots, int nwg,
                                  double* acc, hipStream_t st);

// Per-instance sums of batch partials [n_slots][n_items][3] for instances
// inst0 .. inst0 + n_inst - 1: instance i owns items [first[2 i],
// first[2 i + 1]); acc[3 i + c] += its sum.  slot_acc is scratch of
// [instances][slot_stride][3] doubles (n_slots <= slot_stride <= 64).
hipError_t launch_reduce_batch(const float* partials, int n_slots, int n_items,
                               const int* first, int inst0, int n_inst, double* slot_acc,
                               int slot_stride, double* acc, hipStream_t st);

// ---- setup ---------------------------------------------------------------
// Build internal label bytes from class labels; counts labels >= n_classes.
hipError_t launch_build_labels(Grid3 g, const uint8_t* user, uint8_t* lab,
                               const ClassParams* cp_dev, unsigned* bad, hipStream_t st);
// Reset state: theta = t_fixed - 37 for fixed classes else 0, Omega = 0,
// latch from the initial temperature.
hipError_t launch_reset_state(Grid3 g, uint8_t* lab, float* hi, float* lo, float* om,
                              const ClassParams* cp_dev, float thr, hipStream_t st);
// Stability bound: min over free voxels of rho c / (sum K_f/d^2 + h f).
hipError_t launch_dt_bound(Grid3 g, const uint8_t* lab, const float* perf,
                           const ClassParams* cp_dev, double inv_d2x, double inv_d2y,
                           double inv_d2z, double* partial, int* nblk_out, double* result,
                           hipStream_t st);
// RF source: per-tine sums (pass 1) and field write (pass 2).
hipError_t launch_source_sums(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                              const Chord* chords, const int* tine_first, int n_tines,
                              double sigma, double* partial, int* nblk_out, double* sums,
                              hipStream_t st);
hipError_t launch_source_write(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                               const Chord* chords, const int* tine_first, int n_tines,
                               double sigma, const double* scale, double* q,
                               hipStream_t st);
// Stored per-tine densities u[t][n] (0 on held voxels), their integrals
// (same order as launch_source_sums) and q = sum_t scale[t] u_t.
hipError_t launch_source_fields(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                                const Chord* chords, const int* tine_first, int n_tines,
                                double sigma, double* u, hipStream_t st);
hipError_t launch_field_sums(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                             const double* u, int n_tines, double* partial, double* sums,
                             hipStream_t st);
hipError_t launch_source_combine(Grid3 g, const uint8_t* lab, const double* u, int n_tines,
                                 const double* scale, double* q, hipStream_t st);
// s = dt q / (rho c) on free voxels, 0 on held voxels; the labels' source
// flag (kSource) set exactly where s != 0.
hipError_t launch_source_increment(Grid3 g, uint8_t* lab, const double* q,
                                   const ClassParams* cp_dev, double dt, float* s,
                                   hipStream_t st);
// End-of-call state reduction: {energy J, tmin, tmax, nonfinite count}.
hipError_t launch_state_reduce(Grid3 g, const uint8_t* lab, const float* hi, const float* lo,
                               const ClassParams* cp_dev, double vol, double* partial,
                               double* out4, hipStream_t st);
// Damage mask and per-class dead counts [n][2].
hipError_t launch_damage(Grid3 g, const uint8_t* lab, const float* om, uint8_t* mask,
                         unsigned long long* counts, hipStream_t st);
// *count += voxels whose label has any bit of flag (count zeroed by the caller).
hipError_t launch_count_flag(Grid3 g, const uint8_t* lab, unsigned flag,
                             unsigned long long* count, hipStream_t st);
// p[0 .. n) = 0 (one small work-group; graph-capturable, unlike a memset).
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
// Plain streaming copy b = a of n4 float4 (bandwidth ceiling probe).
// Streaming probe of the step's 25 B/voxel mix: in = {hi, lo, omega},
// out likewise, lab one 32-bit word per four voxels; n4 float4 per array.
hipError_t launch_stream_mix(const float4* const (&in)[3], const unsigned* lab,
                             float4* const (&out)[3], size_t n4, int blocks, hipStream_t st);
hipError_t launch_copy(const float4* a, float4* b, size_t n4, int max_blocks, hipStream_t st);
// The same with non-temporal hints and four float4 per thread per pass.
hipError_t launch_copy_nt(const float4* a, float4* b, size_t n4, hipStream_t st);
// Free voxels per class [16].
hipError_t launch_free_counts(Grid3 g, const uint8_t* lab, unsigned long long* counts,
                              hipStream_t st);
// t_C = 37 + hi + lo (FP64).
hipError_t launch_temperature_out(Grid3 g, const float* hi, const float* lo, double* t,
                                  hipStream_t st);
// hi/lo = split(t_C - 37); latch |= tissue && theta >= thr.
hipError_t launch_temperature_in(Grid3 g, const double* t, float* hi, float* lo,
                                 uint8_t* lab, float thr, hipStream_t st);

}  // namespace rfa
