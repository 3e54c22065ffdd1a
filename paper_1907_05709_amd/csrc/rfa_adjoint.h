// rfa_adjoint.h -- launchers of the adjoint and perfusion-field kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rfa_kernels.h"

namespace rfa {

struct AdjointBuffers {
  const float* lam_in;   // lambda^{n+1}
  float* lam_out;        // lambda^n
  const float* theta;    // theta^n (hi part of the recomputed state)
  const uint8_t* lab;
  const float* perf;     // perfusion multiplier, may be null
  const float* w;        // dL/dOmega^N, zeroed where it cannot act
  const Tables* tab;
  float* sacc;           // += lambda^{n+1}          (dL/ds), on the source's support
  float* facc;           // += -B theta^n lambda^{n+1} (dL/df)
  // sacc is read and written only on voxels flagged kSource (dL/dP needs it
  // only where a tine's density is nonzero, and is exactly 0 elsewhere);
  // sacc_all: on every free voxel (when a tine has zero power its density
  // is nonzero where the flagged increment is not)
  bool sacc_all;
};

hipError_t launch_bspline_eval(Grid3 g, const float* ctrl, int m, float* f, hipStream_t st);
// gctrl[m^3] = sum_p gf_p f_p B(x_p) as three separable contractions (FP64,
// fixed order).  vfirst_a[s] = first voxel of knot span s along axis a,
// s = 0 .. m-3; scratch holds bspline_grad_scratch(g, m) doubles.
size_t bspline_grad_scratch(Grid3 g, int m);
hipError_t launch_bspline_grad(Grid3 g, const float* gf, const float* f, int m,
                               const int* vfirst_x, const int* vfirst_y, const int* vfirst_z,
                               double* scratch, double* gctrl, hipStream_t st);
hipError_t launch_adjoint_weight(Grid3 g, const float* w, const float* om, const uint8_t* lab,
                                 float cap, float* wa, hipStream_t st);
// Reference adjoint step (one thread per voxel).
hipError_t launch_adjoint_step(Grid3 g, const AdjointBuffers& a, const StepConst& K,
                               hipStream_t st);
// The same step with the tiled schedule (ty = 4 or 8 rows, xc x planes per
// work-group); bitwise equal to the reference.
bool adjoint_tiled_fits(Grid3 g, int xc);
hipError_t launch_adjoint_tiled(Grid3 g, int ty, int xc, const AdjointBuffers& a,
                                const StepConst& K, hipStream_t st);
// partial[t * nblk + b]: per-block sums of g_t(p) sacc_p dt / (rho c)_p.
hipError_t launch_source_dot(Grid3 g, double dx, double dy, double dz, const uint8_t* lab,
                             const Chord* chords, const int* tine_first, int n_tines,
                             double sigma, const float* sacc, const ClassParams* cp_dev,
                             double dt, double* partial, int nblk, hipStream_t st);

hipError_t launch_source_dot_fields(Grid3 g, const uint8_t* lab, const double* u, int n_tines,
                                    const float* sacc, const ClassParams* cp_dev, double dt,
                                    double* partial, int nblk, hipStream_t st);

}  // namespace rfa
