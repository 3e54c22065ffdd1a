/*
 * rfa.h -- C ABI of librfa.so, the MI355X (gfx950) explicit bioheat stepper
 * for radio-frequency ablation.
 *
 * Method (Kath, Handels, Mastmeyer, "Robust GPU-based Virtual Reality
 * Simulation of Radio Frequency Ablations for Various Needle Geometries and
 * Locations"): the simplified Pennes equation, Eq. (2675-eq1_Kath),
 *     rho c dT/dt = div(K grad T) + w_b c_b (T_a - T) + Q_m  (+ RF power q),
 * discretised with symmetric second differences, Eq. (2675-eq3), and an
 * explicit forward-Euler voxel update, Eq. (CUDAbioheat3d), on a voxel grid;
 * voxels of "fixed" classes keep their value (Alg. 1, Eq. (2675-eq6)); two
 * temperature images are swapped every step (Alg. 2).  The grid carries, per
 * voxel, the Arrhenius damage integral of Eq. (eq-tissState) and a latch of
 * the 60 degC instantaneous-necrosis threshold (Introduction).  The RF source
 * is a sum of Gaussian line sources, one per needle tine, each delivering a
 * given power.
 *
 * The problem statement maps onto the calls: the label image with its class
 * table is the initial condition g of Eq. (eq:setup) (Sec. "Implementation":
 * labels replaced by tissue temperatures), the needle is the additional term
 * f, held classes are the boundary condition h, and rfa_step advances N time
 * steps (Alg. 1).
 *
 * The arterial blood temperature T_a of Eq. (2675-eq1_Kath) is 37 degC (the
 * paper's value), which is also the initial temperature of free voxels.
 *
 * Conventions
 *  - Layout: every voxel array is C order [nx][ny][nz], z fastest.
 *  - Positions are metres in a frame centred on the grid: voxel i of n along
 *    an axis of spacing d sits at (2 i - (n - 1)) d / 2.
 *  - Units: SI (m, s, W, J, K); temperatures in degC.
 *  - Ownership: inputs are copied during the call, the caller keeps its
 *    buffers.  Outputs go to caller buffers.  A grid owns its device memory
 *    until rfa_destroy_grid.
 *  - Memory spaces: when rfa_options.inputs_on_device is set, every bulk voxel
 *    array argument (labels, temperatures, masks, damage, perfusion fields) is
 *    a device pointer on the grid's device; otherwise it is a host pointer.
 *    Small arguments (class table, needle, diagnostics, dead volumes) are
 *    always host memory.
 *  - Streams: all device work of a grid is issued on rfa_options.stream (a
 *    hipStream_t; NULL = the default stream).  Calls that write host outputs
 *    synchronise that stream before returning.
 *  - Errors: every call returns a status; nothing is thrown across the ABI.
 *    On error the grid is left as it was before the call (set_* calls
 *    validate everything before touching device state), and
 *    rfa_last_error() describes the failure (thread-local).
 *  - Threads: one grid per host thread at a time; distinct grids are
 *    independent.
 */
#ifndef RFA_H_
#define RFA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rfa_grid_s* rfa_grid; /* opaque handle, owned by the library */

typedef enum {
  RFA_OK = 0,
  RFA_ERR_ARG = 1,      /* invalid argument (sizes, NaN, label out of range) */
  RFA_ERR_STATE = 2,    /* call out of order (e.g. step before set_tissue)  */
  RFA_ERR_UNSTABLE = 3, /* dt above the explicit scheme's stability bound   */
  RFA_ERR_OOM = 4,      /* device allocation failed                         */
  RFA_ERR_HIP = 5,      /* HIP runtime error                                */
  RFA_ERR_NUMERIC = 6   /* NaN/Inf in the state after a step                */
} rfa_status;

/* One tissue class (Sec. "Specialized Methods for Liver Ablation
 * Simulation": rho, c_p, K, w_b c_b, Q_m; Eq. (2675-eq6) / Alg. 1 for held
 * classes). */
typedef struct {
  double k;        /* thermal conductivity K, W/m/K (>= 0)                    */
  double rho;      /* density, kg/m^3 (> 0)                                   */
  double c;        /* specific heat capacity c_p, J/kg/K (> 0)                */
  double h_perf;   /* volumetric perfusion coefficient w_b c_b, W/m^3/K (>= 0)*/
  double q_met;    /* metabolic heat Q_m, W/m^3                               */
  double t_fixed;  /* temperature of a held class, degC (used iff fixed)      */
  int fixed;       /* 1: voxels of this class keep their value                */
  int tissue;      /* 1: voxels of this class accumulate damage               */
} rfa_tissue;

/* RF needle: tine t is the polyline pts[pt_offset[t] .. pt_offset[t+1]-1]
 * (xyz triples, metres, grid-centre frame) delivering power[t] watts as a
 * uniform line density convolved with an isotropic Gaussian of standard
 * deviation sigma (metres).  Each tine's field is zeroed on held voxels and
 * scaled so the tine delivers exactly power[t] on the grid. */
typedef struct {
  int n_tines;            /* 0 clears the source                           */
  const int* pt_offset;   /* [n_tines + 1], increasing, >= 2 points a tine */
  const double* pts;      /* [3 * pt_offset[n_tines]]                      */
  const double* power;    /* [n_tines], W, >= 0                            */
  double sigma;           /* m, > 0                                        */
} rfa_needle;

/* Grid options; rfa_default_options fills the defaults given per field. */
typedef struct {
  double t_death;     /* necrosis latch threshold, degC (60)                */
  double A;           /* Arrhenius frequency factor, 1/s, >= 0 (7.39e39)    */
  double Ea;          /* activation energy, J/mol, >= 0 (2.577e5)           */
  double R;           /* gas constant, J/mol/K (8.314)                      */
  double omega_cap;   /* cap of the damage integral (1e30)                  */
  void* stream;       /* hipStream_t for all device work (NULL)            */
  int inputs_on_device; /* bulk voxel arrays are device pointers (0)        */
  int depth;          /* steps per kernel launch: 1, or 2 = temporal
                         blocking (tiled kernel, tile_y 8 or 16; two steps
                         per pass over memory, bitwise equal to two single
                         steps; odd step counts end with a single step;
                         one step per launch while damage-coupled perfusion
                         is on); 0 = automatic (0)                           */
  int kernel;         /* 0 automatic, 1 reference one-thread-per-voxel,
                         2 tiled 2.5-D (0)                                   */
  int tile_y;         /* tiled kernel: y rows per work-group (4, 8, 16);
                         0 = automatic (0)                                   */
  int tile_x;         /* tiled kernel: x planes per work-group; 0 = auto (0)*/
  int time_kernels;   /* N > 0: time step-kernel launches with HIP events,
                         one event pair per block of N consecutive launches
                         (read with rfa_kernel_stats); 0 = off (0)           */
  int z_vec;          /* tiled one-step kernel: consecutive z voxels per
                         lane, 1, 2 or 4 (2 and 4 need nz divisible by it,
                         tile_y 4 or 8; otherwise 1 is used); 0 = auto (0)   */
  int store_policy;   /* tiled kernels' store cache policy: 1 write-back,
                         2 write-through (sc1), 3 streaming (nt); 0 = auto:
                         streaming when the stepping working set exceeds
                         ~3/4 of the 256 MB last-level cache, else
                         write-through (0)                                   */
} rfa_options;

/* Diagnostics of one rfa_step call (energies relative to 37 degC, J). */
typedef struct {
  double energy_J;        /* heat content of free voxels after the call      */
  double injected_J;      /* RF + metabolic heat added during the call       */
  double perfusion_J;     /* heat removed by perfusion during the call       */
  double boundary_J;      /* heat received from held voxels during the call  */
  double residual_J;      /* energy change - (injected - perfusion + boundary)*/
  long long mono_violations; /* sum over steps of free voxels that cooled by
                                more than 2^-18 |T - 37 degC| + 1e-30 K in a
                                step (the check of the monotone rise of Sec.
                                "Results"; smaller falls are FP32 rounding
                                near balance or in the subnormal range)    */
  double t_min_C, t_max_C;   /* temperature range after the call            */
  long long steps;           /* steps taken by the call                      */
} rfa_diag;

rfa_status rfa_default_options(rfa_options* opt);

/* Create an nx x ny x nz grid (each >= 3) with spacing dx, dy, dz metres:
 * the voxel image on which Eq. (CUDAbioheat3d) is discretised, its spacing
 * the voxel distances of that equation (taken in metres; the text's
 * millimetres would be inconsistent with K in W/m/K).  Voxel (i, j, k) sits
 * at [i][j][k], k fastest.  opt may be NULL (defaults).  The grid owns its
 * device memory until rfa_destroy_grid; RFA_ERR_OOM if it does not fit.  The
 * grid has no tissue until rfa_set_tissue. */
rfa_status rfa_create_grid(int nx, int ny, int nz, double dx, double dy, double dz,
                           const rfa_options* opt, rfa_grid* out);

/* Set the class image and the class table (n_classes in 1..16) and reset the
 * state: held classes at t_fixed, all other voxels at 37 degC, damage 0,
 * latches from the initial temperatures.  The outermost voxel layer of the
 * grid is always held at its initial value.  Labels >= n_classes give
 * RFA_ERR_ARG.  (Sec. "Implementation": CT labels -> thermal start image.) */
rfa_status rfa_set_tissue(rfa_grid g, const uint8_t* labels, const rfa_tissue* table,
                          int n_classes);

/* Rasterise the needle's RF power density on the grid (FP64 on the device).
 * Requires tissue (held voxels receive no power).  n_tines == 0 clears it.
 * A tine with no weight on free voxels gives RFA_ERR_ARG. */
rfa_status rfa_set_needle(rfa_grid g, const rfa_needle* needle);

/* Per-voxel multiplier of the class perfusion coefficient (h = h_class * f),
 * f >= 0, [nx*ny*nz] float; NULL removes it (f = 1). */
rfa_status rfa_set_perfusion(rfa_grid g, const float* factor);

/* Damage-coupled perfusion (enable = 1; 0 turns it off, the default): the
 * blood-cooling term of the free voxels is scaled by the surviving cell
 * fraction c(t)/c(0) = exp(-Omega), Linte's tissue-state factor of Eq.
 * (2675-eq1_Linte) read through Eq. (eq-tissState), which defines the damage
 * integral as Omega = ln(c(0)/c(t)); Omega is the voxel's value at the start
 * of each step.  Dead tissue then loses its blood cooling.  Without a
 * perfusion field the grid gets one of ones.  The dt bound is that of the
 * uncoupled grid (exp(-Omega) <= 1).  While it is on, rfa_adjoint returns
 * RFA_ERR_ARG (the step is no longer linear in the temperature alone).
 * RFA_ERR_STATE before rfa_set_tissue; RFA_ERR_ARG for other values. */
rfa_status rfa_set_perfusion_decay(rfa_grid g, int enable);

/* Advance n_steps explicit steps of length dt seconds (Eq. (CUDAbioheat3d),
 * Alg. 1 and 2).  dt above the bound min over free voxels of
 * rho c / (sum_faces K_face / d^2 + h) gives RFA_ERR_UNSTABLE.  diag may be
 * NULL; if given, the call also sums per-step diagnostics and synchronises. */
rfa_status rfa_step(rfa_grid g, int n_steps, double dt, rfa_diag* diag);

/* Largest dt accepted by rfa_step for the current tissue and perfusion. */
rfa_status rfa_dt_max(rfa_grid g, double* dt_max);

/* Damage outputs (any may be NULL): mask bit0 = latched T >= t_death (the
 * Introduction's instant cell death above 60 degC, threshold t_death), bit1 =
 * damage integral >= 1 (Eq. (eq-tissState), Arrhenius with T in Kelvin;
 * tissue classes only); omega = damage integral (float); dead_m3[2*n_classes]
 * = per class dead volume by bit0 then by bit1, m^3 (the ablation zone of
 * Sec. "Results").  mask [nx*ny*nz] u8 and omega [nx*ny*nz] are caller
 * owned, host or device per inputs_on_device; dead_m3 is host memory.  Host
 * outputs synchronise the grid's stream; device outputs with dead_m3 = NULL
 * are only enqueued on it. */
rfa_status rfa_damage(rfa_grid g, uint8_t* mask, float* omega, double* dead_m3);

/* rfa_damage for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same outputs, bit for bit, with no hipMalloc, hipFree or other
 * allocating call.  Its scratch (the per-class dead counters, and the
 * staging of a host mask) is a static device array of 16 MiB + 256 bytes
 * that the library holds on every GPU it runs on until the process ends; a
 * host mask larger than 16 Mi voxels (over 256^3) gives RFA_ERR_ARG (device
 * masks have no limit).  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other threads, other streams) race; the
 * counters are cleared by a kernel at the start of each call.  With device
 * outputs (inputs_on_device) and dead_m3 = NULL the call only enqueues
 * work on the grid's stream and does not synchronise; host outputs
 * synchronise. */
rfa_status rfa_damage_noalloc(rfa_grid g, uint8_t* mask, float* omega, double* dead_m3);

/* Temperature outputs (any may be NULL): the current temperature image, the
 * per-frame output of Alg. 1 and 2 (Sec. "Implementation").  t_C = 37 + hi +
 * lo summed in FP64, degC, [nx*ny*nz] double; hi, lo = the raw float-float
 * excess-temperature state, [nx*ny*nz] float each.  Caller-owned buffers,
 * host or device per inputs_on_device; host outputs synchronise. */
rfa_status rfa_get_temperature(rfa_grid g, double* t_C, float* hi, float* lo);

/* Overwrite the temperature state (degC, double, [nx*ny*nz]); damage and
 * latches are kept.  Held voxels take the given values as well. */
rfa_status rfa_set_temperature(rfa_grid g, const double* t_C);

/* Breathing-motion view of the current temperature (Eq. (eq:breathing)):
 * out[x] = T(x + beta v(x)) in degC, T taken trilinearly between voxel
 * centres from the temperature state, sample positions beyond the grid
 * taken on its walls.  Accuracy: within 1e-4 K of the exact interpolant of
 * the float-float state (sample positions formed as float-float pairs; the
 * lo words of the state enter in cells with a corner at or above 1024 degC,
 * elsewhere they are below half an ulp of the hi word; the result rounded
 * once to float).  A sample exactly on a voxel centre (zero displacement,
 * integer shifts, positions clamped to a wall) is that voxel's float-float
 * state rounded once.  v: [3][nx*ny*nz] float, the
 * x, y and z components of the inverse breathing displacement in metres;
 * beta: the breathing surrogate (finite); out: [nx*ny*nz] float, caller
 * owned.  v and out are host or device pointers per inputs_on_device; on
 * the host path a non-finite displacement gives RFA_ERR_ARG, on the device
 * path it is not checked and samples a wall.  The state is not changed.
 * kernel_ms (may be NULL): if given, the call synchronises and returns the
 * warp kernel's duration measured with HIP events on the grid's stream.
 * Grids of 2^31 voxels or more give RFA_ERR_ARG. */
rfa_status rfa_warp(rfa_grid g, const float* v, double beta, float* out, double* kernel_ms);

/* The same view through a displacement combined from two fields,
 * beta1 v1(x) + beta2 v2(x): the keyframe form of the motion model (two
 * consecutive phase fields weighted 1 - a and a) or a regression on two
 * surrogate signals (Sec. "Consideration of Breathing Motion").  v1, v2 as v
 * above (v2 required); beta2 v2 is added to the float-float position
 * beta1 v1 by an exact two-sum, so beta2 = 0 gives exactly
 * rfa_warp(v1, beta1).
 * Errors as rfa_warp. */
rfa_status rfa_warp2(rfa_grid g, const float* v1, double beta1, const float* v2, double beta2,
                     float* out, double* kernel_ms);

/* Serialise / restore the full dynamic state (temperature, damage, latches,
 * step count) with a checksum.  bytes: in = capacity, out = size needed
 * (call with buf == NULL to query).  A buffer from another grid shape or a
 * corrupted one gives RFA_ERR_STATE. */
rfa_status rfa_save_state(rfa_grid g, void* buf, size_t* bytes);
rfa_status rfa_load_state(rfa_grid g, const void* buf, size_t bytes);

/* Steps taken since the last rfa_set_tissue / rfa_load_state. */
rfa_status rfa_get_step_count(rfa_grid g, long long* steps);

/* Voxels on which the RF increment is nonzero after the last step (the
 * support of the needle's Gaussian line sources, cut where a chord's
 * density falls below 1e-17 of its peak): the step kernels read the
 * source field only there, so a step moves 4 * voxels bytes of it rather
 * than 4 * nx*ny*nz.  RFA_ERR_STATE until a step has followed the last
 * change of tissue, needle or time step. */
rfa_status rfa_source_support(rfa_grid g, long long* voxels);

/* Step-kernel timing accumulated since the last call (requires
 * rfa_options.time_kernels): total milliseconds measured with HIP events
 * around blocks of consecutive step-kernel launches (diagnostic reductions
 * excluded), number of launches in those blocks, voxel-steps they advanced.
 * Resets the counters.  Any argument may be NULL. */
rfa_status rfa_kernel_stats(rfa_grid g, double* kernel_ms, long long* launches,
                            long long* voxel_steps);

/* Adjoint-kernel timing accumulated since the last call (requires
 * rfa_options.time_kernels; kept-trajectory adjoints only, ckpt_every = 0):
 * total milliseconds measured with one pair of HIP events around each
 * adjoint's back-to-back step launches, and the number of those launches.
 * Resets the counters.  Either argument may be NULL. */
rfa_status rfa_adjoint_kernel_stats(rfa_grid g, double* kernel_ms, long long* launches);

/* Current launch plan: kernel (1 reference, 2 tiled), steps per launch,
 * tile rows, x planes per work-group, work-groups per launch, z voxels per
 * lane. */
rfa_status rfa_get_plan(rfa_grid g, int* kernel, int* depth, int* tile_y, int* tile_x,
                        int* workgroups, int* z_vec);

/* Time the candidate launch plans of this grid's shape on scratch copies of
 * its state (the state is not advanced) and keep the fastest per step: the
 * one-step tiled plans, and the two-step plans unless the grid was created
 * with depth 1.  dt as for rfa_step; reps launches per candidate.  Results
 * are cached per grid shape for the process. */
rfa_status rfa_tune(rfa_grid g, double dt, int reps);

/* Measured device-to-device streaming-copy bandwidth over `bytes` bytes
 * (read + write counted), GB/s: the achievable HBM ceiling on this device. */
rfa_status rfa_copy_bandwidth(size_t bytes, int reps, double* gbps);

/* Measured streaming rate of the step kernels' byte mix without their
 * stencil, GB/s: per voxel theta hi and lo, the class byte and Omega read,
 * theta and Omega written (25 B, counted as such), over n_voxels voxels
 * (>= 4096; rounded up to a multiple of 4) in two image sets used in turn,
 * reps passes, the fastest of five launch widths.  The ceiling a step
 * kernel of that grid size could reach; n_voxels * 25 B of device memory
 * is allocated for the call.  Errors: RFA_ERR_ARG (arguments),
 * RFA_ERR_OOM / RFA_ERR_HIP (device). */
rfa_status rfa_mix_bandwidth(long long n_voxels, int reps, double* gbps);

/* ---- Differentiation -------------------------------------------------------
 * The damage integral after N steps, Omega^N (Eq. (eq-tissState) summed by
 * the stepper), is a differentiable function of the tine powers and of the
 * perfusion field.  rfa_forward_checkpointed runs the forward keeping either
 * the temperature of every step (ckpt_every = 0; (N + 1) * 4 bytes per voxel
 * of device memory, 5 GB for 128^3 x 600 steps) or the state every
 * ckpt_every steps; rfa_adjoint then runs the exact discrete adjoint of
 * those steps backwards (with checkpoints, recomputing each segment from its
 * checkpoint, bitwise as in the forward, so both schedules give the same
 * gradients) for a loss whose gradient with respect to Omega^N is given.  The adjoint differentiates the damage rate
 * where its exponent cap is inactive and voxels whose Omega^N reached the
 * cap not at all; latches are not differentiable and do not enter. */

/* Perfusion multiplier f = exp(sum_j B_j(x) ctrl_j) from a uniform cubic
 * B-spline lattice of m x m x m control values spanning the grid (voxel i of
 * n along an axis sits at spline coordinate i (m - 3) / (n - 1)); ctrl is a
 * host float array [m][m][m], m in 4..64, |ctrl| <= 30.  Replaces any
 * rfa_set_perfusion field. */
rfa_status rfa_set_perfusion_bspline(rfa_grid g, int m, const float* ctrl);

/* Back to the state rfa_set_tissue creates (temperature, damage, latches,
 * step count); tissue, needle and perfusion are kept. */
rfa_status rfa_reset_state(rfa_grid g);

/* New tine powers (W, [n_tines]) for the current needle geometry. */
rfa_status rfa_set_tine_powers(rfa_grid g, const double* power);

/* n_steps forward steps (as rfa_step) keeping, for rfa_adjoint, the
 * temperature (hi word) of every step when ckpt_every = 0 (one step per
 * launch, written straight into the kept trajectory; RFA_ERR_OOM if it does
 * not fit: use checkpoints), else the state at steps 0, ckpt_every,
 * 2 ckpt_every, ... plus the hi word of every step of the last segment,
 * written into the adjoint's segment buffer (2 (ckpt_every + 1) images,
 * allocated here), so the first rfa_adjoint after it recomputes every
 * segment but the last. */
rfa_status rfa_forward_checkpointed(rfa_grid g, int n_steps, double dt, int ckpt_every);

/* Adjoint of the last rfa_forward_checkpointed (the grid must not have
 * changed since; RFA_ERR_STATE otherwise).  w_omega = dL/dOmega^N per voxel
 * (float, [nx*ny*nz], memory space per inputs_on_device).  Outputs, each
 * nullable: dL_dP[n_tines] (host, W^-1), dL_dctrl[m^3] (host; requires
 * rfa_set_perfusion_bspline), dL_dperf[nx*ny*nz] = dL/df per voxel (float,
 * memory space per inputs_on_device).  With checkpoints, each segment is
 * recomputed on a second stream owned by the grid, into one half of a
 * double buffer of (ckpt_every + 1) images, while the adjoint steps of the
 * later segment run on the grid's stream; events order the two, so all of
 * the call's work stays ordered after earlier and before later work on the
 * grid's stream. */
rfa_status rfa_adjoint(rfa_grid g, const float* w_omega, double* dL_dP, double* dL_dctrl,
                       float* dL_dperf);

/* ---- Batched stepping of many grids (planning sweeps) ---------------------
 * A batch advances n independent grids -- each with its own shape, spacing,
 * tissue, needle and time step -- by the same number of steps.  Consecutive
 * grids are grouped up to a voxel budget (by default 8 Mi voxels, whose
 * stepping working set fits the 256 MB last-level cache); a group runs
 * all its steps before the next group starts, one kernel launch per step
 * over the concatenated work-item lists of its grids (two when some grids
 * carry a perfusion field and others do not).  The whole launch sequence of an
 * rfa_batch_step call is captured once in a hipGraph and replayed on later
 * calls with the same step count.  The per-voxel
 * arithmetic is that of rfa_step (Eq. (CUDAbioheat3d), Alg. 1 and 2), so a
 * batch step leaves each grid bitwise in the state rfa_step would.
 *
 * The batch borrows the grids (it does not own them; destroy the batch
 * before its grids).  Grids stay usable on their own: a grid stepped or
 * modified outside the batch is picked up again at the next batch call. */
typedef struct rfa_batch_s* rfa_batch;

/* grids[n] must all have tissue; dt[n] seconds, each within its grid's
 * stability bound (RFA_ERR_UNSTABLE otherwise). */
rfa_status rfa_batch_create(int n, const rfa_grid* grids, const double* dt, rfa_batch* out);

/* Advance every grid of the batch by n_steps of its own dt.  diags may be
 * NULL or point to n rfa_diag (filled as rfa_step does for each grid; the
 * call then synchronises). */
rfa_status rfa_batch_step(rfa_batch b, int n_steps, rfa_diag* diags);

/* Work-item layouts of the batch kernel. */
enum {
  RFA_BATCH_TILES = 1, /* 2.5-D tiles: 64 z voxels by tile_y rows */
  RFA_BATCH_FLAT = 2   /* flat segments of 64 * tile_y consecutive voxels of a
                          (y, z) plane; needs nz <= 32 * tile_y in every grid */
};

/* Launch shape of the batch kernel (default: RFA_BATCH_FLAT with 8 waves
 * when every grid has nz <= 256, else RFA_BATCH_TILES with 4 rows; 8 x
 * planes per work item; groups of at most 8 Mi voxels): layout (0: keep,
 * else RFA_BATCH_*),
 * tile_y waves per work-group (tiles: 4 or 8 rows; flat: 8 or 16; 0 keeps
 * the current value, or takes 4 / 8 when the layout changes), tile_x
 * planes per work item, workgroups > 0 persistent work-groups per launch
 * that walk the work list (0, the default: one work-group per work item),
 * group_voxels the grouping budget (0: all grids in one group, i.e.
 * lockstep; < 0: keep the current one).  On error the plan is unchanged.
 * Drops cached graphs. */
rfa_status rfa_batch_set_plan(rfa_batch b, int layout, int tile_y, int tile_x, int workgroups,
                              long long group_voxels);

/* Current launch shape: layout, tile_y, tile_x, work items per step (all
 * groups), work-groups launched per step of all grids, number of groups
 * (each pointer nullable). */
rfa_status rfa_batch_get_plan(rfa_batch b, int* layout, int* tile_y, int* tile_x, int* items,
                              int* workgroups, int* groups);

/* Pick the batch's launch shape by timing: work-item layouts, tile rows and
 * x planes per item at the default grouping, then grouping budgets for the
 * fastest shape (0 included: lockstep), each over reps steps of all grids
 * (one untimed replay first); keeps the fastest.  The grids' states are
 * snapshotted in device memory (13 bytes per voxel) and restored, so the
 * batch and its grids are left exactly as they were apart from the plan.
 * Batch work items take one step per launch; see rfa_tune for the
 * single-grid temporal blocking depth. */
rfa_status rfa_batch_tune(rfa_batch b, int reps);

/* Device time of the last rfa_batch_step's graph, milliseconds (HIP events
 * on the batch's stream), and voxel-steps it advanced. */
rfa_status rfa_batch_last_time(rfa_batch b, double* ms, long long* voxel_steps);

void rfa_batch_destroy(rfa_batch b);

void rfa_destroy_grid(rfa_grid g);
const char* rfa_status_string(rfa_status s);
const char* rfa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RFA_H_ */
