// rfa_api.hip -- runtime and C ABI of librfa.so (see include/rfa.h).
//
// The runtime owns the device state of a grid (ping-pong float-float
// temperature images, label bytes with flags, damage integral, RF source,
// coefficient tables), validates every argument before touching it,
// rebuilds the per-dt coefficient tables and the source increment when dt
// changes, and issues every kernel on the grid's stream.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rfa.h"
#include "rfa_kernels.h"
#include "rfa_adjoint.h"
#include "rfa_step.h"
#include "rfa_warp.h"

using namespace rfa;

namespace {

thread_local std::string g_last_error;

// roctx range around a public call, so rocprofv3 --marker-trace shows the
// library's calls (rfa_step, rfa_batch_step, ...) around their kernels.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

rfa_status fail(rfa_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RFA_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

constexpr int kPartialSlots = 64;  // steps of diagnostic partials per reduction
constexpr size_t kFieldBudget = size_t(16) << 30;  // bytes of kept per-tine source densities
// Voxels per batch group: a group's stepping working set (two state images,
// class bytes, source, damage: ~29 B per voxel, 8 Mi voxels ~ 243 MB) stays
// within the 256 MB last-level cache while its steps run.
constexpr long long kBatchGroupVoxels = 8ll << 20;
constexpr int kTimedBatch = 1024;  // launches between event read-backs
constexpr double kTBodyK = 310.15;
constexpr double kExponentClamp = 80.0;

}  // namespace

struct rfa_grid_s {
  Grid3 g{0, 0, 0};
  double dx = 0, dy = 0, dz = 0;
  rfa_options opt{};
  hipStream_t st = nullptr;
  int device = 0;

  bool has_tissue = false;
  int n_classes = 0;
  rfa_tissue table[kMaxClasses]{};
  ClassParams cp{};
  ClassParams* cp_dev = nullptr;
  unsigned long long free_count[kMaxClasses]{};

  uint8_t* lab = nullptr;
  float* hi[2] = {nullptr, nullptr};
  float* lo[2] = {nullptr, nullptr};
  int cur = 0;
  float* om = nullptr;
  float* src = nullptr;
  double* q64 = nullptr;
  float* perf = nullptr;  // null = no perfusion multiplier
  bool perf_decay = false;  // perfusion scaled by exp(-Omega); needs perf (ones if unset)
  Tables* tab_dev = nullptr;
  Tables tab_host{};
  double tab_dt = -1.0;
  double src_dt = -1.0;

  bool has_needle = false;
  std::vector<int> pt_offset;
  std::vector<double> pts, power;
  double sigma = 0.0;
  double rf_power = 0.0;
  Chord* chords_dev = nullptr;     // chords of the rasterised needle
  int* first_dev = nullptr;        // first chord of each tine (+ end)
  std::vector<double> tine_sums;   // integral of each tine's unnormalised density, m
  double* tine_u = nullptr;        // [n_tines][n] unnormalised densities (if kept)
  size_t tine_u_cap = 0;           // doubles allocated at tine_u
  bool fields_ok = false;          // tine_u holds the current needle's densities
  double* scale_dev = nullptr;     // [scale_cap] power / integral per tine
  size_t scale_cap = 0;

  // perfusion-correction B-spline (m^3 control points), if set
  int bs_m = 0;
  float* bs_ctrl = nullptr;
  int* bs_vfirst = nullptr;        // [3][m - 2] first voxel of each knot span

  // checkpointed forward and adjoint
  int version = 0;                 // bumped by every change of inputs or state
  bool adj_ready = false;
  int adj_version = 0;
  int adj_steps = 0, adj_every = 0, adj_nckpt = 0;
  bool adj_tail_kept = false;      // traj holds the last segment's hi images (see rfa_adjoint)
  double adj_dt = 0.0;
  float* ckpt = nullptr;           // [nckpt][2][N] hi, lo at segment starts
  size_t ckpt_floats = 0;
  float* traj = nullptr;           // hi images: the kept trajectory [N + 1] or a segment [every + 1]
  size_t traj_floats = 0;
  float* adj_work = nullptr;       // lo ping-pong (2N), lambda (2N), sacc, facc, w, omega scratch
  uint8_t* lab_scratch = nullptr;

  double dt_max = 0.0;
  long long steps = 0;

  // scratch
  float* partials = nullptr;
  size_t partial_floats = 0;
  double* dacc = nullptr;          // [3] step partial accumulators
  double* red = nullptr;           // reduction partials
  size_t red_doubles = 0;
  double* out4 = nullptr;          // [4] state reduction result
  unsigned long long* counts = nullptr;  // [32]
  unsigned* bad = nullptr;
  double energy = 0.0;
  bool energy_valid = false;

  StepPlan plan{};

  // step-kernel timing
  std::vector<hipEvent_t> events;
  // second stream of the checkpointed adjoint (segment recomputes run on it
  // while the adjoint steps of the next later segment run on st) and its
  // ordering events: start, recompute done [2], adjoint done [2]
  hipStream_t side = nullptr;
  hipEvent_t side_ev[5] = {};
  double kernel_ms = 0.0;
  long long kernel_launches = 0;
  long long kernel_voxel_steps = 0;
  // adjoint-kernel timing (kept-trajectory schedule)
  double adj_kernel_ms = 0.0;
  long long adj_kernel_launches = 0;
};

namespace {

void free_all(rfa_grid g) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(g->cp_dev);
  f(g->lab);
  f(g->hi[0]);
  f(g->hi[1]);
  f(g->lo[0]);
  f(g->lo[1]);
  f(g->om);
  f(g->src);
  f(g->q64);
  f(g->perf);
  f(g->tab_dev);
  f(g->partials);
  f(g->dacc);
  f(g->red);
  f(g->out4);
  f(g->counts);
  f(g->bad);
  f(g->chords_dev);
  f(g->first_dev);
  f(g->tine_u);
  f(g->scale_dev);
  f(g->bs_ctrl);
  f(g->bs_vfirst);
  f(g->ckpt);
  f(g->traj);
  f(g->adj_work);
  f(g->lab_scratch);
  for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
  g->events.clear();
  for (hipEvent_t& e : g->side_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (g->side) (void)hipStreamSynchronize(g->side);
  if (g->side) (void)hipStreamDestroy(g->side);
  g->side = nullptr;
}

template <class T>
rfa_status dmalloc(T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(RFA_ERR_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  return RFA_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

hipMemcpyKind kind_in(const rfa_grid g) {
  return g->opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_out(const rfa_grid g) {
  return g->opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

// Harmonic-mean face conductivity (series resistance of two half voxels).
double face_k(double a, double b) { return (a + b) == 0.0 ? 0.0 : 2.0 * a * b / (a + b); }

void split(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

// Per-dt coefficient tables (FP64 -> float-float).
void build_tables(rfa_grid g, double dt) {
  Tables& T = g->tab_host;
  std::memset(&T, 0, sizeof T);
  const double d2[3] = {g->dx * g->dx, g->dy * g->dy, g->dz * g->dz};
  const double vol = g->dx * g->dy * g->dz;
  for (int a = 0; a < g->n_classes; ++a) {
    const rfa_tissue& ta = g->table[a];
    const double rc = ta.rho * ta.c;
    for (int b = 0; b < g->n_classes; ++b) {
      const double kf = face_k(ta.k, g->table[b].k);
      for (int ax = 0; ax < 3; ++ax) {
        float h, l;
        split(dt * kf / (rc * d2[ax]), h, l);
        T.cf[ax][a * kMaxClasses + b] = make_float2(h, l);
      }
    }
    float bh, bl;
    split(dt * ta.h_perf / rc, bh, bl);
    T.cls[a] = make_float4(bh, bl, (float)(dt * ta.q_met / rc), (float)(rc * vol));
  }
}

StepConst step_const(rfa_grid g, double dt) {
  StepConst K;
  const double c = g->opt.Ea / (g->opt.R * kTBodyK);
  K.dtka = (float)(dt * g->opt.A * std::exp(-c));
  K.c2 = (float)(c * M_LOG2E);
  K.tak = (float)kTBodyK;
  K.clamp2 = (float)(kExponentClamp * M_LOG2E);
  K.cap = (float)g->opt.omega_cap;
  K.thr = (float)(g->opt.t_death - 37.0);
  K.decay2 = g->perf_decay ? (float)M_LOG2E : 0.0f;
  return K;
}

// A perfusion field of ones (allocated if missing), for damage-coupled
// perfusion without a multiplier of its own.
rfa_status unit_perf(rfa_grid g) {
  if (!g->perf) {
    rfa_status s = dmalloc(&g->perf, g->g.n());
    if (s != RFA_OK) return s;
  }
  HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)g->perf, 0x3f800000, g->g.n(), g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  return RFA_OK;
}

rfa_status compute_dt_max(rfa_grid g) {
  int nblk = 0;
  HIP_TRY(launch_dt_bound(g->g, g->lab, g->perf, g->cp_dev, 1.0 / (g->dx * g->dx),
                          1.0 / (g->dy * g->dy), 1.0 / (g->dz * g->dz), g->red, &nblk,
                          g->out4, g->st));
  double v = 0.0;
  HIP_TRY(hipMemcpyAsync(&v, g->out4, sizeof v, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  g->dt_max = v;
  return RFA_OK;
}

// Rasterise the stored needle into q64 (zero if none) and invalidate s.
rfa_status rasterise(rfa_grid g) {
  g->src_dt = -1.0;
  ++g->version;
  g->fields_ok = false;
  if (!g->has_needle) {
    HIP_TRY(hipMemsetAsync(g->q64, 0, g->g.n() * sizeof(double), g->st));
    g->rf_power = 0.0;
    return RFA_OK;
  }
  const int nt = (int)g->power.size();
  std::vector<Chord> chords;
  std::vector<int> first(nt + 1, 0);
  for (int t = 0; t < nt; ++t) {
    first[t] = (int)chords.size();
    for (int p = g->pt_offset[t]; p + 1 < g->pt_offset[t + 1]; ++p) {
      const double* a = &g->pts[3 * p];
      const double* b = &g->pts[3 * (p + 1)];
      const double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
      const double len = std::sqrt(ux * ux + uy * uy + uz * uz);
      if (len == 0.0) continue;
      Chord c;
      c.mx = 0.5 * (a[0] + b[0]);
      c.my = 0.5 * (a[1] + b[1]);
      c.mz = 0.5 * (a[2] + b[2]);
      c.ux = ux / len;
      c.uy = uy / len;
      c.uz = uz / len;
      c.half = 0.5 * len;
      c.tine = t;
      c.pad = 0;
      chords.push_back(c);
    }
  }
  first[nt] = (int)chords.size();
  Chord* d_chords = nullptr;
  int* d_first = nullptr;
  double* d_sums = nullptr;
  double* d_partial = nullptr;
  rfa_status s;
  if ((s = dmalloc(&d_chords, chords.size())) != RFA_OK) return s;
  if ((s = dmalloc(&d_first, first.size())) != RFA_OK) { (void)hipFree(d_chords); return s; }
  if ((s = dmalloc(&d_sums, 2 * (size_t)nt)) != RFA_OK) {
    (void)hipFree(d_chords); (void)hipFree(d_first); return s;
  }
  if ((s = dmalloc(&d_partial, (size_t)nt * 1024)) != RFA_OK) {
    (void)hipFree(d_chords); (void)hipFree(d_first); (void)hipFree(d_sums); return s;
  }
  auto cleanup = [&]() {
    (void)hipFree(d_chords);
    (void)hipFree(d_first);
    (void)hipFree(d_sums);
    (void)hipFree(d_partial);
  };
  std::vector<double> sums(nt), scale(nt);
  hipError_t e = hipSuccess;
  int nblk = 0;
  // Keep the per-tine densities when they fit the budget: new tine powers
  // then only recombine them, and dL/dP reads them instead of recomputing.
  const size_t nu = (size_t)nt * g->g.n();
  bool keep = nu * sizeof(double) <= kFieldBudget;
  if (keep && g->tine_u_cap < nu) {
    if (g->tine_u) (void)hipFree(g->tine_u);
    g->tine_u = nullptr;
    g->tine_u_cap = 0;
    if (hipMalloc((void**)&g->tine_u, nu * sizeof(double)) == hipSuccess)
      g->tine_u_cap = nu;
    else
      keep = false;  // fall back to recomputing the densities
    (void)hipGetLastError();
  }
  g->fields_ok = false;
  do {
    if ((e = hipMemcpyAsync(d_chords, chords.data(), chords.size() * sizeof(Chord),
                            hipMemcpyHostToDevice, g->st)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(d_first, first.data(), first.size() * sizeof(int),
                            hipMemcpyHostToDevice, g->st)) != hipSuccess) break;
    if (keep) {
      if ((e = launch_source_fields(g->g, g->dx, g->dy, g->dz, g->lab, d_chords, d_first, nt,
                                    g->sigma, g->tine_u, g->st)) != hipSuccess) break;
      if ((e = launch_field_sums(g->g, g->dx, g->dy, g->dz, g->lab, g->tine_u, nt, d_partial,
                                 d_sums, g->st)) != hipSuccess) break;
    } else if ((e = launch_source_sums(g->g, g->dx, g->dy, g->dz, g->lab, d_chords, d_first,
                                       nt, g->sigma, d_partial, &nblk, d_sums, g->st)) !=
               hipSuccess) {
      break;
    }
    if ((e = hipMemcpyAsync(sums.data(), d_sums, nt * sizeof(double), hipMemcpyDeviceToHost,
                            g->st)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(g->st)) != hipSuccess) break;
  } while (false);
  if (e != hipSuccess) {
    cleanup();
    return fail(RFA_ERR_HIP, "source rasterisation failed: %s", hipGetErrorString(e));
  }
  for (int t = 0; t < nt; ++t) {
    if (!(sums[t] > 0.0)) {
      cleanup();
      return fail(RFA_ERR_ARG, "tine %d has no weight on free voxels", t);
    }
    scale[t] = g->power[t] / sums[t];
  }
  do {
    if ((e = hipMemcpyAsync(d_sums + nt, scale.data(), nt * sizeof(double),
                            hipMemcpyHostToDevice, g->st)) != hipSuccess) break;
    if (keep)
      e = launch_source_combine(g->g, g->lab, g->tine_u, nt, d_sums + nt, g->q64, g->st);
    else
      e = launch_source_write(g->g, g->dx, g->dy, g->dz, g->lab, d_chords, d_first, nt,
                              g->sigma, d_sums + nt, g->q64, g->st);
    if (e != hipSuccess) break;
    if ((e = hipStreamSynchronize(g->st)) != hipSuccess) break;
  } while (false);
  if (e != hipSuccess) {
    cleanup();
    return fail(RFA_ERR_HIP, "source write failed: %s", hipGetErrorString(e));
  }
  g->fields_ok = keep;
  // keep the chord list and tine integrals for the adjoint's dL/dP
  (void)hipFree(d_sums);
  (void)hipFree(d_partial);
  if (g->chords_dev) (void)hipFree(g->chords_dev);
  if (g->first_dev) (void)hipFree(g->first_dev);
  g->chords_dev = d_chords;
  g->first_dev = d_first;
  g->tine_sums = sums;
  double tot = 0.0;
  for (double p : g->power) tot += p;
  g->rf_power = tot;
  return RFA_OK;
}

rfa_status ensure_events(rfa_grid g, int count) {
  while ((int)g->events.size() < count) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    g->events.push_back(e);
  }
  return RFA_OK;
}

// The adjoint's second stream (default priority, not blocking on the null
// stream) and its ordering events, created on first use.
rfa_status ensure_side_stream(rfa_grid g) {
  if (!g->side) HIP_TRY(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking));
  for (hipEvent_t& e : g->side_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return RFA_OK;
}

// Per-dt coefficient tables and source increment of grid g.
rfa_status prepare_dt(rfa_grid g, double dt) {
  if (dt != g->tab_dt) {
    build_tables(g, dt);
    HIP_TRY(hipMemcpyAsync(g->tab_dev, &g->tab_host, sizeof(Tables), hipMemcpyHostToDevice, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    g->tab_dt = dt;
  }
  if (dt != g->src_dt) {
    HIP_TRY(launch_source_increment(g->g, g->lab, g->q64, g->cp_dev, dt, g->src, g->st));
    g->src_dt = dt;
  }
  return RFA_OK;
}

rfa_status state_reduce(rfa_grid g, double out[4]);
rfa_status ensure_events(rfa_grid g, int count);

// Advance the grid's current state n_steps with its launch plan (step
// partials into g->dacc when diag), timing launch blocks with HIP events
// when the grid was created with time_kernels.  Updates the step count.
// With traj: one step per launch, the hi image of step *traj_t read from
// traj[*traj_t] and written to traj[*traj_t + 1] (the grid's hi images are
// not touched).
rfa_status timed_steps(rfa_grid g, const StepConst& K, int n_steps, bool diag,
                       float* traj = nullptr, int* traj_t = nullptr) {
  StepState ss{g->hi, g->lo, &g->cur, g->lab, g->src, g->om, g->perf, g->tab_dev,
               g->n_classes};
  // one step per launch for the kept trajectory, and with damage-coupled
  // perfusion: the two-step kernel reads the damage integral of its halo
  // voxels while the neighbouring work-groups overwrite it, harmless while
  // the damage integral feeds no temperature
  const StepPlan plan = (traj || g->perf_decay) ? plan_one(g->plan) : g->plan;
  if (traj) {
    ss.traj = traj;
    ss.traj_t = traj_t;
    ss.traj_n = g->g.n();
  }
  rfa_status s = RFA_OK;
  for (int done = 0; done < n_steps;) {
    const int batch = std::min(n_steps - done, kTimedBatch);
    hipEvent_t* ev = nullptr;
    if (g->opt.time_kernels) {
      if ((s = ensure_events(g, 2 * batch)) != RFA_OK) return s;
      ev = g->events.data();
    }
    int timed = 0, launches = 0;
    s = run_steps(g->g, plan, ss, K, batch, diag ? g->partials : nullptr, kPartialSlots,
                  g->dacc, ev, g->opt.time_kernels, &timed, &launches, g->st);
    if (s != RFA_OK)
      return fail(s, "step launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (ev && timed > 0) {
      HIP_TRY(hipEventSynchronize(ev[2 * timed - 1]));
      for (int k = 0; k < timed; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
        g->kernel_ms += ms;
      }
      g->kernel_launches += launches;
      g->kernel_voxel_steps += (long long)launches * plan.depth * (long long)g->g.n();
    }
    done += batch;
    g->steps += batch;
  }
  return RFA_OK;
}

rfa_status ensure_energy(rfa_grid g) {
  if (g->energy_valid) return RFA_OK;
  double r[4];
  rfa_status s = state_reduce(g, r);
  if (s != RFA_OK) return s;
  g->energy = r[0];
  g->energy_valid = true;
  return RFA_OK;
}

// Fill an rfa_diag from accumulated step partials acc[3] (perfusion J,
// heat from held voxels J, cooling voxel count) and a fresh state reduction.
rfa_status finish_diag(rfa_grid g, const double* acc, double e0, double dt, int n_steps,
                       rfa_diag* diag);

rfa_status state_reduce(rfa_grid g, double out[4]) {
  HIP_TRY(launch_state_reduce(g->g, g->lab, g->hi[g->cur], g->lo[g->cur], g->cp_dev,
                              g->dx * g->dy * g->dz, g->red, g->out4, g->st));
  HIP_TRY(hipMemcpyAsync(out, g->out4, 4 * sizeof(double), hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  return RFA_OK;
}

rfa_status finish_diag(rfa_grid g, const double* acc, double e0, double dt, int n_steps,
                       rfa_diag* diag) {
  double r[4];
  rfa_status s = state_reduce(g, r);
  if (s != RFA_OK) return s;
  g->energy = r[0];
  g->energy_valid = true;
  const double vol = g->dx * g->dy * g->dz;
  double met = 0.0;
  for (int c = 0; c < g->n_classes; ++c)
    met += g->table[c].q_met * (double)g->free_count[c] * vol;
  diag->energy_J = r[0];
  diag->injected_J = (g->rf_power + met) * dt * n_steps;
  diag->perfusion_J = acc[0];
  diag->boundary_J = acc[1];
  diag->residual_J = (r[0] - e0) - (diag->injected_J - diag->perfusion_J + diag->boundary_J);
  diag->mono_violations = (long long)std::llround(acc[2]);
  diag->t_min_C = r[1];
  diag->t_max_C = r[2];
  diag->steps = n_steps;
  if (r[3] > 0.0) return fail(RFA_ERR_NUMERIC, "%.0f non-finite voxels after step", r[3]);
  return RFA_OK;
}

// ---- allocation-free damage outputs -------------------------------------------
// Scratch of rfa_damage_noalloc in a file-scope device array: the per-class
// dead counters (32 x 8 bytes) and the staging of a host mask (up to
// kNoAllocMaskBytes voxels).  Each device holds its own copy for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a host
// stand-in, not a device address).
constexpr size_t kNoAllocCountBytes = 256;
constexpr size_t kNoAllocMaskBytes = size_t(16) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocCountBytes + kNoAllocMaskBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// with that device current.
rfa_status scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(RFA_ERR_ARG, "device %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    if (prev != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p)
      return fail(RFA_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_dev[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_dev[device]);
  return RFA_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

rfa_status rfa_damage_noalloc(rfa_grid g, uint8_t* mask, float* omega, double* dead_m3) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  const bool host_mask = mask && !g->opt.inputs_on_device;
  if (host_mask && n > kNoAllocMaskBytes)
    return fail(RFA_ERR_ARG, "a host mask of %zu voxels exceeds the %zu-byte scratch", n,
                kNoAllocMaskBytes);
  unsigned char* sp = nullptr;
  rfa_status s = scratch_ptr(g->device, &sp);
  if (s != RFA_OK) return s;
  auto* counts = reinterpret_cast<unsigned long long*>(sp);
  uint8_t* dmask = host_mask ? sp + kNoAllocCountBytes : mask;
  HIP_TRY(launch_zero_u64(counts, 2 * kMaxClasses, g->st));
  HIP_TRY(launch_damage(g->g, g->lab, g->om, dmask, counts, g->st));
  if (host_mask) HIP_TRY(hipMemcpyAsync(mask, dmask, n, hipMemcpyDeviceToHost, g->st));
  if (omega) HIP_TRY(hipMemcpyAsync(omega, g->om, n * sizeof(float), kind_out(g), g->st));
  unsigned long long cnt[2 * kMaxClasses] = {};
  if (dead_m3)
    HIP_TRY(hipMemcpyAsync(cnt, counts, sizeof cnt, hipMemcpyDeviceToHost, g->st));
  if (dead_m3 || host_mask || (omega && !g->opt.inputs_on_device))
    HIP_TRY(hipStreamSynchronize(g->st));
  if (dead_m3) {
    const double vol = g->dx * g->dy * g->dz;
    for (int c = 0; c < g->n_classes; ++c) {
      dead_m3[2 * c] = (double)cnt[2 * c] * vol;
      dead_m3[2 * c + 1] = (double)cnt[2 * c + 1] * vol;
    }
  }
  return RFA_OK;
}

rfa_status rfa_default_options(rfa_options* opt) {
  if (!opt) return fail(RFA_ERR_ARG, "opt is NULL");
  std::memset(opt, 0, sizeof *opt);
  opt->t_death = 60.0;
  opt->A = 7.39e39;
  opt->Ea = 2.577e5;
  opt->R = 8.314;
  opt->omega_cap = 1e30;
  opt->stream = nullptr;
  opt->inputs_on_device = 0;
  opt->depth = 0;
  opt->kernel = 0;
  opt->tile_y = 0;
  opt->tile_x = 0;
  opt->time_kernels = 0;
  opt->z_vec = 0;
  opt->store_policy = 0;
  return RFA_OK;
}

rfa_status rfa_create_grid(int nx, int ny, int nz, double dx, double dy, double dz,
                           const rfa_options* opt, rfa_grid* out) {
  if (!out) return fail(RFA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nx < 3 || ny < 3 || nz < 3) return fail(RFA_ERR_ARG, "grid must be at least 3^3");
  if ((double)nx * ny * nz > 4.0e9) return fail(RFA_ERR_ARG, "grid too large");
  if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
    return fail(RFA_ERR_ARG, "spacing must be finite and positive");
  rfa_options o;
  if (opt) {
    o = *opt;
  } else {
    rfa_default_options(&o);
  }
  if (!std::isfinite(o.t_death) || !(o.A >= 0.0) || !std::isfinite(o.A) || !(o.Ea >= 0.0) ||
      !std::isfinite(o.Ea) ||
      !finite_pos(o.R) || !finite_pos(o.omega_cap) || o.omega_cap > 3.0e38)
    return fail(RFA_ERR_ARG, "invalid damage options");
  if (o.depth < 0 || o.depth > kMaxDepth) return fail(RFA_ERR_ARG, "depth must be 0, 1 or 2");
  if (o.depth == 2 && (o.kernel == kStepNaive || o.tile_y == 4))
    return fail(RFA_ERR_ARG, "depth 2 needs the tiled kernel with tile_y 0, 8 or 16");
  if (o.kernel < 0 || o.kernel > 2) return fail(RFA_ERR_ARG, "kernel must be 0, 1 or 2");
  if (o.tile_y != 0 && o.tile_y != 4 && o.tile_y != 8 && o.tile_y != 16)
    return fail(RFA_ERR_ARG, "tile_y must be 0, 4, 8 or 16");
  if (o.tile_x < 0) return fail(RFA_ERR_ARG, "tile_x must be >= 0");
  if (o.z_vec != 0 && o.z_vec != 1 && o.z_vec != 2 && o.z_vec != 4)
    return fail(RFA_ERR_ARG, "z_vec must be 0, 1, 2 or 4");
  if (o.store_policy < 0 || o.store_policy > 3)
    return fail(RFA_ERR_ARG, "store_policy must be 0, 1, 2 or 3");
  if (o.time_kernels < 0 || o.time_kernels > kTimedBatch)
    return fail(RFA_ERR_ARG, "time_kernels must be in 0..%d", kTimedBatch);
  rfa_grid g = new (std::nothrow) rfa_grid_s();
  if (!g) return fail(RFA_ERR_OOM, "host allocation failed");
  g->g = Grid3{nx, ny, nz};
  g->dx = dx;
  g->dy = dy;
  g->dz = dz;
  g->opt = o;
  g->st = (hipStream_t)o.stream;
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return fail(RFA_ERR_HIP, "no HIP device");
  }
  const size_t n = g->g.n();
  g->plan = plan_default(g->g, o.kernel, o.depth, o.tile_y, o.tile_x, o.z_vec, o.store_policy);
  const size_t nwg = (size_t)plan_max_wg(g->g);
  g->partial_floats = nwg * 3 * kPartialSlots;
  g->red_doubles = 4 * 1024 + 64;
  rfa_status s = RFA_OK;
  if ((s = dmalloc(&g->cp_dev, 1)) || (s = dmalloc(&g->lab, n)) || (s = dmalloc(&g->hi[0], n)) ||
      (s = dmalloc(&g->hi[1], n)) || (s = dmalloc(&g->lo[0], n)) || (s = dmalloc(&g->lo[1], n)) ||
      (s = dmalloc(&g->om, n)) || (s = dmalloc(&g->src, n)) || (s = dmalloc(&g->q64, n)) ||
      (s = dmalloc(&g->tab_dev, 1)) || (s = dmalloc(&g->partials, g->partial_floats)) ||
      (s = dmalloc(&g->dacc, 4)) || (s = dmalloc(&g->red, g->red_doubles)) ||
      (s = dmalloc(&g->out4, 4)) || (s = dmalloc(&g->counts, 2 * kMaxClasses)) ||
      (s = dmalloc(&g->bad, 1))) {
    free_all(g);
    delete g;
    return s;
  }
  *out = g;
  return RFA_OK;
}

rfa_status rfa_set_tissue(rfa_grid g, const uint8_t* labels, const rfa_tissue* table,
                          int n_classes) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!labels || !table) return fail(RFA_ERR_ARG, "labels and table are required");
  if (n_classes < 1 || n_classes > kMaxClasses)
    return fail(RFA_ERR_ARG, "n_classes must be in 1..%d", kMaxClasses);
  for (int c = 0; c < n_classes; ++c) {
    const rfa_tissue& t = table[c];
    if (!(t.k >= 0.0) || !std::isfinite(t.k) || !finite_pos(t.rho) || !finite_pos(t.c) ||
        !(t.h_perf >= 0.0) || !std::isfinite(t.h_perf) || !std::isfinite(t.q_met) ||
        (t.fixed && !std::isfinite(t.t_fixed)) || (t.fixed != 0 && t.fixed != 1) ||
        (t.tissue != 0 && t.tissue != 1))
      return fail(RFA_ERR_ARG, "invalid parameters in class %d", c);
  }
  const size_t n = g->g.n();
  if (!g->opt.inputs_on_device) {
    for (size_t p = 0; p < n; ++p)
      if (labels[p] >= n_classes)
        return fail(RFA_ERR_ARG, "label %d at voxel %zu >= n_classes", labels[p], p);
  }
  ClassParams cp{};
  for (int c = 0; c < n_classes; ++c) {
    cp.k[c] = table[c].k;
    cp.rc[c] = table[c].rho * table[c].c;
    cp.h[c] = table[c].h_perf;
    cp.t_fixed[c] = table[c].t_fixed;
    cp.fixed[c] = table[c].fixed;
    cp.tissue[c] = table[c].tissue;
  }
  cp.n = n_classes;
  // Build the new label bytes into a fresh buffer so an invalid device label
  // image leaves the grid untouched.
  uint8_t* user = nullptr;
  uint8_t* nlab = nullptr;
  ClassParams* ncp = nullptr;
  rfa_status s;
  if ((s = dmalloc(&nlab, n)) != RFA_OK) return s;
  if ((s = dmalloc(&ncp, 1)) != RFA_OK) { (void)hipFree(nlab); return s; }
  if (!g->opt.inputs_on_device) {
    if ((s = dmalloc(&user, n)) != RFA_OK) { (void)hipFree(nlab); (void)hipFree(ncp); return s; }
  }
  unsigned bad = 0;
  hipError_t e = hipSuccess;
  do {
    if (user && (e = hipMemcpyAsync(user, labels, n, hipMemcpyHostToDevice, g->st)) != hipSuccess)
      break;
    if ((e = hipMemcpyAsync(ncp, &cp, sizeof cp, hipMemcpyHostToDevice, g->st)) != hipSuccess) break;
    if ((e = hipMemsetAsync(g->bad, 0, sizeof(unsigned), g->st)) != hipSuccess) break;
    if ((e = launch_build_labels(g->g, user ? user : labels, nlab, ncp, g->bad, g->st)) !=
        hipSuccess) break;
    if ((e = hipMemcpyAsync(&bad, g->bad, sizeof bad, hipMemcpyDeviceToHost, g->st)) != hipSuccess)
      break;
    if ((e = hipStreamSynchronize(g->st)) != hipSuccess) break;
  } while (false);
  if (user) (void)hipFree(user);
  if (e != hipSuccess || bad) {
    (void)hipFree(nlab);
    (void)hipFree(ncp);
    if (e != hipSuccess) return fail(RFA_ERR_HIP, "set_tissue failed: %s", hipGetErrorString(e));
    return fail(RFA_ERR_ARG, "%u labels >= n_classes", bad);
  }
  // commit
  (void)hipFree(g->lab);
  (void)hipFree(g->cp_dev);
  g->lab = nlab;
  g->cp_dev = ncp;
  g->cp = cp;
  g->n_classes = n_classes;
  std::memcpy(g->table, table, n_classes * sizeof(rfa_tissue));
  g->has_tissue = true;
  g->cur = 0;
  g->steps = 0;
  g->tab_dt = -1.0;
  g->src_dt = -1.0;
  g->energy_valid = false;
  HIP_TRY(launch_reset_state(g->g, g->lab, g->hi[0], g->lo[0], g->om, g->cp_dev,
                             (float)(g->opt.t_death - 37.0), g->st));
  HIP_TRY(hipMemsetAsync(g->counts, 0, 2 * kMaxClasses * sizeof(unsigned long long), g->st));
  HIP_TRY(launch_free_counts(g->g, g->lab, g->counts, g->st));
  HIP_TRY(hipMemcpyAsync(g->free_count, g->counts, kMaxClasses * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  if ((s = compute_dt_max(g)) != RFA_OK) return s;
  return rasterise(g);
}

rfa_status rfa_set_needle(rfa_grid g, const rfa_needle* nd) {
  if (!g || !nd) return fail(RFA_ERR_ARG, "grid and needle are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before set_needle");
  if (nd->n_tines < 0 || nd->n_tines > 4096) return fail(RFA_ERR_ARG, "n_tines out of range");
  if (nd->n_tines == 0) {
    g->has_needle = false;
    g->pt_offset.clear();
    g->pts.clear();
    g->power.clear();
    return rasterise(g);
  }
  if (!nd->pt_offset || !nd->pts || !nd->power) return fail(RFA_ERR_ARG, "needle arrays missing");
  if (!finite_pos(nd->sigma)) return fail(RFA_ERR_ARG, "sigma must be positive");
  if (nd->pt_offset[0] != 0) return fail(RFA_ERR_ARG, "pt_offset[0] must be 0");
  for (int t = 0; t < nd->n_tines; ++t) {
    if (nd->pt_offset[t + 1] - nd->pt_offset[t] < 2)
      return fail(RFA_ERR_ARG, "tine %d has fewer than 2 points", t);
    if (!(nd->power[t] >= 0.0) || !std::isfinite(nd->power[t]))
      return fail(RFA_ERR_ARG, "power of tine %d must be finite and >= 0", t);
  }
  const int np = nd->pt_offset[nd->n_tines];
  for (int i = 0; i < 3 * np; ++i)
    if (!std::isfinite(nd->pts[i])) return fail(RFA_ERR_ARG, "needle point not finite");
  // keep the previous needle to restore on failure
  auto old_off = g->pt_offset;
  auto old_pts = g->pts;
  auto old_pw = g->power;
  double old_sigma = g->sigma;
  bool old_has = g->has_needle;
  g->pt_offset.assign(nd->pt_offset, nd->pt_offset + nd->n_tines + 1);
  g->pts.assign(nd->pts, nd->pts + 3 * np);
  g->power.assign(nd->power, nd->power + nd->n_tines);
  g->sigma = nd->sigma;
  g->has_needle = true;
  rfa_status s = rasterise(g);
  if (s != RFA_OK) {
    std::string err = g_last_error;
    g->pt_offset = old_off;
    g->pts = old_pts;
    g->power = old_pw;
    g->sigma = old_sigma;
    g->has_needle = old_has;
    rasterise(g);
    g_last_error = err;
  }
  return s;
}

rfa_status rfa_set_perfusion(rfa_grid g, const float* factor) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before set_perfusion");
  const size_t n = g->g.n();
  ++g->version;
  g->bs_m = 0;  // a plain multiplier replaces any B-spline field
  if (!factor) {
    if (g->perf_decay) {
      rfa_status s = unit_perf(g);
      if (s != RFA_OK) return s;
      return compute_dt_max(g);
    }
    if (g->perf) (void)hipFree(g->perf);
    g->perf = nullptr;
    return compute_dt_max(g);
  }
  if (!g->opt.inputs_on_device) {
    for (size_t p = 0; p < n; ++p)
      if (!(factor[p] >= 0.0f) || !std::isfinite(factor[p]))
        return fail(RFA_ERR_ARG, "perfusion factor at voxel %zu is not finite and >= 0", p);
  }
  if (!g->perf) {
    rfa_status s = dmalloc(&g->perf, n);
    if (s != RFA_OK) return s;
  }
  HIP_TRY(hipMemcpyAsync(g->perf, factor, n * sizeof(float), kind_in(g), g->st));
  return compute_dt_max(g);
}

rfa_status rfa_set_perfusion_decay(rfa_grid g, int enable) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before set_perfusion_decay");
  if (enable != 0 && enable != 1) return fail(RFA_ERR_ARG, "enable must be 0 or 1");
  if (enable && !g->perf) {
    // the coupling is applied by the kernels that read a perfusion field
    rfa_status s = unit_perf(g);
    if (s != RFA_OK) return s;
  }
  if ((bool)enable != g->perf_decay) ++g->version;
  g->perf_decay = enable != 0;
  return RFA_OK;
}

rfa_status rfa_dt_max(rfa_grid g, double* dt_max) {
  if (!g || !dt_max) return fail(RFA_ERR_ARG, "grid and dt_max are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  *dt_max = g->dt_max;
  return RFA_OK;
}

rfa_status rfa_step(rfa_grid g, int n_steps, double dt, rfa_diag* diag) {
  Range range("rfa_step");
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before step");
  if (n_steps < 0) return fail(RFA_ERR_ARG, "n_steps must be >= 0");
  if (!finite_pos(dt)) return fail(RFA_ERR_ARG, "dt must be finite and positive");
  if (dt > g->dt_max)
    return fail(RFA_ERR_UNSTABLE, "dt %.6g s exceeds the stability bound %.6g s", dt, g->dt_max);
  rfa_status sp = prepare_dt(g, dt);
  if (sp != RFA_OK) return sp;
  const StepConst K = step_const(g, dt);
  double e0 = 0.0;
  if (diag) {
    if ((sp = ensure_energy(g)) != RFA_OK) return sp;
    e0 = g->energy;
    HIP_TRY(hipMemsetAsync(g->dacc, 0, 4 * sizeof(double), g->st));
  }
  rfa_status s = timed_steps(g, K, n_steps, diag != nullptr);
  if (s != RFA_OK) return s;
  if (n_steps > 0) {
    g->energy_valid = false;
    ++g->version;
  }
  if (diag) {
    double acc[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(acc, g->dacc, 3 * sizeof(double), hipMemcpyDeviceToHost, g->st));
    return finish_diag(g, acc, e0, dt, n_steps, diag);
  }
  return RFA_OK;
}

rfa_status rfa_damage(rfa_grid g, uint8_t* mask, float* omega, double* dead_m3) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  uint8_t* dmask = nullptr;
  if (mask) {
    if (g->opt.inputs_on_device) {
      dmask = mask;
    } else {
      rfa_status s = dmalloc(&dmask, n);
      if (s != RFA_OK) return s;
    }
  }
  hipError_t e = hipSuccess;
  unsigned long long cnt[2 * kMaxClasses] = {};
  // the mask kernel (which also counts) runs only for a mask or dead
  // volumes; only host outputs make the call synchronise
  const bool host_out = dead_m3 || ((mask || omega) && !g->opt.inputs_on_device);
  do {
    if (mask || dead_m3) {
      if ((e = hipMemsetAsync(g->counts, 0, sizeof cnt, g->st)) != hipSuccess) break;
      if ((e = launch_damage(g->g, g->lab, g->om, dmask, g->counts, g->st)) != hipSuccess) break;
    }
    if (mask && !g->opt.inputs_on_device &&
        (e = hipMemcpyAsync(mask, dmask, n, hipMemcpyDeviceToHost, g->st)) != hipSuccess) break;
    if (omega && (e = hipMemcpyAsync(omega, g->om, n * sizeof(float), kind_out(g), g->st)) !=
                     hipSuccess) break;
    if (dead_m3 && (e = hipMemcpyAsync(cnt, g->counts, sizeof cnt, hipMemcpyDeviceToHost,
                                       g->st)) != hipSuccess) break;
    if (host_out && (e = hipStreamSynchronize(g->st)) != hipSuccess) break;
  } while (false);
  if (dmask && dmask != mask) (void)hipFree(dmask);
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "damage failed: %s", hipGetErrorString(e));
  if (dead_m3) {
    const double vol = g->dx * g->dy * g->dz;
    for (int c = 0; c < g->n_classes; ++c) {
      dead_m3[2 * c] = (double)cnt[2 * c] * vol;
      dead_m3[2 * c + 1] = (double)cnt[2 * c + 1] * vol;
    }
  }
  return RFA_OK;
}

rfa_status rfa_get_temperature(rfa_grid g, double* t_C, float* hi, float* lo) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  if (t_C) {
    double* dt = nullptr;
    if (g->opt.inputs_on_device) {
      dt = t_C;
    } else {
      rfa_status s = dmalloc(&dt, n);
      if (s != RFA_OK) return s;
    }
    hipError_t e = launch_temperature_out(g->g, g->hi[g->cur], g->lo[g->cur], dt, g->st);
    if (e == hipSuccess && dt != t_C)
      e = hipMemcpyAsync(t_C, dt, n * sizeof(double), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (dt != t_C) (void)hipFree(dt);
    if (e != hipSuccess) return fail(RFA_ERR_HIP, "get_temperature: %s", hipGetErrorString(e));
  }
  if (hi) HIP_TRY(hipMemcpyAsync(hi, g->hi[g->cur], n * sizeof(float), kind_out(g), g->st));
  if (lo) HIP_TRY(hipMemcpyAsync(lo, g->lo[g->cur], n * sizeof(float), kind_out(g), g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  return RFA_OK;
}

rfa_status rfa_set_temperature(rfa_grid g, const double* t_C) {
  if (!g || !t_C) return fail(RFA_ERR_ARG, "grid and t_C are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  if (!g->opt.inputs_on_device) {
    for (size_t p = 0; p < n; ++p)
      if (!std::isfinite(t_C[p])) return fail(RFA_ERR_ARG, "temperature not finite at %zu", p);
  }
  const double* src = t_C;
  double* tmp = nullptr;
  if (!g->opt.inputs_on_device) {
    rfa_status s = dmalloc(&tmp, n);
    if (s != RFA_OK) return s;
    hipError_t e = hipMemcpyAsync(tmp, t_C, n * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return fail(RFA_ERR_HIP, "set_temperature: %s", hipGetErrorString(e));
    }
    src = tmp;
  }
  hipError_t e = launch_temperature_in(g->g, src, g->hi[g->cur], g->lo[g->cur], g->lab,
                                       (float)(g->opt.t_death - 37.0), g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "set_temperature: %s", hipGetErrorString(e));
  g->energy_valid = false;
  ++g->version;
  return RFA_OK;
}

namespace {

// Breathing view with one field (v2 == nullptr) or two.
rfa_status warp_impl(rfa_grid g, const float* v, double beta, const float* v2, double beta2,
                     float* out, double* kernel_ms) {
  if (!g || !v || !out) return fail(RFA_ERR_ARG, "grid, v and out are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  if (!std::isfinite(beta) || !std::isfinite(beta2)) return fail(RFA_ERR_ARG, "beta not finite");
  const size_t n = g->g.n();
  if (n >= (size_t(1) << 31)) return fail(RFA_ERR_ARG, "warp needs fewer than 2^31 voxels");
  const bool dev = g->opt.inputs_on_device != 0;
  const int nf = v2 ? 2 : 1;
  if (!dev) {
    for (int f = 0; f < nf; ++f) {
      const float* w = f ? v2 : v;
      for (size_t p = 0; p < 3 * n; ++p)
        if (!std::isfinite(w[p]))
          return fail(RFA_ERR_ARG, "displacement %d not finite at %zu", f + 1, p);
    }
  }
  // surrogate / spacing (FP64): s_a = scale_a * v_a in voxels
  const double scale[3] = {beta / g->dx, beta / g->dy, beta / g->dz};
  const double scale2[3] = {beta2 / g->dx, beta2 / g->dy, beta2 / g->dz};
  float* dv = const_cast<float*>(v);
  float* dv2 = const_cast<float*>(v2);
  float* dout = out;
  if (!dev) {
    rfa_status s = dmalloc(&dv, (size_t)nf * 3 * n);
    if (s != RFA_OK) return s;
    if ((s = dmalloc(&dout, n)) != RFA_OK) {
      (void)hipFree(dv);
      return s;
    }
    dv2 = v2 ? dv + 3 * n : nullptr;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  if (!dev) e = hipMemcpyAsync(dv, v, 3 * n * sizeof(float), hipMemcpyHostToDevice, g->st);
  if (e == hipSuccess && !dev && v2)
    e = hipMemcpyAsync(dv2, v2, 3 * n * sizeof(float), hipMemcpyHostToDevice, g->st);
  if (e == hipSuccess && kernel_ms) {
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], g->st);
  }
  if (e == hipSuccess)
    e = launch_warp(g->g, g->hi[g->cur], g->lo[g->cur], dv, scale, dv2, scale2, dout, g->st);
  if (e == hipSuccess && kernel_ms) e = hipEventRecord(ev[1], g->st);
  if (e == hipSuccess && !dev)
    e = hipMemcpyAsync(out, dout, n * sizeof(float), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess && (kernel_ms || !dev)) e = hipStreamSynchronize(g->st);
  if (e == hipSuccess && kernel_ms) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    *kernel_ms = ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (!dev) {
    (void)hipFree(dv);
    (void)hipFree(dout);
  }
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "warp: %s", hipGetErrorString(e));
  return RFA_OK;
}

}  // namespace

rfa_status rfa_warp(rfa_grid g, const float* v, double beta, float* out, double* kernel_ms) {
  Range range("rfa_warp");
  return warp_impl(g, v, beta, nullptr, 0.0, out, kernel_ms);
}

rfa_status rfa_warp2(rfa_grid g, const float* v1, double beta1, const float* v2, double beta2,
                     float* out, double* kernel_ms) {
  if (!v2) return fail(RFA_ERR_ARG, "v2 is required");
  return warp_impl(g, v1, beta1, v2, beta2, out, kernel_ms);
}

// ---- checkpoint ---------------------------------------------------------------
namespace {
struct StateHeader {
  char magic[8];
  uint32_t version;
  int32_t nx, ny, nz;
  int64_t steps;
  uint64_t payload;
  uint64_t checksum;
};

uint64_t fnv1a(const uint8_t* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}
}  // namespace

rfa_status rfa_save_state(rfa_grid g, void* buf, size_t* bytes) {
  if (!g || !bytes) return fail(RFA_ERR_ARG, "grid and bytes are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  const size_t payload = n * (4 + 4 + 4 + 1);
  const size_t need = sizeof(StateHeader) + payload;
  if (!buf) {
    *bytes = need;
    return RFA_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(RFA_ERR_ARG, "buffer too small (%zu bytes needed)", need);
  }
  uint8_t* out = (uint8_t*)buf;
  StateHeader h{};
  std::memcpy(h.magic, "RFASTAT1", 8);
  h.version = 1;
  h.nx = g->g.nx;
  h.ny = g->g.ny;
  h.nz = g->g.nz;
  h.steps = g->steps;
  h.payload = payload;
  uint8_t* p = out + sizeof h;
  HIP_TRY(hipMemcpyAsync(p, g->hi[g->cur], n * 4, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipMemcpyAsync(p + n * 4, g->lo[g->cur], n * 4, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipMemcpyAsync(p + n * 8, g->om, n * 4, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipMemcpyAsync(p + n * 12, g->lab, n, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  h.checksum = fnv1a(p, payload);
  std::memcpy(out, &h, sizeof h);
  *bytes = need;
  return RFA_OK;
}

rfa_status rfa_load_state(rfa_grid g, const void* buf, size_t bytes) {
  if (!g || !buf) return fail(RFA_ERR_ARG, "grid and buf are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  const size_t n = g->g.n();
  if (bytes < sizeof(StateHeader)) return fail(RFA_ERR_STATE, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, buf, sizeof h);
  const uint8_t* p = (const uint8_t*)buf + sizeof h;
  if (std::memcmp(h.magic, "RFASTAT1", 8) != 0 || h.version != 1)
    return fail(RFA_ERR_STATE, "not a state buffer");
  if (h.nx != g->g.nx || h.ny != g->g.ny || h.nz != g->g.nz || h.payload != n * 13 ||
      bytes < sizeof h + h.payload)
    return fail(RFA_ERR_STATE, "state buffer is for another grid shape");
  if (fnv1a(p, h.payload) != h.checksum) return fail(RFA_ERR_STATE, "state checksum mismatch");
  // class, tissue and held bits must agree with the current tissue (the
  // latch is state; the source flag follows the needle and is rebuilt)
  constexpr unsigned kFixedBits = kClassMask | kTissue | kHeld;
  std::vector<uint8_t> cur(n);
  HIP_TRY(hipMemcpyAsync(cur.data(), g->lab, n, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  for (size_t i = 0; i < n; ++i)
    if ((cur[i] & kFixedBits) != (p[n * 12 + i] & kFixedBits))
      return fail(RFA_ERR_STATE, "state buffer was saved with different tissue");
  g->cur = 0;
  HIP_TRY(hipMemcpyAsync(g->hi[0], p, n * 4, hipMemcpyHostToDevice, g->st));
  HIP_TRY(hipMemcpyAsync(g->lo[0], p + n * 4, n * 4, hipMemcpyHostToDevice, g->st));
  HIP_TRY(hipMemcpyAsync(g->om, p + n * 8, n * 4, hipMemcpyHostToDevice, g->st));
  HIP_TRY(hipMemcpyAsync(g->lab, p + n * 12, n, hipMemcpyHostToDevice, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  g->steps = h.steps;
  g->energy_valid = false;
  // the saved class bytes carry the source flags of the saving grid's
  // source: rebuild them with the increment before the next step
  g->src_dt = -1.0;
  ++g->version;
  return RFA_OK;
}

rfa_status rfa_get_step_count(rfa_grid g, long long* steps) {
  if (!g || !steps) return fail(RFA_ERR_ARG, "grid and steps are required");
  *steps = g->steps;
  return RFA_OK;
}

rfa_status rfa_adjoint_kernel_stats(rfa_grid g, double* kernel_ms, long long* launches) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (kernel_ms) *kernel_ms = g->adj_kernel_ms;
  if (launches) *launches = g->adj_kernel_launches;
  g->adj_kernel_ms = 0.0;
  g->adj_kernel_launches = 0;
  return RFA_OK;
}

rfa_status rfa_kernel_stats(rfa_grid g, double* kernel_ms, long long* launches,
                            long long* voxel_steps) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (kernel_ms) *kernel_ms = g->kernel_ms;
  if (launches) *launches = g->kernel_launches;
  if (voxel_steps) *voxel_steps = g->kernel_voxel_steps;
  g->kernel_ms = 0.0;
  g->kernel_launches = 0;
  g->kernel_voxel_steps = 0;
  return RFA_OK;
}

rfa_status rfa_source_support(rfa_grid g, long long* voxels) {
  if (!g || !voxels) return fail(RFA_ERR_ARG, "grid and voxels are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  if (g->src_dt <= 0.0)
    return fail(RFA_ERR_STATE, "the source increment is built by the first step after a "
                               "change of tissue, needle or time step");
  unsigned long long c = 0;
  HIP_TRY(hipMemsetAsync(g->counts, 0, sizeof c, g->st));
  HIP_TRY(launch_count_flag(g->g, g->lab, kSource, g->counts, g->st));
  HIP_TRY(hipMemcpyAsync(&c, g->counts, sizeof c, hipMemcpyDeviceToHost, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  *voxels = (long long)c;
  return RFA_OK;
}

rfa_status rfa_get_plan(rfa_grid g, int* kernel, int* depth, int* tile_y, int* tile_x,
                        int* workgroups, int* z_vec) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (kernel) *kernel = g->plan.kind;
  if (depth) *depth = g->plan.depth;
  if (tile_y) *tile_y = g->plan.ty;
  if (tile_x) *tile_x = g->plan.xc;
  if (workgroups) *workgroups = g->plan.nwg;
  if (z_vec) *z_vec = g->plan.zv;
  return RFA_OK;
}

namespace {
struct TuneKey {
  int nx, ny, nz, perf, one_step;
  bool operator==(const TuneKey& o) const {
    return nx == o.nx && ny == o.ny && nz == o.nz && perf == o.perf && one_step == o.one_step;
  }
};
std::vector<std::pair<TuneKey, StepPlan>> g_tuned;
}  // namespace

rfa_status rfa_tune(rfa_grid g, double dt, int reps) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before tune");
  if (!finite_pos(dt) || reps < 1) return fail(RFA_ERR_ARG, "dt > 0 and reps >= 1 required");
  if (dt > g->dt_max)
    return fail(RFA_ERR_UNSTABLE, "dt %.6g s exceeds the stability bound %.6g s", dt, g->dt_max);
  const TuneKey key{g->g.nx, g->g.ny, g->g.nz, g->perf ? 1 : 0, g->opt.depth == 1 ? 1 : 0};
  for (auto& kv : g_tuned)
    if (kv.first == key) {
      g->plan = kv.second;
      return RFA_OK;
    }
  if (dt != g->tab_dt) {
    build_tables(g, dt);
    HIP_TRY(hipMemcpyAsync(g->tab_dev, &g->tab_host, sizeof(Tables), hipMemcpyHostToDevice, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    g->tab_dt = dt;
  }
  if (dt != g->src_dt) {
    HIP_TRY(launch_source_increment(g->g, g->lab, g->q64, g->cp_dev, dt, g->src, g->st));
    g->src_dt = dt;
  }
  const size_t n = g->g.n();
  float* om2 = nullptr;
  uint8_t* lab2 = nullptr;
  rfa_status s;
  if ((s = dmalloc(&om2, n)) != RFA_OK) return s;
  if ((s = dmalloc(&lab2, n)) != RFA_OK) { (void)hipFree(om2); return s; }
  if ((s = ensure_events(g, 2)) != RFA_OK) { (void)hipFree(om2); (void)hipFree(lab2); return s; }
  StepPlan cand[64];
  const int nc = plan_candidates(g->g, g->opt.depth == 1 ? 1 : kMaxDepth, cand, 64);
  const StepConst K = step_const(g, dt);
  StepBuffers b;
  b.hi_in = g->hi[g->cur];
  b.lo_in = g->lo[g->cur];
  b.hi_out = g->hi[1 - g->cur];
  b.lo_out = g->lo[1 - g->cur];
  b.lab = lab2;
  b.src = g->src;
  b.omega = om2;
  b.perf = g->perf;
  b.tab = g->tab_dev;
  b.n_classes = g->n_classes;
  b.partials = g->partials;
  double best_ms = 1e300;
  StepPlan best = g->plan;
  hipError_t e = hipSuccess;
  if (g->opt.store_policy > 0)  // a requested store policy holds for every candidate
    for (int c = 0; c < nc; ++c) cand[c].store = g->opt.store_policy - 1;
  for (int c = 0; c < nc && e == hipSuccess; ++c) {
    if ((e = hipMemcpyAsync(om2, g->om, n * sizeof(float), hipMemcpyDeviceToDevice, g->st))) break;
    if ((e = hipMemcpyAsync(lab2, g->lab, n, hipMemcpyDeviceToDevice, g->st))) break;
    if ((e = launch_plan(g->g, cand[c], b, K, g->st))) break;  // warm-up
    if ((e = hipEventRecord(g->events[0], g->st))) break;
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_plan(g->g, cand[c], b, K, g->st);
    if (e) break;
    if ((e = hipEventRecord(g->events[1], g->st))) break;
    if ((e = hipEventSynchronize(g->events[1]))) break;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, g->events[0], g->events[1]))) break;
    ms /= (float)cand[c].depth;  // per step
    if (ms < best_ms) {
      best_ms = ms;
      best = cand[c];
    }
  }
  (void)hipStreamSynchronize(g->st);
  (void)hipFree(om2);
  (void)hipFree(lab2);
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "tune failed: %s", hipGetErrorString(e));
  g->plan = best;
  g_tuned.push_back({key, best});
  return RFA_OK;
}

rfa_status rfa_copy_bandwidth(size_t bytes, int reps, double* gbps) {
  if (!gbps || bytes < 4096 || reps < 1) return fail(RFA_ERR_ARG, "bytes >= 4096, reps >= 1");
  const size_t n4 = bytes / 2 / sizeof(float4);
  float4* a = nullptr;
  float4* b = nullptr;
  rfa_status s;
  if ((s = dmalloc(&a, n4)) != RFA_OK) return s;
  if ((s = dmalloc(&b, n4)) != RFA_OK) { (void)hipFree(a); return s; }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  float best_ms = 1e30f;
  // the plain copy at three launch widths (a grid-stride loop over 1024
  // work-groups streams best on MI355X) and the non-temporal x4 copy; the
  // fastest is the ceiling
  const int widths[3] = {1024, 4096, 16384};
  for (int variant = 0; variant < 4 && e == hipSuccess; ++variant) {
    auto launch = [&]() {
      return variant < 3 ? launch_copy(a, b, n4, widths[variant], nullptr)
                         : launch_copy_nt(a, b, n4, nullptr);
    };
    float ms = 0.f;
    do {
      if (!e0 && ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1)))) break;
      if ((e = hipMemsetAsync(a, 0, n4 * sizeof(float4), nullptr))) break;
      if ((e = launch())) break;
      if ((e = hipEventRecord(e0, nullptr))) break;
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
      if (e) break;
      if ((e = hipEventRecord(e1, nullptr)) || (e = hipEventSynchronize(e1))) break;
      e = hipEventElapsedTime(&ms, e0, e1);
    } while (false);
    if (e == hipSuccess) best_ms = std::min(best_ms, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "copy bandwidth: %s", hipGetErrorString(e));
  *gbps = 2.0 * n4 * sizeof(float4) * reps / (best_ms * 1e-3) / 1e9;
  return RFA_OK;
}

rfa_status rfa_mix_bandwidth(long long n_voxels, int reps, double* gbps) {
  if (!gbps || n_voxels < 4096 || reps < 1)
    return fail(RFA_ERR_ARG, "n_voxels >= 4096, reps >= 1");
  const size_t n4 = ((size_t)n_voxels + 3) / 4;
  float4* buf[6] = {};
  unsigned* lab = nullptr;
  rfa_status s = RFA_OK;
  for (int k = 0; k < 6 && s == RFA_OK; ++k) s = dmalloc(&buf[k], n4);
  if (s == RFA_OK) s = dmalloc(&lab, n4);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  float best_ms = 1e30f;
  if (s == RFA_OK) {
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
      e = hipMemsetAsync(buf[k], 0, n4 * sizeof(float4), nullptr);
    if (e == hipSuccess) e = hipMemsetAsync(lab, 0, n4 * sizeof(unsigned), nullptr);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const float4* const ping_in[3] = {buf[0], buf[1], buf[2]};
    float4* const ping_out[3] = {buf[3], buf[4], buf[5]};
    const float4* const pong_in[3] = {buf[3], buf[4], buf[5]};
    float4* const pong_out[3] = {buf[0], buf[1], buf[2]};
    // a few launch widths; the fastest is the ceiling.  Passes alternate
    // between the two image sets, as the stepper's do.
    for (int blocks : {1024, 2048, 4096, 8192, 16384}) {
      float ms = 0.f;
      if (e == hipSuccess) e = launch_stream_mix(ping_in, lab, ping_out, n4, blocks, nullptr);
      if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
      for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = (r & 1) ? launch_stream_mix(pong_in, lab, pong_out, n4, blocks, nullptr)
                    : launch_stream_mix(ping_in, lab, ping_out, n4, blocks, nullptr);
      if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) best_ms = std::min(best_ms, ms);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (float4* b : buf)
    if (b) (void)hipFree(b);
  if (lab) (void)hipFree(lab);
  if (s != RFA_OK) return s;
  if (e != hipSuccess) return fail(RFA_ERR_HIP, "mix bandwidth: %s", hipGetErrorString(e));
  *gbps = 25.0 * (double)(4 * n4) * reps / (best_ms * 1e-3) / 1e9;
  return RFA_OK;
}

// ---- differentiation ----------------------------------------------------------------
rfa_status rfa_set_perfusion_bspline(rfa_grid g, int m, const float* ctrl) {
  if (!g || !ctrl) return fail(RFA_ERR_ARG, "grid and ctrl are required");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before set_perfusion_bspline");
  if (m < 4 || m > 64) return fail(RFA_ERR_ARG, "m must be in 4..64");
  const size_t nc = (size_t)m * m * m;
  for (size_t j = 0; j < nc; ++j)
    if (!std::isfinite(ctrl[j]) || std::fabs(ctrl[j]) > 30.0f)
      return fail(RFA_ERR_ARG, "control value %zu not finite or |c| > 30", j);
  const int dims[3] = {g->g.nx, g->g.ny, g->g.nz};
  std::vector<int> vfirst(3 * (size_t)(m - 2), 0);
  for (int a = 0; a < 3; ++a) {
    const int n = dims[a];
    int* vf = &vfirst[(size_t)a * (m - 2)];
    // first voxel of knot span s (same span rule as the device kernels)
    for (int s = 0; s <= m - 3; ++s) vf[s] = n;
    for (int i = n - 1; i >= 0; --i) {
      const double u = n > 1 ? (double)i * (double)(m - 3) / (double)(n - 1) : 0.0;
      int s = (int)std::floor(u);
      s = std::min(std::max(s, 0), m - 4);
      for (int t = 0; t <= s; ++t) vf[t] = std::min(vf[t], i);
    }
    vf[m - 3] = n;
  }
  rfa_status s;
  if (g->bs_m != m) {
    if (g->bs_ctrl) (void)hipFree(g->bs_ctrl);
    if (g->bs_vfirst) (void)hipFree(g->bs_vfirst);
    g->bs_ctrl = nullptr;
    g->bs_vfirst = nullptr;
    g->bs_m = 0;
    if ((s = dmalloc(&g->bs_ctrl, nc)) != RFA_OK) return s;
    if ((s = dmalloc(&g->bs_vfirst, vfirst.size())) != RFA_OK) return s;
  }
  if (!g->perf && (s = dmalloc(&g->perf, g->g.n())) != RFA_OK) return s;
  HIP_TRY(hipMemcpyAsync(g->bs_ctrl, ctrl, nc * sizeof(float), hipMemcpyHostToDevice, g->st));
  HIP_TRY(hipMemcpyAsync(g->bs_vfirst, vfirst.data(), vfirst.size() * sizeof(int),
                         hipMemcpyHostToDevice, g->st));
  HIP_TRY(launch_bspline_eval(g->g, g->bs_ctrl, m, g->perf, g->st));
  HIP_TRY(hipStreamSynchronize(g->st));
  g->bs_m = m;
  ++g->version;
  return compute_dt_max(g);
}

rfa_status rfa_reset_state(rfa_grid g) {
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "no tissue");
  g->cur = 0;
  g->steps = 0;
  g->energy_valid = false;
  ++g->version;
  HIP_TRY(launch_reset_state(g->g, g->lab, g->hi[0], g->lo[0], g->om, g->cp_dev,
                             (float)(g->opt.t_death - 37.0), g->st));
  return RFA_OK;
}

rfa_status rfa_set_tine_powers(rfa_grid g, const double* power) {
  if (!g || !power) return fail(RFA_ERR_ARG, "grid and power are required");
  if (!g->has_needle) return fail(RFA_ERR_STATE, "no needle");
  const size_t nt = g->power.size();
  for (size_t t = 0; t < nt; ++t)
    if (!(power[t] >= 0.0) || !std::isfinite(power[t]))
      return fail(RFA_ERR_ARG, "power of tine %zu must be finite and >= 0", t);
  if (g->fields_ok) {
    // recombine the kept per-tine densities with the new powers
    std::vector<double> scale(nt);
    for (size_t t = 0; t < nt; ++t) scale[t] = power[t] / g->tine_sums[t];
    rfa_status s;
    if (g->scale_cap < nt) {
      if (g->scale_dev) (void)hipFree(g->scale_dev);
      g->scale_dev = nullptr;
      g->scale_cap = 0;
      if ((s = dmalloc(&g->scale_dev, nt)) != RFA_OK) return s;
      g->scale_cap = nt;
    }
    HIP_TRY(hipMemcpyAsync(g->scale_dev, scale.data(), nt * sizeof(double),
                           hipMemcpyHostToDevice, g->st));
    HIP_TRY(launch_source_combine(g->g, g->lab, g->tine_u, (int)nt, g->scale_dev, g->q64, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    g->power.assign(power, power + nt);
    g->src_dt = -1.0;
    ++g->version;
    double tot = 0.0;
    for (double p : g->power) tot += p;
    g->rf_power = tot;
    return RFA_OK;
  }
  std::vector<double> old = g->power;
  g->power.assign(power, power + nt);
  rfa_status s = rasterise(g);
  if (s != RFA_OK) {
    std::string err = g_last_error;
    g->power = old;
    rasterise(g);
    g_last_error = err;
  }
  return s;
}

rfa_status rfa_forward_checkpointed(rfa_grid g, int n_steps, double dt, int ckpt_every) {
  Range range("rfa_forward_checkpointed");
  if (!g) return fail(RFA_ERR_ARG, "grid is NULL");
  if (!g->has_tissue) return fail(RFA_ERR_STATE, "set_tissue before forward");
  if (n_steps < 1 || ckpt_every < 0) return fail(RFA_ERR_ARG, "n_steps >= 1, ckpt_every >= 0");
  if (!finite_pos(dt)) return fail(RFA_ERR_ARG, "dt must be finite and positive");
  if (dt > g->dt_max)
    return fail(RFA_ERR_UNSTABLE, "dt %.6g s exceeds the stability bound %.6g s", dt, g->dt_max);
  rfa_status s = prepare_dt(g, dt);
  if (s != RFA_OK) return s;
  const size_t n = g->g.n();
  if (ckpt_every == 0) {
    // the whole hi trajectory, written by the steps themselves
    const size_t need = (size_t)(n_steps + 1) * n;
    if (g->traj_floats < need) {
      if (g->traj) (void)hipFree(g->traj);
      g->traj = nullptr;
      g->traj_floats = 0;
      if ((s = dmalloc(&g->traj, need)) != RFA_OK) return s;
      g->traj_floats = need;
    }
    g->adj_ready = false;
    const StepConst K = step_const(g, dt);
    HIP_TRY(hipMemcpyAsync(g->traj, g->hi[g->cur], n * sizeof(float), hipMemcpyDeviceToDevice,
                           g->st));
    int t = 0;
    if ((s = timed_steps(g, K, n_steps, false, g->traj, &t)) != RFA_OK) return s;
    HIP_TRY(hipMemcpyAsync(g->hi[g->cur], g->traj + (size_t)n_steps * n, n * sizeof(float),
                           hipMemcpyDeviceToDevice, g->st));
    g->energy_valid = false;
    ++g->version;
    g->adj_ready = true;
    g->adj_version = g->version;
    g->adj_steps = n_steps;
    g->adj_every = 0;
    g->adj_nckpt = 0;
    g->adj_tail_kept = false;
    g->adj_dt = dt;
    return RFA_OK;
  }
  const int every = std::min(ckpt_every, n_steps);
  const int nck = (n_steps + every - 1) / every;
  const size_t need = (size_t)nck * 2 * n;
  if (g->ckpt_floats < need) {
    if (g->ckpt) (void)hipFree(g->ckpt);
    g->ckpt = nullptr;
    g->ckpt_floats = 0;
    if ((s = dmalloc(&g->ckpt, need)) != RFA_OK) return s;
    g->ckpt_floats = need;
  }
  // the adjoint's two segment buffers; the last segment's hi images go
  // straight into its buffer, so the adjoint starts without a recompute
  const size_t seg_floats = (size_t)(every + 1) * n;
  if (g->traj_floats < 2 * seg_floats) {
    if (g->traj) (void)hipFree(g->traj);
    g->traj = nullptr;
    g->traj_floats = 0;
    if ((s = dmalloc(&g->traj, 2 * seg_floats)) != RFA_OK) return s;
    g->traj_floats = 2 * seg_floats;
  }
  g->adj_ready = false;
  g->adj_tail_kept = false;
  const StepConst K = step_const(g, dt);
  for (int seg = 0; seg < nck; ++seg) {
    float* c = g->ckpt + (size_t)seg * 2 * n;
    HIP_TRY(hipMemcpyAsync(c, g->hi[g->cur], n * sizeof(float), hipMemcpyDeviceToDevice, g->st));
    HIP_TRY(hipMemcpyAsync(c + n, g->lo[g->cur], n * sizeof(float), hipMemcpyDeviceToDevice,
                           g->st));
    const int k = std::min(every, n_steps - seg * every);
    if (seg < nck - 1) {
      if ((s = timed_steps(g, K, k, false)) != RFA_OK) return s;
      continue;
    }
    float* traj = g->traj + (size_t)(seg & 1) * seg_floats;
    HIP_TRY(hipMemcpyAsync(traj, g->hi[g->cur], n * sizeof(float), hipMemcpyDeviceToDevice,
                           g->st));
    int t = 0;
    if ((s = timed_steps(g, K, k, false, traj, &t)) != RFA_OK) return s;
    HIP_TRY(hipMemcpyAsync(g->hi[g->cur], traj + (size_t)k * n, n * sizeof(float),
                           hipMemcpyDeviceToDevice, g->st));
  }
  g->adj_tail_kept = true;
  g->energy_valid = false;
  ++g->version;
  g->adj_ready = true;
  g->adj_version = g->version;
  g->adj_steps = n_steps;
  g->adj_every = every;
  g->adj_nckpt = nck;
  g->adj_dt = dt;
  return RFA_OK;
}

rfa_status rfa_adjoint(rfa_grid g, const float* w_omega, double* dL_dP, double* dL_dctrl,
                       float* dL_dperf) {
  Range range("rfa_adjoint");
  if (!g || !w_omega) return fail(RFA_ERR_ARG, "grid and w_omega are required");
  if (g->perf_decay)
    return fail(RFA_ERR_ARG, "no adjoint for damage-coupled perfusion (the step is then "
                             "nonlinear in the damage integral)");
  if (!g->adj_ready || g->version != g->adj_version)
    return fail(RFA_ERR_STATE, "no checkpointed forward for the current state");
  if (dL_dctrl && !g->bs_m) return fail(RFA_ERR_STATE, "no B-spline perfusion field");
  if (dL_dP && !g->has_needle) return fail(RFA_ERR_STATE, "no needle");
  const size_t n = g->g.n();
  const int every = g->adj_every;  // 0: the forward kept the whole trajectory
  rfa_status s;
  // two halves of (every + 1) hi images: segment seg is recomputed into
  // half seg & 1 while the adjoint steps read the other half
  const size_t seg_floats = (size_t)(every + 1) * n;
  const size_t tneed = 2 * seg_floats;
  if (every > 0 && g->traj_floats < tneed) {
    if (g->traj) (void)hipFree(g->traj);
    g->traj = nullptr;
    g->traj_floats = 0;
    g->adj_tail_kept = false;
    if ((s = dmalloc(&g->traj, tneed)) != RFA_OK) return s;
    g->traj_floats = tneed;
  }
  if (!g->adj_work && (s = dmalloc(&g->adj_work, 8 * n)) != RFA_OK) return s;
  if (!g->lab_scratch && (s = dmalloc(&g->lab_scratch, n)) != RFA_OK) return s;
  float* lopp[2] = {g->adj_work, g->adj_work + n};
  float* lam[2] = {g->adj_work + 2 * n, g->adj_work + 3 * n};
  float* sacc = g->adj_work + 4 * n;
  float* facc = g->adj_work + 5 * n;
  float* wv = g->adj_work + 6 * n;
  float* om_s = g->adj_work + 7 * n;
  HIP_TRY(hipMemcpyAsync(wv, w_omega, n * sizeof(float), kind_in(g), g->st));
  HIP_TRY(launch_adjoint_weight(g->g, wv, g->om, g->lab, (float)g->opt.omega_cap, wv, g->st));
  HIP_TRY(hipMemsetAsync(g->adj_work + 2 * n, 0, 4 * n * sizeof(float), g->st));
  // the recompute's damage integral is never read back, but the step kernels
  // take it as an input: keep it finite
  HIP_TRY(hipMemsetAsync(om_s, 0, n * sizeof(float), g->st));
  HIP_TRY(hipMemcpyAsync(g->lab_scratch, g->lab, n, hipMemcpyDeviceToDevice, g->st));
  if ((s = prepare_dt(g, g->adj_dt)) != RFA_OK) return s;
  const StepConst K = step_const(g, g->adj_dt);
  // adjoint schedule: the tiled kernel (8 rows, x chunks sized for about
  // one work-group per compute unit; at 128^3: 256 work-groups of 16 planes,
  // 8 % faster than 1024 work-groups of 4 rows x 8 planes) unless the grid
  // asked for the reference kernels.  Beside the segment recomputes (which
  // leave each compute unit fewer free cycles) two work-groups per compute
  // unit of half the length finish sooner: 512 work-groups of 8 planes at
  // 128^3 (the recompute-and-adjoint phase 5 % shorter; alone both widths
  // take the same time)
  constexpr int adj_ty = 8;
  int adj_xc = 4;
  {
    const int target = every > 0 ? 512 : 256;
    const int tiles = ((g->g.nz + 63) / 64) * ((g->g.ny + adj_ty - 1) / adj_ty);
    const int chunks = std::max(1, (target + tiles - 1) / tiles);
    adj_xc = std::min(g->g.nx, std::max(4, (g->g.nx + chunks - 1) / chunks));
  }
  const bool tiled_adj = g->plan.kind != kStepNaive && adjoint_tiled_fits(g->g, adj_xc);
  int lc = 0;
  // Lambda is accumulated on the flagged source support, unless a tine has
  // zero power (its density then reaches voxels whose increment is 0)
  bool sacc_all = false;
  for (double p : g->power) sacc_all = sacc_all || !(p > 0.0);
  // adjoint step from theta^t = traj[t]
  auto adjoint_step = [&](const float* theta) {
    AdjointBuffers a;
    a.lam_in = lam[lc];
    a.lam_out = lam[1 - lc];
    a.theta = theta;
    a.lab = g->lab;
    a.perf = g->perf;
    a.w = wv;
    a.tab = g->tab_dev;
    a.sacc = sacc;
    a.facc = facc;
    a.sacc_all = sacc_all;
    lc = 1 - lc;
    return tiled_adj ? launch_adjoint_tiled(g->g, adj_ty, adj_xc, a, K, g->st)
                     : launch_adjoint_step(g->g, a, K, g->st);
  };
  if (every == 0) {  // the forward kept every theta^t: no recomputation
    // with time_kernels, one event pair brackets the back-to-back launches
    const bool timed = g->opt.time_kernels != 0 && g->adj_steps > 0;
    if (timed) {
      if ((s = ensure_events(g, 2)) != RFA_OK) return s;
      HIP_TRY(hipEventRecord(g->events[0], g->st));
    }
    for (int t = g->adj_steps - 1; t >= 0; --t)
      HIP_TRY(adjoint_step(g->traj + (size_t)t * n));
    if (timed) {
      float ms = 0.0f;
      HIP_TRY(hipEventRecord(g->events[1], g->st));
      HIP_TRY(hipEventSynchronize(g->events[1]));
      HIP_TRY(hipEventElapsedTime(&ms, g->events[0], g->events[1]));
      g->adj_kernel_ms += ms;
      g->adj_kernel_launches += g->adj_steps;
    }
  }
  // Checkpointed: segments from the last one back.  The recompute of a
  // segment (from its checkpoint, bitwise as the forward) runs on the side
  // stream into one half of traj while the adjoint steps of the later
  // segment read the other half on the grid's stream; events order each
  // half's reuse.  The recompute reproduces only the temperature (the
  // adjoint refuses damage-coupled perfusion, so nothing else feeds it): it
  // writes traj and the lo ping-pong, and with kernels other than the wide
  // one also the scratch class bytes and damage integral, none of which the
  // adjoint reads.
  if (every > 0) {
    if ((s = ensure_side_stream(g)) != RFA_OK) return s;
    hipEvent_t start = g->side_ev[0];
    hipEvent_t ready[2] = {g->side_ev[1], g->side_ev[2]};
    hipEvent_t read[2] = {g->side_ev[3], g->side_ev[4]};
    bool used[2] = {false, false};
    HIP_TRY(hipEventRecord(start, g->st));
    HIP_TRY(hipStreamWaitEvent(g->side, start, 0));
    for (int seg = g->adj_nckpt - 1; seg >= 0; --seg) {
      const int k = std::min(every, g->adj_steps - seg * every);
      const int half = seg & 1;
      float* traj = g->traj + (size_t)half * seg_floats;
      const float* c = g->ckpt + (size_t)seg * 2 * n;
      if (seg == g->adj_nckpt - 1 && g->adj_tail_kept) {
        // written by the forward itself: no recompute
        for (int t = k - 1; t >= 0; --t) HIP_TRY(adjoint_step(traj + (size_t)t * n));
        HIP_TRY(hipEventRecord(read[half], g->st));
        used[half] = true;
        continue;
      }
      if (used[half]) HIP_TRY(hipStreamWaitEvent(g->side, read[half], 0));
      HIP_TRY(hipMemcpyAsync(traj, c, n * sizeof(float), hipMemcpyDeviceToDevice, g->side));
      HIP_TRY(
          hipMemcpyAsync(lopp[0], c + n, n * sizeof(float), hipMemcpyDeviceToDevice, g->side));
      for (int t = 0; t < k; ++t) {
        StepBuffers b;
        b.hi_in = traj + (size_t)t * n;
        b.lo_in = lopp[t & 1];
        b.hi_out = traj + (size_t)(t + 1) * n;
        b.lo_out = lopp[(t + 1) & 1];
        b.lab = g->lab_scratch;
        b.src = g->src;
        b.omega = om_s;
        b.perf = g->perf;
        b.tab = g->tab_dev;
        b.partials = nullptr;
        b.n_classes = g->n_classes;
        HIP_TRY(launch_plan_temperature(g->g, plan_one(g->plan), b, K, g->side));
      }
      HIP_TRY(hipEventRecord(ready[half], g->side));
      HIP_TRY(hipStreamWaitEvent(g->st, ready[half], 0));
      for (int t = k - 1; t >= 0; --t) HIP_TRY(adjoint_step(traj + (size_t)t * n));
      HIP_TRY(hipEventRecord(read[half], g->st));
      used[half] = true;
    }
    // later segments may have overwritten the kept one: a second adjoint
    // of this forward recomputes every segment
    g->adj_tail_kept = false;
  }
  if (dL_dP) {
    const int nt = (int)g->power.size();
    constexpr int kBlk = 512;
    double* part = nullptr;
    if ((s = dmalloc(&part, (size_t)nt * kBlk)) != RFA_OK) return s;
    std::vector<double> host((size_t)nt * kBlk);
    hipError_t e = g->fields_ok
                       ? launch_source_dot_fields(g->g, g->lab, g->tine_u, nt, sacc, g->cp_dev,
                                                  g->adj_dt, part, kBlk, g->st)
                       : launch_source_dot(g->g, g->dx, g->dy, g->dz, g->lab, g->chords_dev,
                                           g->first_dev, nt, g->sigma, sacc, g->cp_dev,
                                           g->adj_dt, part, kBlk, g->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(host.data(), part, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                         g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(RFA_ERR_HIP, "adjoint dL/dP: %s", hipGetErrorString(e));
    for (int t = 0; t < nt; ++t) {
      double acc = 0.0;
      for (int b = 0; b < kBlk; ++b) acc += host[(size_t)t * kBlk + b];
      dL_dP[t] = acc / g->tine_sums[t];
    }
  }
  if (dL_dperf)
    HIP_TRY(hipMemcpyAsync(dL_dperf, facc, n * sizeof(float), kind_out(g), g->st));
  if (dL_dctrl) {
    const int m = g->bs_m;
    const size_t nc = (size_t)m * m * m;
    double* gc = nullptr;
    if ((s = dmalloc(&gc, nc + bspline_grad_scratch(g->g, m))) != RFA_OK) return s;
    hipError_t e = launch_bspline_grad(g->g, facc, g->perf, m, g->bs_vfirst,
                                       g->bs_vfirst + (m - 2), g->bs_vfirst + 2 * (m - 2),
                                       gc + nc, gc, g->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dL_dctrl, gc, nc * sizeof(double), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    (void)hipFree(gc);
    if (e != hipSuccess) return fail(RFA_ERR_HIP, "adjoint dL/dctrl: %s", hipGetErrorString(e));
  }
  HIP_TRY(hipStreamSynchronize(g->st));
  return RFA_OK;
}

// ---- batches ---------------------------------------------------------------------
}  // extern "C"

struct rfa_batch_s {
  std::vector<rfa_grid> grids;
  std::vector<double> dt;
  std::vector<BatchInstance> inst;  // host copy of the descriptor table
  std::vector<int> first;           // item range of each instance
  BatchInstance* inst_dev = nullptr;
  BatchItem* items_dev = nullptr;
  int* first_dev = nullptr;
  float* partials = nullptr;        // [kPartialSlots][n_items][3]
  double* dacc = nullptr;           // [n][3]
  double* slot_acc = nullptr;       // [n][kPartialSlots][3] reduction scratch
  int n_items = 0;
  int ty = 4;
  int xc = 8;
  bool flat = false;                // items are flat plane segments (else 2.5-D tiles)
  int n_wg = 0;
  int req_wg = 0;                   // persistent work-groups (0: one per item)
  long long group_budget = kBatchGroupVoxels;  // voxels per group (0: one group)
  struct Group {
    int inst0, inst1;               // instances [inst0, inst1)
    int plain0, plain1;             // items of its grids without a perfusion field
    int perf0, perf1;               // items of its grids with one
  };
  std::vector<Group> groups;
  int parity = 0;
  long long voxels = 0;
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  long long last_vs = 0;
  struct Cached {
    int n_steps, parity, diag;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Cached> graphs;
};

namespace {


void batch_free_device(rfa_batch b) {
  for (auto& c : b->graphs) {
    (void)hipGraphExecDestroy(c.exec);
    (void)hipGraphDestroy(c.graph);
  }
  b->graphs.clear();
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(b->inst_dev);
  f(b->items_dev);
  f(b->first_dev);
  f(b->partials);
  f(b->dacc);
  f(b->slot_acc);
  b->inst_dev = nullptr;
  b->items_dev = nullptr;
  b->first_dev = nullptr;
  b->partials = nullptr;
  b->dacc = nullptr;
  b->slot_acc = nullptr;
}

// (Re)build the device descriptor table and work list from the grids'
// current state; resets the batch parity and drops cached graphs.
rfa_status batch_build(rfa_batch b) {
  batch_free_device(b);
  const int n = (int)b->grids.size();
  b->inst.assign(n, BatchInstance{});
  b->first.assign(2 * (size_t)n, 0);
  std::vector<BatchItem> items;
  b->voxels = 0;
  for (int i = 0; i < n; ++i) {
    rfa_grid g = b->grids[i];
    rfa_status s = prepare_dt(g, b->dt[i]);
    if (s != RFA_OK) return s;
    HIP_TRY(hipStreamSynchronize(g->st));
    BatchInstance& I = b->inst[i];
    I.hi[0] = g->hi[g->cur];
    I.hi[1] = g->hi[1 - g->cur];
    I.lo[0] = g->lo[g->cur];
    I.lo[1] = g->lo[1 - g->cur];
    I.lab = g->lab;
    I.src = g->src;
    I.om = g->om;
    I.perf = g->perf;
    I.tab = g->tab_dev;
    I.K = step_const(g, b->dt[i]);
    I.n_classes = g->n_classes;
    I.nx = g->g.nx;
    I.ny = g->g.ny;
    I.nz = g->g.nz;
    I.xc = std::min(b->xc, g->g.nx);
    if (!tiled_fits(g->g, I.xc)) return fail(RFA_ERR_ARG, "grid %d too large for a batch", i);
    if (b->flat && g->g.nz > flat_max_nz(b->ty))
      return fail(RFA_ERR_ARG, "grid %d: nz = %d exceeds %d for flat items of %d waves", i,
                  g->g.nz, flat_max_nz(b->ty), b->ty);
    b->voxels += (long long)g->g.n();
  }
  // Groups of consecutive grids up to the voxel budget; a group runs all its
  // steps before the next starts (the grids are independent), so its
  // working set stays in the last-level cache.  Work items of a group:
  // grids without a perfusion field first, then those with one (two kernel
  // variants); each grid's items are contiguous.
  b->groups.clear();
  for (int i0 = 0; i0 < n;) {
    int i1 = i0 + 1;
    long long vox = (long long)b->grids[i0]->g.n();
    while (i1 < n && b->group_budget > 0 &&
           vox + (long long)b->grids[i1]->g.n() <= b->group_budget)
      vox += (long long)b->grids[i1++]->g.n();
    if (b->group_budget == 0) i1 = n;
    rfa_batch_s::Group G{i0, i1, 0, 0, 0, 0};
    for (int pass = 0; pass < 2; ++pass) {
      (pass == 0 ? G.plain0 : G.perf0) = (int)items.size();
      for (int i = i0; i < i1; ++i) {
        const BatchInstance& I = b->inst[i];
        if ((I.perf != nullptr) != (pass == 1)) continue;
        const TiledShape sh = b->flat ? flat_shape(b->grids[i]->g, b->ty, I.xc)
                                      : tiled_shape(b->grids[i]->g, b->ty, I.xc);
        b->first[2 * i] = (int)items.size();
        for (int tx = 0; tx < sh.chunks_x; ++tx)
          for (int ty = 0; ty < sh.tiles_y; ++ty)
            for (int tz = 0; tz < sh.tiles_z; ++tz) items.push_back(BatchItem{i, tz, ty, tx});
        b->first[2 * i + 1] = (int)items.size();
      }
      (pass == 0 ? G.plain1 : G.perf1) = (int)items.size();
    }
    b->groups.push_back(G);
    i0 = i1;
  }
  b->n_items = (int)items.size();
  rfa_status s;
  if ((s = dmalloc(&b->inst_dev, n)) || (s = dmalloc(&b->items_dev, items.size())) ||
      (s = dmalloc(&b->first_dev, 2 * (size_t)n)) ||
      (s = dmalloc(&b->partials, (size_t)kPartialSlots * b->n_items * 3)) ||
      (s = dmalloc(&b->dacc, 3 * (size_t)n)) ||
      (s = dmalloc(&b->slot_acc, (size_t)kPartialSlots * 3 * n)))
    return s;
  HIP_TRY(hipMemcpyAsync(b->inst_dev, b->inst.data(), n * sizeof(BatchInstance),
                         hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipMemcpyAsync(b->items_dev, items.data(), items.size() * sizeof(BatchItem),
                         hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipMemcpyAsync(b->first_dev, b->first.data(), 2 * (size_t)n * sizeof(int),
                         hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipStreamSynchronize(b->st));
  // persistent work-groups if requested, else one work-group per work item
  b->n_wg = b->req_wg > 0 ? std::min(b->req_wg, b->n_items) : 0;
  b->parity = 0;
  return RFA_OK;
}

// Whether the grids still match the descriptor table (nobody stepped or
// re-tissued a grid outside the batch, no dt change).
bool batch_in_sync(rfa_batch b) {
  for (size_t i = 0; i < b->grids.size(); ++i) {
    rfa_grid g = b->grids[i];
    const BatchInstance& I = b->inst[i];
    if (!g->has_tissue || I.hi[b->parity] != g->hi[g->cur] || I.lab != g->lab ||
        I.src != g->src || I.om != g->om || I.perf != g->perf || I.tab != g->tab_dev ||
        I.n_classes != g->n_classes || g->tab_dt != b->dt[i] || g->src_dt != b->dt[i])
      return false;
  }
  return true;
}

rfa_status batch_graph(rfa_batch b, int n_steps, bool diag, hipGraphExec_t* out) {
  for (auto& c : b->graphs)
    if (c.n_steps == n_steps && c.parity == b->parity && c.diag == (int)diag) {
      *out = c.exec;
      return RFA_OK;
    }
  if (b->graphs.size() >= 4) {
    (void)hipGraphExecDestroy(b->graphs.front().exec);
    (void)hipGraphDestroy(b->graphs.front().graph);
    b->graphs.erase(b->graphs.begin());
  }
  HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (const auto& G : b->groups) {
    // every step of this group's grids, then the next group
    const int n_plain = G.plain1 - G.plain0, n_perf = G.perf1 - G.perf0;
    const int wg_plain = b->n_wg > 0 ? std::min(b->n_wg, n_plain) : 0;
    const int wg_perf = b->n_wg > 0 ? std::min(b->n_wg, n_perf) : 0;
    int pending = 0;
    for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
      float* part = diag ? b->partials + (size_t)pending * b->n_items * 3 : nullptr;
      const int par = (b->parity + s) & 1;
      e = launch_step_batch(b->ty, b->flat, false, b->inst_dev, b->items_dev, G.plain0,
                            n_plain, wg_plain, par, part, b->st);
      if (e == hipSuccess)
        e = launch_step_batch(b->ty, b->flat, true, b->inst_dev, b->items_dev, G.perf0, n_perf,
                              wg_perf, par, part, b->st);
      if (e == hipSuccess && diag && ++pending == kPartialSlots) {
        e = launch_reduce_batch(b->partials, pending, b->n_items, b->first_dev, G.inst0,
                                G.inst1 - G.inst0, b->slot_acc, kPartialSlots, b->dacc,
                                b->st);
        pending = 0;
      }
    }
    if (e == hipSuccess && diag && pending > 0)
      e = launch_reduce_batch(b->partials, pending, b->n_items, b->first_dev, G.inst0,
                              G.inst1 - G.inst0, b->slot_acc, kPartialSlots, b->dacc, b->st);
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->st, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(RFA_ERR_HIP, "batch graph capture failed: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(RFA_ERR_HIP, "batch graph instantiate failed: %s", hipGetErrorString(e));
  }
  b->graphs.push_back(rfa_batch_s::Cached{n_steps, b->parity, (int)diag, graph, exec});
  *out = exec;
  return RFA_OK;
}

}  // namespace

extern "C" {

rfa_status rfa_batch_create(int n, const rfa_grid* grids, const double* dt, rfa_batch* out) {
  if (!out) return fail(RFA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || !grids || !dt) return fail(RFA_ERR_ARG, "n >= 1 grids and dt required");
  for (int i = 0; i < n; ++i) {
    if (!grids[i] || !grids[i]->has_tissue)
      return fail(RFA_ERR_STATE, "grid %d has no tissue", i);
    if (!finite_pos(dt[i])) return fail(RFA_ERR_ARG, "dt[%d] must be finite and positive", i);
    if (dt[i] > grids[i]->dt_max)
      return fail(RFA_ERR_UNSTABLE, "dt[%d] = %.6g s exceeds the stability bound %.6g s", i,
                  dt[i], grids[i]->dt_max);
    if (grids[i]->device != grids[0]->device)
      return fail(RFA_ERR_ARG, "all grids of a batch must be on one device");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(RFA_ERR_ARG, "grid %d appears twice", i);
  }
  rfa_batch b = new (std::nothrow) rfa_batch_s();
  if (!b) return fail(RFA_ERR_OOM, "host allocation failed");
  b->grids.assign(grids, grids + n);
  b->dt.assign(dt, dt + n);
  // default layout: flat plane segments of 8 waves (no lanes lost to rows
  // shorter than a multiple of 64) where every grid allows them
  b->flat = true;
  for (int i = 0; i < n; ++i) b->flat = b->flat && grids[i]->g.nz <= flat_max_nz(8);
  b->ty = b->flat ? 8 : 4;
  hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e != hipSuccess) {
    rfa_batch_destroy(b);
    return fail(RFA_ERR_HIP, "batch stream: %s", hipGetErrorString(e));
  }
  rfa_status s = batch_build(b);
  if (s != RFA_OK) {
    std::string err = g_last_error;
    rfa_batch_destroy(b);
    g_last_error = err;
    return s;
  }
  *out = b;
  return RFA_OK;
}

rfa_status rfa_batch_step(rfa_batch b, int n_steps, rfa_diag* diags) {
  Range range("rfa_batch_step");
  if (!b) return fail(RFA_ERR_ARG, "batch is NULL");
  if (n_steps < 0) return fail(RFA_ERR_ARG, "n_steps must be >= 0");
  if (n_steps == 0) return RFA_OK;
  const int n = (int)b->grids.size();
  for (int i = 0; i < n; ++i) {
    rfa_grid g = b->grids[i];
    if (!g->has_tissue) return fail(RFA_ERR_STATE, "grid %d lost its tissue", i);
    if (b->dt[i] > g->dt_max)
      return fail(RFA_ERR_UNSTABLE, "dt[%d] exceeds the grid's stability bound", i);
    HIP_TRY(hipStreamSynchronize(g->st));
  }
  rfa_status s;
  if (!batch_in_sync(b) && (s = batch_build(b)) != RFA_OK) return s;
  std::vector<double> e0(n, 0.0);
  if (diags) {
    for (int i = 0; i < n; ++i) {
      if ((s = ensure_energy(b->grids[i])) != RFA_OK) return s;
      e0[i] = b->grids[i]->energy;
    }
    HIP_TRY(hipMemsetAsync(b->dacc, 0, 3 * (size_t)n * sizeof(double), b->st));
  }
  hipGraphExec_t exec = nullptr;
  if ((s = batch_graph(b, n_steps, diags != nullptr, &exec)) != RFA_OK) return s;
  HIP_TRY(hipEventRecord(b->ev0, b->st));
  HIP_TRY(hipGraphLaunch(exec, b->st));
  HIP_TRY(hipEventRecord(b->ev1, b->st));
  b->last_vs = b->voxels * n_steps;
  b->last_ms = -1.0;
  b->parity = (b->parity + n_steps) & 1;
  for (int i = 0; i < n; ++i) {
    rfa_grid g = b->grids[i];
    // later work on the grid's own stream waits for the batch
    HIP_TRY(hipStreamWaitEvent(g->st, b->ev1, 0));
    if (n_steps & 1) g->cur = 1 - g->cur;
    g->steps += n_steps;
    g->energy_valid = false;
    ++g->version;
  }
  if (diags) {
    HIP_TRY(hipStreamSynchronize(b->st));
    std::vector<double> acc(3 * (size_t)n);
    HIP_TRY(hipMemcpy(acc.data(), b->dacc, acc.size() * sizeof(double), hipMemcpyDeviceToHost));
    rfa_status worst = RFA_OK;
    for (int i = 0; i < n; ++i) {
      s = finish_diag(b->grids[i], &acc[3 * i], e0[i], b->dt[i], n_steps, &diags[i]);
      if (s != RFA_OK) worst = s;
    }
    if (worst != RFA_OK) return worst;
  }
  return RFA_OK;
}

rfa_status rfa_batch_set_plan(rfa_batch b, int layout, int tile_y, int tile_x, int workgroups,
                              long long group_voxels) {
  if (!b) return fail(RFA_ERR_ARG, "batch is NULL");
  if (layout < 0 || layout > RFA_BATCH_FLAT) return fail(RFA_ERR_ARG, "layout: 0, 1 or 2");
  const bool flat = layout ? layout == RFA_BATCH_FLAT : b->flat;
  const int ty = tile_y ? tile_y : (flat == b->flat ? b->ty : (flat ? 8 : 4));
  if (!flat && ty != 4 && ty != 8) return fail(RFA_ERR_ARG, "tile_y of 2.5-D tiles: 4 or 8");
  if (flat && ty != 8 && ty != 16) return fail(RFA_ERR_ARG, "tile_y of flat items: 8 or 16");
  if (tile_x < 0 || workgroups < 0) return fail(RFA_ERR_ARG, "tile_x, workgroups >= 0");
  if (b->st) HIP_TRY(hipStreamSynchronize(b->st));
  const bool flat0 = b->flat;
  const int ty0 = b->ty, xc0 = b->xc, wg0 = b->req_wg;
  const long long gv0 = b->group_budget;
  b->flat = flat;
  b->ty = ty;
  if (tile_x) b->xc = tile_x;
  b->req_wg = workgroups;
  if (group_voxels >= 0) b->group_budget = group_voxels;
  rfa_status s = batch_build(b);
  if (s != RFA_OK) {  // keep the previous plan
    std::string err = g_last_error;
    b->flat = flat0;
    b->ty = ty0;
    b->xc = xc0;
    b->req_wg = wg0;
    b->group_budget = gv0;
    (void)batch_build(b);
    g_last_error = err;
  }
  return s;
}

rfa_status rfa_batch_get_plan(rfa_batch b, int* layout, int* tile_y, int* tile_x, int* items,
                              int* workgroups, int* groups) {
  if (!b) return fail(RFA_ERR_ARG, "batch is NULL");
  if (layout) *layout = b->flat ? RFA_BATCH_FLAT : RFA_BATCH_TILES;
  if (tile_y) *tile_y = b->ty;
  if (tile_x) *tile_x = b->xc;
  if (items) *items = b->n_items;
  if (workgroups) {
    int w = 0;
    for (const auto& G : b->groups)
      w += b->n_wg > 0 ? std::min(b->n_wg, G.plain1 - G.plain0) +
                             std::min(b->n_wg, G.perf1 - G.perf0)
                       : (G.plain1 - G.plain0) + (G.perf1 - G.perf0);
    *workgroups = w;
  }
  if (groups) *groups = (int)b->groups.size();
  return RFA_OK;
}

rfa_status rfa_batch_tune(rfa_batch b, int reps) {
  if (!b) return fail(RFA_ERR_ARG, "batch is NULL");
  if (reps < 1) return fail(RFA_ERR_ARG, "reps must be >= 1");
  const int n = (int)b->grids.size();
  rfa_status s;
  if (!batch_in_sync(b) && (s = batch_build(b)) != RFA_OK) return s;
  // snapshot of what a step reads and writes: the current images, damage
  // and latch bytes (the other images are scratch to the batch)
  std::vector<void*> snap(4 * (size_t)n, nullptr);
  auto release = [&]() {
    for (void* p : snap)
      if (p) (void)hipFree(p);
  };
  auto copy_state = [&](bool save) -> hipError_t {
    for (int i = 0; i < n; ++i) {
      rfa_grid g = b->grids[i];
      const size_t nv = g->g.n();
      void* live[4] = {g->hi[g->cur], g->lo[g->cur], g->om, g->lab};
      const size_t bytes[4] = {nv * 4, nv * 4, nv * 4, nv};
      for (int k = 0; k < 4; ++k) {
        void* dst = save ? snap[4 * i + k] : live[k];
        const void* src = save ? live[k] : snap[4 * i + k];
        const hipError_t e = hipMemcpyAsync(dst, src, bytes[k], hipMemcpyDeviceToDevice, b->st);
        if (e != hipSuccess) return e;
      }
    }
    return hipStreamSynchronize(b->st);
  };
  for (int i = 0; i < n; ++i) {
    HIP_TRY(hipStreamSynchronize(b->grids[i]->st));
    const size_t nv = b->grids[i]->g.n();
    for (int k = 0; k < 4; ++k) {
      uint8_t* p = nullptr;
      if ((s = dmalloc(&p, k < 3 ? 4 * nv : nv)) != RFA_OK) {
        release();
        return s;
      }
      snap[4 * i + k] = p;
    }
  }
  hipError_t e = copy_state(true);
  if (e != hipSuccess) {
    release();
    return fail(RFA_ERR_HIP, "tune snapshot: %s", hipGetErrorString(e));
  }
  struct Cand {
    bool flat;
    int ty, xc;
    long long group;
  };
  bool flat_ok = true;
  for (rfa_grid g : b->grids) flat_ok = flat_ok && g->g.nz <= flat_max_nz(8);
  const long long g0 = kBatchGroupVoxels;
  std::vector<Cand> shapes = {{false, 4, 8, g0}, {false, 8, 8, g0}, {false, 4, 16, g0}};
  if (flat_ok) shapes.insert(shapes.begin(), {{true, 8, 8, g0}, {true, 8, 4, g0}, {true, 8, 16, g0}});
  const Cand keep{b->flat, b->ty, b->xc, b->group_budget};
  const int keep_wg = b->req_wg;
  // time reps steps of one candidate (after one untimed replay), then put
  // the state back; ms < 0 on failure
  auto time_cand = [&](const Cand& c, double* ms) -> rfa_status {
    b->flat = c.flat;
    b->ty = c.ty;
    b->xc = c.xc;
    b->group_budget = c.group;
    b->req_wg = 0;
    rfa_status st = batch_build(b);
    if (st != RFA_OK) return st;
    hipGraphExec_t exec = nullptr;
    if ((st = batch_graph(b, reps, false, &exec)) != RFA_OK) return st;
    HIP_TRY(hipGraphLaunch(exec, b->st));
    HIP_TRY(hipEventRecord(b->ev0, b->st));
    HIP_TRY(hipGraphLaunch(exec, b->st));
    HIP_TRY(hipEventRecord(b->ev1, b->st));
    HIP_TRY(hipEventSynchronize(b->ev1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, b->ev0, b->ev1));
    *ms = t;
    const hipError_t er = copy_state(false);
    if (er != hipSuccess) return fail(RFA_ERR_HIP, "tune restore: %s", hipGetErrorString(er));
    return RFA_OK;
  };
  Cand best = keep;
  double best_ms = -1.0;
  auto consider = [&](const Cand& c) -> rfa_status {
    double ms = 0.0;
    const rfa_status st = time_cand(c, &ms);
    if (st != RFA_OK) return st;
    if (best_ms < 0.0 || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return RFA_OK;
  };
  // tile shapes at the default group budget, then group budgets for the best shape
  for (const Cand& c : shapes)
    if ((s = consider(c)) != RFA_OK) break;
  if (s == RFA_OK) {
    const Cand shape = best;
    for (long long gv : {4ll << 20, 6ll << 20, 10ll << 20, 0ll}) {
      Cand c = shape;
      c.group = gv;
      if ((s = consider(c)) != RFA_OK) break;
    }
  }
  if (s != RFA_OK) {  // leave the batch as it was
    std::string err = g_last_error;
    (void)copy_state(false);
    release();
    b->flat = keep.flat;
    b->ty = keep.ty;
    b->xc = keep.xc;
    b->group_budget = keep.group;
    b->req_wg = keep_wg;
    (void)batch_build(b);
    g_last_error = err;
    return s;
  }
  release();
  b->flat = best.flat;
  b->ty = best.ty;
  b->xc = best.xc;
  b->group_budget = best.group;
  b->req_wg = 0;
  return batch_build(b);
}

rfa_status rfa_batch_last_time(rfa_batch b, double* ms, long long* voxel_steps) {
  if (!b) return fail(RFA_ERR_ARG, "batch is NULL");
  if (b->last_ms < 0.0 && b->last_vs > 0) {
    HIP_TRY(hipEventSynchronize(b->ev1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, b->ev0, b->ev1));
    b->last_ms = t;
  }
  if (ms) *ms = b->last_ms < 0.0 ? 0.0 : b->last_ms;
  if (voxel_steps) *voxel_steps = b->last_vs;
  return RFA_OK;
}

void rfa_batch_destroy(rfa_batch b) {
  if (!b) return;
  if (b->st) (void)hipStreamSynchronize(b->st);
  batch_free_device(b);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
}

void rfa_destroy_grid(rfa_grid g) {
  if (!g) return;
  if (g->st) (void)hipStreamSynchronize(g->st);
  else (void)hipDeviceSynchronize();
  free_all(g);
  delete g;
}

const char* rfa_status_string(rfa_status s) {
  switch (s) {
    case RFA_OK: return "ok";
    case RFA_ERR_ARG: return "invalid argument";
    case RFA_ERR_STATE: return "invalid state";
    case RFA_ERR_UNSTABLE: return "dt above the stability bound";
    case RFA_ERR_OOM: return "out of device memory";
    case RFA_ERR_HIP: return "HIP runtime error";
    case RFA_ERR_NUMERIC: return "non-finite state";
  }
  return "unknown status";
}

const char* rfa_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
