/*
 * rfa_oracle.c -- plain FP64 CPU oracle of the explicit bioheat stepper.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library; the two meet only through the seeded
 * inputs of the workload generator.
 *
 * Written for clarity, not speed: one pass per time step, every voxel
 * evaluated from the previous step only (Jacobi), double precision
 * throughout, compiled with -O2 -ffp-contract=off.  An OpenMP pragma
 * parallelises the voxel loops over x-planes; results do not depend on the
 * thread count (reductions are summed per plane, then over planes in order).
 *
 * What it computes (paper: Kath, Handels, Mastmeyer, "Robust GPU-based
 * Virtual Reality Simulation of Radio Frequency Ablations for Various Needle
 * Geometries and Locations"):
 *
 *  - model: the simplified Pennes equation, Eq. (2675-eq1_Kath), i.e.
 *    rho c dT/dt = div(K grad T) + w_b c_b (T_a - T) + Q_m, plus an RF power
 *    density q from the needle (the paper's AT term f of Eq. (eq:setup));
 *  - discretisation: symmetric second differences, Eq. (2675-eq3), and the
 *    explicit forward-Euler voxel update, Eq. (CUDAbioheat3d); voxel-wise
 *    conductivity enters through the conservative flux form with the
 *    harmonic mean of the two voxel conductivities on each face (reading of
 *    the garbled parentheses of Eq. (CUDAbioheat3d) together with the
 *    div(K grad T) of Eq. (2675-eq1_Kath));
 *  - held voxels: per Alg. 1, voxels of a "fixed" class (vessel / tip in the
 *    paper) and the outermost voxel layer keep their input value; all other
 *    voxels take the full update;
 *  - double buffer: Alg. 2 (two images, swapped every step);
 *  - damage: the Arrhenius integral of Eq. (eq-tissState) with T in Kelvin,
 *    Omega += dt A exp(-Ea / (R T_K)) evaluated at the start of the step, and
 *    the instantaneous-necrosis latch T >= t_death (60 degC, Introduction);
 *  - RF source: each tine's polyline is a chain of segments, each a uniform
 *    line density convolved with an isotropic 3-D Gaussian of width sigma;
 *    the field is zeroed on held voxels and scaled so the tine delivers its
 *    power exactly on the grid.  No truncation.
 *  - optionally, Linte's tissue-state factor on the perfusion term (Eq.
 *    (2675-eq1_Linte), Eq. (eq-tissState)): blood cooling scaled by the
 *    surviving cell fraction exp(-Omega) (perfusion_h);
 *  - discrete adjoint of the stepper (transpose of the linear step, plus the
 *    damage-rate derivative), for gradient checks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double k;        /* thermal conductivity K, W/m/K                        */
  double rho;      /* density, kg/m^3                                       */
  double c;        /* specific heat capacity c_p, J/kg/K                    */
  double h;        /* volumetric perfusion coefficient w_b c_b, W/m^3/K     */
  double q_met;    /* metabolic heat Q_m, W/m^3                             */
  double t_fixed;  /* held temperature of a fixed class, degC               */
  int fixed;       /* 1: class keeps its value (Alg. 1 "else" branch)       */
  int tissue;      /* 1: class accumulates damage                           */
} oracle_tissue;

typedef struct {
  int nx, ny, nz;              /* voxels; layout [x][y][z], z fastest       */
  double dx, dy, dz;           /* voxel spacing, metres                     */
  const uint8_t* labels;       /* class per voxel                           */
  const oracle_tissue* tab;    /* class table                               */
  int n_classes;
  const double* q;             /* RF power density W/m^3 per voxel, or NULL */
  const double* perf;          /* perfusion multiplier per voxel, or NULL   */
  double t_blood;              /* arterial blood temperature T_a, degC      */
  double t_death;              /* necrosis threshold, degC                  */
  double A, Ea, R;             /* Arrhenius: 1/s, J/mol, J/mol/K            */
  double omega_cap;            /* guard on the damage integral              */
  int perf_decay;              /* 1: perfusion scaled by the surviving cell
                                  fraction exp(-Omega) (see perfusion_h)    */
} oracle_problem;

enum { DIAG_ENERGY = 0, DIAG_INJECTED, DIAG_PERFUSION, DIAG_BOUNDARY,
       DIAG_RESIDUAL, DIAG_MONO, DIAG_TMIN, DIAG_TMAX, DIAG_N };

static const double KELVIN = 273.15;
static const double T_BODY_K = 310.15;   /* 37 degC in Kelvin            */
static const double EXPONENT_CLAMP = 80.0;

static size_t vidx(const oracle_problem* P, int i, int j, int k) {
  return ((size_t)i * (size_t)P->ny + (size_t)j) * (size_t)P->nz + (size_t)k;
}

static int on_outer_layer(const oracle_problem* P, int i, int j, int k) {
  return i == 0 || j == 0 || k == 0 || i == P->nx - 1 || j == P->ny - 1 ||
         k == P->nz - 1;
}

/* A voxel is updated by the step (Alg. 1 "if" branch) unless its class is
 * fixed or it lies on the outermost layer of the grid. */
static int is_free(const oracle_problem* P, int i, int j, int k) {
  const oracle_tissue* t = &P->tab[P->labels[vidx(P, i, j, k)]];
  return !t->fixed && !on_outer_layer(P, i, j, k);
}

/* Face conductivity between two classes: harmonic mean (series resistance
 * of the two half voxels). */
static double face_k(const oracle_problem* P, int a, int b) {
  double ka = P->tab[a].k, kb = P->tab[b].k;
  if (ka + kb == 0.0) return 0.0;
  return 2.0 * ka * kb / (ka + kb);
}

/* Perfusion coefficient of voxel p.  With perf_decay, Linte's tissue-state
 * factor of Eq. (2675-eq1_Linte) scales it: the healthy-cell fraction
 * c(t)/c(0) = exp(-Omega), since Eq. (eq-tissState) defines the damage
 * integral as Omega = ln(c(0)/c(t)); it falls from 1 for intact tissue to 0
 * for dead tissue without blood cooling, as the paper describes the term.
 * (The printed alpha = 1/ln(c(0)/c(t)) is singular at t = 0, which the
 * paper points out; the healthy-cell fraction is the reading that has the
 * stated limits.)  Omega is the voxel's value at the start of the step
 * (left point, as the damage increment); omega may be NULL (Omega = 0). */
static double perfusion_h(const oracle_problem* P, size_t p, const double* omega) {
  double h = P->tab[P->labels[p]].h;
  if (P->perf) h *= P->perf[p];
  if (P->perf_decay && omega) h *= exp(-omega[p]);
  return h;
}

/* Arrhenius damage rate A exp(-Ea / (R T_K)) with T_K = T + 273.15, capped
 * at the value the rate takes where its exponent relative to 37 degC reaches
 * EXPONENT_CLAMP (a guard far above any physical temperature). */
double oracle_damage_rate(double A, double Ea, double R, double t_c) {
  double r = A * exp(-Ea / (R * (t_c + KELVIN)));
  double rmax = A * exp(-Ea / (R * T_BODY_K)) * exp(EXPONENT_CLAMP);
  return r < rmax ? r : rmax;
}

/* d rate / dT, zero where the cap is active. */
static double damage_rate_deriv(double A, double Ea, double R, double t_c) {
  double tk = t_c + KELVIN;
  double r = A * exp(-Ea / (R * tk));
  double rmax = A * exp(-Ea / (R * T_BODY_K)) * exp(EXPONENT_CLAMP);
  if (r >= rmax) return 0.0;
  return r * Ea / (R * tk * tk);
}

/* ------------------------------------------------------------------------ */
/* RF source                                                                */
/* ------------------------------------------------------------------------ */

/* Density at point x of the segment a->b carrying unit line density,
 * convolved with an isotropic 3-D Gaussian of standard deviation sigma:
 *   (2 pi s^2)^-1 exp(-d_perp^2 / 2 s^2) * 1/2 [erf((L/2 - s)/(sqrt2 sigma))
 *                                             + erf((L/2 + s)/(sqrt2 sigma))]
 * with s the signed axial offset from the segment midpoint and d_perp the
 * distance from the segment's line.  Units: 1/m^2. */
double oracle_segment_density(const double* a, const double* b, double sigma,
                              const double* x) {
  double m[3], u[3], r[3];
  double len2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    m[d] = 0.5 * (a[d] + b[d]);
    u[d] = b[d] - a[d];
    len2 += u[d] * u[d];
  }
  double len = sqrt(len2);
  if (len == 0.0) return 0.0;
  double s = 0.0, r2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    u[d] /= len;
    r[d] = x[d] - m[d];
    s += r[d] * u[d];
    r2 += r[d] * r[d];
  }
  double dperp2 = r2 - s * s;
  if (dperp2 < 0.0) dperp2 = 0.0;
  double radial = exp(-dperp2 / (2.0 * sigma * sigma)) / (2.0 * M_PI * sigma * sigma);
  double w = sqrt(2.0) * sigma;
  double axial = 0.5 * (erf((0.5 * len - s) / w) + erf((0.5 * len + s) / w));
  return radial * axial;
}

static void voxel_centre(const oracle_problem* P, int i, int j, int k, double* x) {
  x[0] = (2.0 * i - (P->nx - 1)) * P->dx / 2.0;
  x[1] = (2.0 * j - (P->ny - 1)) * P->dy / 2.0;
  x[2] = (2.0 * k - (P->nz - 1)) * P->dz / 2.0;
}

/* Unnormalised density of one tine (sum over its segments) at voxel (i,j,k). */
double oracle_tine_density_at(const oracle_problem* P, const int* pt_offset,
                              const double* pts, double sigma, int tine,
                              int i, int j, int k) {
  double x[3];
  voxel_centre(P, i, j, k, x);
  double g = 0.0;
  for (int p = pt_offset[tine]; p + 1 < pt_offset[tine + 1]; ++p)
    g += oracle_segment_density(pts + 3 * p, pts + 3 * (p + 1), sigma, x);
  return g;
}

/* Per-tine shapes g_hat[t][p] in 1/m^3 (zero on held voxels, sum g_hat V = 1)
 * and the total power density q = sum_t power[t] g_hat[t].  unnorm[t]
 * receives sum_p g_t(p) V before normalisation.  Returns 0, or -1 if a tine
 * has no weight on free voxels (cannot be normalised). */
int oracle_source(const oracle_problem* P, int n_tines, const int* pt_offset,
                  const double* pts, const double* power, double sigma,
                  double* q, double* g_hat, double* unnorm) {
  size_t n = (size_t)P->nx * P->ny * P->nz;
  double vol = P->dx * P->dy * P->dz;
  if (q) memset(q, 0, n * sizeof(double));
  int status = 0;
  for (int t = 0; t < n_tines; ++t) {
    double* g = g_hat ? g_hat + (size_t)t * n : (double*)malloc(n * sizeof(double));
    double* plane = (double*)calloc((size_t)P->nx, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nx; ++i) {
      double acc = 0.0;
      for (int j = 0; j < P->ny; ++j)
        for (int k = 0; k < P->nz; ++k) {
          size_t p = vidx(P, i, j, k);
          double v = is_free(P, i, j, k)
                         ? oracle_tine_density_at(P, pt_offset, pts, sigma, t, i, j, k)
                         : 0.0;
          g[p] = v;
          acc += v;
        }
      plane[i] = acc;
    }
    double total = 0.0;
    for (int i = 0; i < P->nx; ++i) total += plane[i];
    free(plane);
    total *= vol;
    if (unnorm) unnorm[t] = total;
    if (total > 0.0) {
      for (size_t p = 0; p < n; ++p) g[p] /= total;
    } else {
      status = -1;
    }
    if (q)
      for (size_t p = 0; p < n; ++p) q[p] += power[t] * g[p];
    if (!g_hat) free(g);
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* Stepper                                                                  */
/* ------------------------------------------------------------------------ */

/* Conduction term sum_d [K_f(-)(T_- - T) + K_f(+)(T_+ - T)] / dd^2 at a free
 * voxel; the two faces of an axis are summed first (mirror symmetry). */
static double conduction(const oracle_problem* P, const double* T, int i, int j, int k) {
  size_t p = vidx(P, i, j, k);
  int l = P->labels[p];
  size_t xm = vidx(P, i - 1, j, k), xp = vidx(P, i + 1, j, k);
  size_t ym = vidx(P, i, j - 1, k), yp = vidx(P, i, j + 1, k);
  size_t zm = vidx(P, i, j, k - 1), zp = vidx(P, i, j, k + 1);
  double fx = (face_k(P, l, P->labels[xm]) * (T[xm] - T[p]) +
               face_k(P, l, P->labels[xp]) * (T[xp] - T[p])) / (P->dx * P->dx);
  double fy = (face_k(P, l, P->labels[ym]) * (T[ym] - T[p]) +
               face_k(P, l, P->labels[yp]) * (T[yp] - T[p])) / (P->dy * P->dy);
  double fz = (face_k(P, l, P->labels[zm]) * (T[zm] - T[p]) +
               face_k(P, l, P->labels[zp]) * (T[zp] - T[p])) / (P->dz * P->dz);
  return (fx + fy) + fz;
}

/* Heat flowing into free voxel (i,j,k) from held neighbours, W/m^3. */
static double held_inflow(const oracle_problem* P, const double* T, int i, int j, int k) {
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  size_t p = vidx(P, i, j, k);
  int l = P->labels[p];
  double d2[3] = {P->dx * P->dx, P->dy * P->dy, P->dz * P->dz};
  double f = 0.0;
  for (int n = 0; n < 6; ++n) {
    int a = i + off[n][0], b = j + off[n][1], c = k + off[n][2];
    if (is_free(P, a, b, c)) continue;
    size_t nb = vidx(P, a, b, c);
    f += face_k(P, l, P->labels[nb]) * (T[nb] - T[p]) / d2[n / 2];
  }
  return f;
}

/* Initial state: held classes at their temperature, everything else at the
 * blood temperature of 37 degC; no damage; running maximum = T. */
void oracle_init(const oracle_problem* P, double* T, double* omega, double* tmax) {
  size_t n = (size_t)P->nx * P->ny * P->nz;
  for (size_t p = 0; p < n; ++p) {
    const oracle_tissue* t = &P->tab[P->labels[p]];
    T[p] = t->fixed ? t->t_fixed : 37.0;
    if (omega) omega[p] = 0.0;
    if (tmax) tmax[p] = T[p];
  }
}

/* Energy above 37 degC held by the free voxels, J. */
static double free_energy(const oracle_problem* P, const double* T) {
  double vol = P->dx * P->dy * P->dz;
  double* plane = (double*)calloc((size_t)P->nx, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int i = 0; i < P->nx; ++i) {
    double acc = 0.0;
    for (int j = 0; j < P->ny; ++j)
      for (int k = 0; k < P->nz; ++k) {
        if (!is_free(P, i, j, k)) continue;
        size_t p = vidx(P, i, j, k);
        const oracle_tissue* t = &P->tab[P->labels[p]];
        acc += t->rho * t->c * (T[p] - 37.0) * vol;
      }
    plane[i] = acc;
  }
  double e = 0.0;
  for (int i = 0; i < P->nx; ++i) e += plane[i];
  free(plane);
  return e;
}

/*
 * Advance n_steps explicit Euler steps of length dt.
 * T, omega, tmax are [N] in/out (degC, dimensionless, degC).  If traj is
 * not NULL it receives T^s for s = 0 .. n_steps-1 (n_steps * N doubles).
 * If diag is not NULL it receives DIAG_N doubles per step: energy of free
 * voxels after the step, injected energy (RF + metabolic), perfusion loss,
 * heat from held voxels, balance residual (all J), count of free voxels
 * whose temperature fell, min and max temperature after the step.
 */
int oracle_run(const oracle_problem* P, int n_steps, double dt, double* T,
               double* omega, double* tmax, double* diag, double* traj) {
  size_t n = (size_t)P->nx * P->ny * P->nz;
  double vol = P->dx * P->dy * P->dz;
  double* buf = (double*)malloc(n * sizeof(double));
  double* acc = (double*)malloc((size_t)P->nx * 5 * sizeof(double));
  if (!buf || !acc) { free(buf); free(acc); return -1; }
  double* cur = T;   /* Alg. 2: the two images of the double buffer */
  double* nxt = buf;
  double energy = diag ? free_energy(P, cur) : 0.0;
  for (int s = 0; s < n_steps; ++s) {
    if (traj) memcpy(traj + (size_t)s * n, cur, n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nx; ++i) {
      double inj = 0.0, perf = 0.0, bnd = 0.0, mono = 0.0;
      for (int j = 0; j < P->ny; ++j)
        for (int k = 0; k < P->nz; ++k) {
          size_t p = vidx(P, i, j, k);
          const oracle_tissue* t = &P->tab[P->labels[p]];
          if (is_free(P, i, j, k)) {
            double h = perfusion_h(P, p, omega);
            double q = P->q ? P->q[p] : 0.0;
            double rhs = conduction(P, cur, i, j, k) + h * (P->t_blood - cur[p]) +
                         t->q_met + q;
            nxt[p] = cur[p] + dt / (t->rho * t->c) * rhs;
            if (diag) {
              inj += (t->q_met + q) * dt * vol;
              perf += h * (cur[p] - P->t_blood) * dt * vol;
              bnd += held_inflow(P, cur, i, j, k) * dt * vol;
              if (nxt[p] < cur[p]) mono += 1.0;
            }
          } else {
            nxt[p] = cur[p];
          }
          if (t->tissue && omega) {
            double w = omega[p] + dt * oracle_damage_rate(P->A, P->Ea, P->R, cur[p]);
            omega[p] = w < P->omega_cap ? w : P->omega_cap;
          }
          if (tmax && nxt[p] > tmax[p]) tmax[p] = nxt[p];
        }
      acc[5 * i + 0] = inj;
      acc[5 * i + 1] = perf;
      acc[5 * i + 2] = bnd;
      acc[5 * i + 3] = mono;
    }
    if (diag) {
      double inj = 0.0, perf = 0.0, bnd = 0.0, mono = 0.0;
      for (int i = 0; i < P->nx; ++i) {
        inj += acc[5 * i + 0];
        perf += acc[5 * i + 1];
        bnd += acc[5 * i + 2];
        mono += acc[5 * i + 3];
      }
      double e1 = free_energy(P, nxt);
      double tmin = nxt[0], tmx = nxt[0];
      for (size_t p = 1; p < n; ++p) {
        if (nxt[p] < tmin) tmin = nxt[p];
        if (nxt[p] > tmx) tmx = nxt[p];
      }
      double* d = diag + (size_t)s * DIAG_N;
      d[DIAG_ENERGY] = e1;
      d[DIAG_INJECTED] = inj;
      d[DIAG_PERFUSION] = perf;
      d[DIAG_BOUNDARY] = bnd;
      d[DIAG_RESIDUAL] = (e1 - energy) - (inj - perf + bnd);
      d[DIAG_MONO] = mono;
      d[DIAG_TMIN] = tmin;
      d[DIAG_TMAX] = tmx;
      energy = e1;
    }
    double* sw = cur; cur = nxt; nxt = sw;
  }
  if (cur != T) memcpy(T, cur, n * sizeof(double));
  free(buf);
  free(acc);
  return 0;
}

/* Largest stable dt: the explicit update is a convex combination of the
 * voxel and its neighbours (maximum principle, monotone rise) iff
 * dt <= rho c / (sum_faces K_f / dd^2 + h) at every free voxel. */
double oracle_dt_max(const oracle_problem* P) {
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  double d2[3] = {P->dx * P->dx, P->dy * P->dy, P->dz * P->dz};
  double best = INFINITY;
  for (int i = 0; i < P->nx; ++i)
    for (int j = 0; j < P->ny; ++j)
      for (int k = 0; k < P->nz; ++k) {
        if (!is_free(P, i, j, k)) continue;
        size_t p = vidx(P, i, j, k);
        int l = P->labels[p];
        /* the full coefficient bounds the decayed one (exp(-Omega) <= 1) */
        double s = perfusion_h(P, p, NULL);
        for (int m = 0; m < 6; ++m) {
          size_t nb = vidx(P, i + off[m][0], j + off[m][1], k + off[m][2]);
          s += face_k(P, l, P->labels[nb]) / d2[m / 2];
        }
        double dtm = P->tab[l].rho * P->tab[l].c / s;
        if (dtm < best) best = dtm;
      }
  return best;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint                                                         */
/* ------------------------------------------------------------------------ */

/* y = M x, the linear part of one step (sources removed): free rows carry
 * the explicit stencil including the perfusion sink, held rows the identity. */
void oracle_step_linear(const oracle_problem* P, double dt, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < P->nx; ++i)
    for (int j = 0; j < P->ny; ++j)
      for (int k = 0; k < P->nz; ++k) {
        size_t p = vidx(P, i, j, k);
        if (!is_free(P, i, j, k)) { y[p] = x[p]; continue; }
        const oracle_tissue* t = &P->tab[P->labels[p]];
        double rhs = conduction(P, x, i, j, k) - perfusion_h(P, p, NULL) * x[p];
        y[p] = x[p] + dt / (t->rho * t->c) * rhs;
      }
}

/* y = M^T x.  Column q of M collects: the diagonal of q's own row, and for
 * each free neighbour p of q the coefficient dt K_f / (rho_p c_p dd^2) that
 * q's value carries in p's row.  Written as an explicit gather (no shared
 * code with oracle_step_linear) so the dot-product test compares two
 * independent constructions. */
void oracle_step_linear_transpose(const oracle_problem* P, double dt, const double* x,
                                  double* y) {
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  double d2[3] = {P->dx * P->dx, P->dy * P->dy, P->dz * P->dz};
#pragma omp parallel for schedule(static)
  for (int i = 0; i < P->nx; ++i)
    for (int j = 0; j < P->ny; ++j)
      for (int k = 0; k < P->nz; ++k) {
        size_t q = vidx(P, i, j, k);
        int lq = P->labels[q];
        double v;
        int qfree = is_free(P, i, j, k);
        if (qfree) {
          double diag = perfusion_h(P, q, NULL);
          for (int m = 0; m < 6; ++m) {
            size_t nb = vidx(P, i + off[m][0], j + off[m][1], k + off[m][2]);
            diag += face_k(P, lq, P->labels[nb]) / d2[m / 2];
          }
          v = (1.0 - dt / (P->tab[lq].rho * P->tab[lq].c) * diag) * x[q];
        } else {
          v = x[q];
        }
        for (int m = 0; m < 6; ++m) {
          int a = i + off[m][0], b = j + off[m][1], c = k + off[m][2];
          if (a < 0 || b < 0 || c < 0 || a >= P->nx || b >= P->ny || c >= P->nz) continue;
          if (!is_free(P, a, b, c)) continue;
          size_t p = vidx(P, a, b, c);
          int lp = P->labels[p];
          v += dt * face_k(P, lp, lq) / (P->tab[lp].rho * P->tab[lp].c * d2[m / 2]) * x[p];
        }
        y[q] = v;
      }
}

/*
 * Discrete adjoint of n_steps forward steps starting from T0 (degC) with
 * Omega^0 = 0, for a loss whose gradient with respect to the final damage
 * integral Omega^N is w (per voxel).  Outputs (either may be NULL):
 *   dq[p] = dL / dq_p   (q: RF power density, W/m^3)
 *   dperf[p] = dL / dperf_p  (perf: per-voxel multiplier of the class
 *              perfusion coefficient, h_p = h_class * perf_p)
 * The whole trajectory is kept in memory (plain, no checkpointing).
 * Voxels whose Omega^N reached omega_cap contribute no damage gradient,
 * and the exponent cap of the damage rate has zero derivative.
 */
int oracle_adjoint(const oracle_problem* P, int n_steps, double dt, const double* T0,
                   const double* w, double* dq, double* dperf) {
  /* the damage-coupled perfusion makes the step nonlinear in (T, Omega);
   * its adjoint is not part of this oracle */
  if (P->perf_decay) return -2;
  size_t n = (size_t)P->nx * P->ny * P->nz;
  double* traj = (double*)malloc((size_t)n_steps * n * sizeof(double));
  double* T = (double*)malloc(n * sizeof(double));
  double* om = (double*)malloc(n * sizeof(double));
  double* lam = (double*)calloc(n, sizeof(double));
  double* tmp = (double*)malloc(n * sizeof(double));
  double* wa = (double*)malloc(n * sizeof(double));
  if (!traj || !T || !om || !lam || !tmp || !wa) {
    free(traj); free(T); free(om); free(lam); free(tmp); free(wa);
    return -1;
  }
  memcpy(T, T0, n * sizeof(double));
  memset(om, 0, n * sizeof(double));
  oracle_run(P, n_steps, dt, T, om, NULL, NULL, traj);
  for (size_t p = 0; p < n; ++p) {
    const oracle_tissue* t = &P->tab[P->labels[p]];
    wa[p] = (t->tissue && om[p] < P->omega_cap) ? w[p] : 0.0;
  }
  if (dq) memset(dq, 0, n * sizeof(double));
  if (dperf) memset(dperf, 0, n * sizeof(double));
  /* lam holds lambda^{s+1} = dL/dT^{s+1}; lambda^N = 0. */
  for (int s = n_steps - 1; s >= 0; --s) {
    const double* Ts = traj + (size_t)s * n;
    for (int i = 0; i < P->nx; ++i)
      for (int j = 0; j < P->ny; ++j)
        for (int k = 0; k < P->nz; ++k) {
          if (!is_free(P, i, j, k)) continue;
          size_t p = vidx(P, i, j, k);
          const oracle_tissue* t = &P->tab[P->labels[p]];
          double g = dt / (t->rho * t->c) * lam[p];
          if (dq) dq[p] += g;
          if (dperf) dperf[p] += g * (P->t_blood - Ts[p]) * t->h;
        }
    oracle_step_linear_transpose(P, dt, lam, tmp);
    for (size_t p = 0; p < n; ++p)
      lam[p] = tmp[p] + wa[p] * dt * damage_rate_deriv(P->A, P->Ea, P->R, Ts[p]);
  }
  free(traj); free(T); free(om); free(lam); free(tmp); free(wa);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Perfusion-correction field: uniform cubic B-spline on a control lattice  */
/* ------------------------------------------------------------------------ */

/* Knot span and local coordinate of voxel i of n along an axis carried by
 * m control points: u = i (m - 3) / (n - 1), span = min(floor(u), m - 4). */
static void bspline_span(int i, int n, int m, int* span, double* t) {
  double u = n > 1 ? (double)i * (double)(m - 3) / (double)(n - 1) : 0.0;
  int s = (int)floor(u);
  if (s > m - 4) s = m - 4;
  if (s < 0) s = 0;
  *span = s;
  *t = u - s;
}

/* Uniform cubic B-spline basis values at local coordinate t in [0,1]. */
static void bspline_basis(double t, double* b) {
  double s = 1.0 - t;
  b[0] = s * s * s / 6.0;
  b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  b[3] = t * t * t / 6.0;
}

/* f[p] = exp(sum_j B_j(x_p) ctrl_j): multiplier of the perfusion
 * coefficient, ctrl is [m][m][m] (x slowest). */
void oracle_bspline_field(int nx, int ny, int nz, int m, const double* ctrl, double* f) {
  for (int i = 0; i < nx; ++i) {
    int si; double ti, bi[4];
    bspline_span(i, nx, m, &si, &ti);
    bspline_basis(ti, bi);
    for (int j = 0; j < ny; ++j) {
      int sj; double tj, bj[4];
      bspline_span(j, ny, m, &sj, &tj);
      bspline_basis(tj, bj);
      for (int k = 0; k < nz; ++k) {
        int sk; double tk, bk[4];
        bspline_span(k, nz, m, &sk, &tk);
        bspline_basis(tk, bk);
        double v = 0.0;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
              v += bi[a] * bj[b] * bk[c] *
                   ctrl[((size_t)(si + a) * m + (sj + b)) * m + (sk + c)];
        f[((size_t)i * ny + j) * nz + k] = exp(v);
      }
    }
  }
}

/* Transpose of the field map: with f = exp(sum_j B_j c_j) and gf = dL/df,
 * gctrl[j] = dL/dc_j = sum_p gf_p f_p B_j(x_p). */
void oracle_bspline_grad(int nx, int ny, int nz, int m, const double* f, const double* gf,
                         double* gctrl) {
  memset(gctrl, 0, (size_t)m * m * m * sizeof(double));
  for (int i = 0; i < nx; ++i) {
    int si; double ti, bi[4];
    bspline_span(i, nx, m, &si, &ti);
    bspline_basis(ti, bi);
    for (int j = 0; j < ny; ++j) {
      int sj; double tj, bj[4];
      bspline_span(j, ny, m, &sj, &tj);
      bspline_basis(tj, bj);
      for (int k = 0; k < nz; ++k) {
        int sk; double tk, bk[4];
        bspline_span(k, nz, m, &sk, &tk);
        bspline_basis(tk, bk);
        size_t p = ((size_t)i * ny + j) * nz + k;
        double g = gf[p] * f[p];
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
              gctrl[((size_t)(si + a) * m + (sj + b)) * m + (sk + c)] +=
                  bi[a] * bj[b] * bk[c] * g;
      }
    }
  }
}
