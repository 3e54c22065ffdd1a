/*
 * Exercises every entry point of the FP64 oracle (oracle/rfa_oracle.c) on a
 * small heterogeneous case, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: source rasterisation with per-tine shapes,
 * the stability bound, stepping with diagnostics and a kept trajectory, the
 * damage-coupled perfusion variant, the linear step and its transpose
 * (dot-product identity), the discrete adjoint and the B-spline field and
 * its transpose.  Exits 0 when the checks hold and the sanitizers report
 * nothing (they abort the run on the first finding).
 */
#include "../oracle/rfa_oracle.c"

#include <stdio.h>

#define NX 14
#define NY 13
#define NZ 15
#define N (NX * NY * NZ)

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

static int check(int ok, const char* what) {
  if (!ok) fprintf(stderr, "check failed: %s\n", what);
  return ok ? 0 : 1;
}

int main(void) {
  int bad = 0;
  unsigned seed = 12345u;
  oracle_tissue tab[4] = {
      {0.52, 1060.0, 3600.0, 0.0, 0.0, 37.0, 1, 0},
      {0.52, 1060.0, 3600.0, 24306.0, 0.0, 37.0, 0, 1},
      {0.57, 1060.0, 3600.0, 7596.0, 10714.0, 37.0, 0, 1},
      {0.52, 1060.0, 3600.0, 0.0, 0.0, 80.0, 1, 0},
  };
  uint8_t* labels = malloc(N);
  for (int i = 0; i < NX; ++i)
    for (int j = 0; j < NY; ++j)
      for (int k = 0; k < NZ; ++k) {
        size_t p = ((size_t)i * NY + j) * NZ + k;
        int outer = i == 0 || j == 0 || k == 0 || i == NX - 1 || j == NY - 1 || k == NZ - 1;
        labels[p] = outer ? 0 : (uint8_t)(1 + (urand(&seed) < 0.3) + (urand(&seed) < 0.05));
      }
  double* perf = malloc(N * sizeof(double));
  for (int p = 0; p < N; ++p) perf[p] = 0.5 + urand(&seed);
  oracle_problem P = {NX, NY, NZ, 1e-3, 0.9e-3, 1.1e-3, labels, tab, 4, NULL, perf,
                      37.0, 60.0, 7.39e39, 2.577e5, 8.314, 1e30, 0};
  /* two tines: a straight segment and a three-chord polyline */
  int off[3] = {0, 2, 6};
  double pts[18] = {-2e-3, 0, -3e-3, 1e-3, 0, 3e-3,
                    0, -2e-3, 0, 1e-3, -1e-3, 1e-3, 2e-3, 1e-3, 2e-3, 3e-3, 2e-3, 3e-3};
  double power[2] = {8.0, 5.0};
  double* q = malloc(N * sizeof(double));
  double* g = malloc(2 * N * sizeof(double));
  double un[2];
  bad += check(oracle_source(&P, 2, off, pts, power, 1.2e-3, q, g, un) == 0, "source");
  double total = 0.0, vol = P.dx * P.dy * P.dz;
  for (int p = 0; p < N; ++p) total += q[p] * vol;
  bad += check(fabs(total - 13.0) < 1e-9, "source normalisation");
  P.q = q;
  double dt = 0.5 * oracle_dt_max(&P);
  bad += check(dt > 0.0 && isfinite(dt), "dt_max");

  double *T = malloc(N * sizeof(double)), *om = malloc(N * sizeof(double));
  double *tm = malloc(N * sizeof(double)), *diag = malloc(30 * DIAG_N * sizeof(double));
  double* traj = malloc((size_t)30 * N * sizeof(double));
  oracle_init(&P, T, om, tm);
  bad += check(oracle_run(&P, 30, dt, T, om, tm, diag, traj) == 0, "run");
  for (int s = 0; s < 30; ++s) {
    double scale = fabs(diag[s * DIAG_N + DIAG_INJECTED]) + fabs(diag[s * DIAG_N + DIAG_PERFUSION]) +
                   fabs(diag[s * DIAG_N + DIAG_BOUNDARY]);
    bad += check(fabs(diag[s * DIAG_N + DIAG_RESIDUAL]) <= 1e-9 * scale, "energy balance");
  }
  P.perf_decay = 1;
  oracle_init(&P, T, om, tm);
  bad += check(oracle_run(&P, 10, dt, T, om, tm, NULL, NULL) == 0, "coupled run");
  P.perf_decay = 0;

  double *x = malloc(N * sizeof(double)), *y = malloc(N * sizeof(double));
  double *Mx = malloc(N * sizeof(double)), *MTy = malloc(N * sizeof(double));
  for (int p = 0; p < N; ++p) {
    x[p] = urand(&seed) - 0.5;
    y[p] = urand(&seed) - 0.5;
  }
  oracle_step_linear(&P, dt, x, Mx);
  oracle_step_linear_transpose(&P, dt, y, MTy);
  double l = 0.0, r = 0.0, a = 0.0;
  for (int p = 0; p < N; ++p) {
    l += Mx[p] * y[p];
    r += x[p] * MTy[p];
    a += fabs(Mx[p] * y[p]);
  }
  bad += check(fabs(l - r) <= 1e-13 * a, "adjoint dot product");

  double *T0 = malloc(N * sizeof(double)), *w = malloc(N * sizeof(double));
  double *dq = malloc(N * sizeof(double)), *dperf = malloc(N * sizeof(double));
  oracle_init(&P, T0, NULL, NULL);
  for (int p = 0; p < N; ++p) w[p] = urand(&seed);
  bad += check(oracle_adjoint(&P, 12, dt, T0, w, dq, dperf) == 0, "adjoint");
  for (int p = 0; p < N; ++p) bad += check(isfinite(dq[p]) && isfinite(dperf[p]), "adjoint finite");
  P.perf_decay = 1;
  bad += check(oracle_adjoint(&P, 12, dt, T0, w, dq, dperf) == -2, "coupled adjoint refused");
  P.perf_decay = 0;

  const int m = 6;
  double *ctrl = malloc(m * m * m * sizeof(double)), *f = malloc(N * sizeof(double));
  double* gc = malloc(m * m * m * sizeof(double));
  for (int c = 0; c < m * m * m; ++c) ctrl[c] = 0.2 * (urand(&seed) - 0.5);
  oracle_bspline_field(NX, NY, NZ, m, ctrl, f);
  oracle_bspline_grad(NX, NY, NZ, m, f, w, gc);
  for (int c = 0; c < m * m * m; ++c) bad += check(isfinite(gc[c]), "bspline grad finite");
  bad += check(oracle_damage_rate(7.39e39, 2.577e5, 8.314, 60.0) > 0.28, "damage rate");
  double d1 = oracle_tine_density_at(&P, off, pts, 1.2e-3, 1, 7, 6, 7);
  bad += check(d1 > 0.0 && isfinite(d1), "tine density");

  free(labels); free(perf); free(q); free(g); free(T); free(om); free(tm); free(diag);
  free(traj); free(x); free(y); free(Mx); free(MTy); free(T0); free(w); free(dq);
  free(dperf); free(ctrl); free(f); free(gc);
  if (bad) fprintf(stderr, "%d checks failed\n", bad);
  else printf("oracle sanitizer run: all checks passed\n");
  return bad ? 1 : 0;
}
