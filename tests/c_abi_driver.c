/* Plain C99 client of librfa.so (include/rfa.h): reads a case from a binary
 * file and drives the library through the C ABI alone.  Built and run by
 * tests/test_gpu_c_abi.py, which writes the input and checks the output
 * against the FP64 oracle or the Python binding.
 *
 * usage: c_abi_driver input output [step|batch|adjoint]
 *   step    (default) steps the case and writes its temperature, damage
 *           mask, damage integral and diagnostics;
 *   batch   steps two copies of the case in one batch and a third copy
 *           alone, and writes 1 if all three raw states are bitwise equal
 *           (else 0), then the batch plan;
 *   adjoint a checkpointed forward (a checkpoint every n_steps / 3 + 1
 *           steps) with a zero 4^3 perfusion lattice, then the adjoint of
 *           L = sum of the damage integral over tissue voxels: writes
 *           dL/dP [n_tines] and dL/dctrl [64].
 *
 * Input (little-endian, packed in this order):
 *   int32 nx, ny, nz; float64 dx, dy, dz;
 *   float64 t_death, A, Ea, R, omega_cap;
 *   int32 n_classes; n_classes x { float64 k, rho, c, h_perf, q_met, t_fixed;
 *                                  int32 fixed, tissue };
 *   uint8 labels[nx*ny*nz];
 *   int32 n_tines; int32 pt_offset[n_tines + 1]; float64 pts[3 * n_points];
 *   float64 power[n_tines]; float64 sigma;
 *   float64 dt; int32 n_steps.
 * Output of step: float64 T[n] (degC), uint8 mask[n], float32 omega[n],
 *   then float64 energy_J, injected_J, residual_J; int64 mono_violations.
 * Output of batch: int32 equal; int32 layout, tile_y, tile_x, items,
 *   workgroups, groups.
 * Output of adjoint: float64 dL_dP[n_tines], float64 dL_dctrl[64].
 * Exit status 0 on success; otherwise the failing call and
 * rfa_last_error() are printed to stderr. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/rfa.h"

typedef struct {
  int32_t nx, ny, nz, n_classes, n_tines, n_steps;
  double dx, dy, dz, dt;
  rfa_options opt;
  rfa_tissue table[16];
  uint8_t* labels;
  rfa_needle needle;
  int32_t* off;
  double* pts;
  double* power;
} Case;

static FILE* in;

static void rd(void* p, size_t size, size_t count) {
  if (fread(p, size, count, in) != count) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}

static int check(rfa_status s, const char* what) {
  if (s != RFA_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, rfa_status_string(s), rfa_last_error());
    return 1;
  }
  return 0;
}

static int read_case(const char* path, Case* c) {
  in = fopen(path, "rb");
  if (!in) return 2;
  if (check(rfa_default_options(&c->opt), "rfa_default_options")) return 1;
  rd(&c->nx, 4, 1);
  rd(&c->ny, 4, 1);
  rd(&c->nz, 4, 1);
  rd(&c->dx, 8, 1);
  rd(&c->dy, 8, 1);
  rd(&c->dz, 8, 1);
  rd(&c->opt.t_death, 8, 1);
  rd(&c->opt.A, 8, 1);
  rd(&c->opt.Ea, 8, 1);
  rd(&c->opt.R, 8, 1);
  rd(&c->opt.omega_cap, 8, 1);
  rd(&c->n_classes, 4, 1);
  if (c->n_classes < 1 || c->n_classes > 16) return 2;
  for (int i = 0; i < c->n_classes; ++i) {
    double v[6];
    int32_t f[2];
    rd(v, 8, 6);
    rd(f, 4, 2);
    c->table[i].k = v[0];
    c->table[i].rho = v[1];
    c->table[i].c = v[2];
    c->table[i].h_perf = v[3];
    c->table[i].q_met = v[4];
    c->table[i].t_fixed = v[5];
    c->table[i].fixed = f[0];
    c->table[i].tissue = f[1];
  }
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  c->labels = (uint8_t*)malloc(n);
  if (!c->labels) return 2;
  rd(c->labels, 1, n);
  rd(&c->n_tines, 4, 1);
  if (c->n_tines < 0 || c->n_tines > 64) return 2;
  c->off = (int32_t*)malloc(sizeof(int32_t) * (size_t)(c->n_tines + 1));
  rd(c->off, 4, (size_t)c->n_tines + 1);
  const int n_points = c->off[c->n_tines];
  if (n_points < 0) return 2;
  c->pts = (double*)malloc(sizeof(double) * 3 * (size_t)(n_points > 0 ? n_points : 1));
  c->power = (double*)malloc(sizeof(double) * (size_t)(c->n_tines > 0 ? c->n_tines : 1));
  rd(c->pts, 8, 3 * (size_t)n_points);
  rd(c->power, 8, (size_t)c->n_tines);
  rd(&c->needle.sigma, 8, 1);
  rd(&c->dt, 8, 1);
  rd(&c->n_steps, 4, 1);
  fclose(in);
  c->needle.n_tines = c->n_tines;
  c->needle.pt_offset = c->off;
  c->needle.pts = c->pts;
  c->needle.power = c->power;
  return 0;
}

/* A grid with the case's tissue and needle. */
static int make_grid(const Case* c, rfa_grid* g) {
  *g = NULL;
  if (check(rfa_create_grid(c->nx, c->ny, c->nz, c->dx, c->dy, c->dz, &c->opt, g),
            "rfa_create_grid"))
    return 1;
  if (check(rfa_set_tissue(*g, c->labels, c->table, c->n_classes), "rfa_set_tissue")) return 1;
  return check(rfa_set_needle(*g, &c->needle), "rfa_set_needle");
}

static int run_step(const Case* c, FILE* out) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  rfa_grid g = NULL;
  rfa_diag diag;
  double* t = (double*)malloc(sizeof(double) * n);
  uint8_t* mask = (uint8_t*)malloc(n);
  float* omega = (float*)malloc(sizeof(float) * n);
  int bad = !t || !mask || !omega;
  if (!bad) bad = make_grid(c, &g);
  if (!bad) bad = check(rfa_step(g, c->n_steps, c->dt, &diag), "rfa_step");
  if (!bad) bad = check(rfa_get_temperature(g, t, NULL, NULL), "rfa_get_temperature");
  if (!bad) bad = check(rfa_damage(g, mask, omega, NULL), "rfa_damage");
  if (!bad) {
    const int64_t mono = diag.mono_violations;
    fwrite(t, sizeof(double), n, out);
    fwrite(mask, 1, n, out);
    fwrite(omega, sizeof(float), n, out);
    fwrite(&diag.energy_J, 8, 1, out);
    fwrite(&diag.injected_J, 8, 1, out);
    fwrite(&diag.residual_J, 8, 1, out);
    fwrite(&mono, 8, 1, out);
    printf("c driver: %dx%dx%d, %d steps, Tmax %.3f degC\n", c->nx, c->ny, c->nz, c->n_steps,
           diag.t_max_C);
  }
  if (g) rfa_destroy_grid(g);
  free(t);
  free(mask);
  free(omega);
  return bad;
}

static int run_batch(const Case* c, FILE* out) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  rfa_grid g[3] = {NULL, NULL, NULL};
  rfa_batch b = NULL;
  float* hi = (float*)malloc(sizeof(float) * 3 * n);
  float* lo = (float*)malloc(sizeof(float) * 3 * n);
  int bad = !hi || !lo;
  for (int i = 0; i < 3 && !bad; ++i) bad = make_grid(c, &g[i]);
  const double dts[2] = {c->dt, c->dt};
  if (!bad) bad = check(rfa_batch_create(2, g, dts, &b), "rfa_batch_create");
  if (!bad) bad = check(rfa_batch_step(b, c->n_steps, NULL), "rfa_batch_step");
  if (!bad) bad = check(rfa_step(g[2], c->n_steps, c->dt, NULL), "rfa_step");
  for (int i = 0; i < 3 && !bad; ++i)
    bad = check(rfa_get_temperature(g[i], NULL, hi + i * n, lo + i * n), "rfa_get_temperature");
  int32_t plan[6] = {0, 0, 0, 0, 0, 0};
  if (!bad)
    bad = check(rfa_batch_get_plan(b, &plan[0], &plan[1], &plan[2], &plan[3], &plan[4], &plan[5]),
                "rfa_batch_get_plan");
  if (!bad) {
    const int32_t equal = memcmp(hi, hi + n, 4 * n) == 0 && memcmp(hi, hi + 2 * n, 4 * n) == 0 &&
                          memcmp(lo, lo + n, 4 * n) == 0 && memcmp(lo, lo + 2 * n, 4 * n) == 0;
    fwrite(&equal, 4, 1, out);
    fwrite(plan, 4, 6, out);
    printf("c driver batch: %d steps, states equal %d, %d groups\n", c->n_steps, equal, plan[5]);
  }
  if (b) rfa_batch_destroy(b); /* the batch borrows the grids: destroy it first */
  for (int i = 0; i < 3; ++i)
    if (g[i]) rfa_destroy_grid(g[i]);
  free(hi);
  free(lo);
  return bad;
}

static int run_adjoint(const Case* c, FILE* out) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  enum { M = 4 };
  float ctrl[M * M * M];
  double dctrl[M * M * M];
  memset(ctrl, 0, sizeof ctrl);
  rfa_grid g = NULL;
  float* w = (float*)malloc(sizeof(float) * n);
  double* dP = (double*)malloc(sizeof(double) * (size_t)(c->n_tines > 0 ? c->n_tines : 1));
  int bad = !w || !dP;
  for (size_t i = 0; i < n && !bad; ++i) w[i] = 1.0f;
  if (!bad) bad = make_grid(c, &g);
  if (!bad) bad = check(rfa_set_perfusion_bspline(g, M, ctrl), "rfa_set_perfusion_bspline");
  if (!bad)
    bad = check(rfa_forward_checkpointed(g, c->n_steps, c->dt, c->n_steps / 3 + 1),
                "rfa_forward_checkpointed");
  if (!bad) bad = check(rfa_adjoint(g, w, dP, dctrl, NULL), "rfa_adjoint");
  if (!bad) {
    fwrite(dP, 8, (size_t)c->n_tines, out);
    fwrite(dctrl, 8, M * M * M, out);
    printf("c driver adjoint: %d steps, dL/dP[0] = %.6e\n", c->n_steps, dP[0]);
  }
  if (g) rfa_destroy_grid(g);
  free(w);
  free(dP);
  return bad;
}

int main(int argc, char** argv) {
  if (argc < 3 || argc > 4) {
    fprintf(stderr, "usage: %s input output [step|batch|adjoint]\n", argv[0]);
    return 2;
  }
  const char* mode = argc == 4 ? argv[3] : "step";
  Case c;
  memset(&c, 0, sizeof c);
  int rc = read_case(argv[1], &c);
  if (rc) return rc;
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  int bad;
  if (strcmp(mode, "step") == 0)
    bad = run_step(&c, out);
  else if (strcmp(mode, "batch") == 0)
    bad = run_batch(&c, out);
  else if (strcmp(mode, "adjoint") == 0)
    bad = run_adjoint(&c, out);
  else
    bad = 2;
  fclose(out);
  if (bad) remove(argv[2]);
  free(c.labels);
  free(c.off);
  free(c.pts);
  free(c.power);
  return bad;
}
