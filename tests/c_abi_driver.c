/* Plain C99 client of librfa.so (include/rfa.h): reads a case from a binary
 * file, steps it on the GPU through the C ABI alone and writes the
 * temperature, damage mask and damage integral.  Built and run by
 * tests/test_gpu_c_abi.py, which writes the input and checks the output
 * against the FP64 oracle.
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
 * Output: float64 T[n] (degC), uint8 mask[n], float32 omega[n], then
 *   float64 energy_J, injected_J, residual_J; int64 mono_violations.
 * Exit status 0 on success; otherwise the failing call and
 * rfa_last_error() are printed to stderr. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../include/rfa.h"

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

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  in = fopen(argv[1], "rb");
  if (!in) return 2;
  int32_t nx, ny, nz, n_classes, n_tines, n_steps;
  double dx, dy, dz, dt, sigma;
  rfa_options opt;
  if (check(rfa_default_options(&opt), "rfa_default_options")) return 1;
  rd(&nx, 4, 1);
  rd(&ny, 4, 1);
  rd(&nz, 4, 1);
  rd(&dx, 8, 1);
  rd(&dy, 8, 1);
  rd(&dz, 8, 1);
  rd(&opt.t_death, 8, 1);
  rd(&opt.A, 8, 1);
  rd(&opt.Ea, 8, 1);
  rd(&opt.R, 8, 1);
  rd(&opt.omega_cap, 8, 1);
  rd(&n_classes, 4, 1);
  if (n_classes < 1 || n_classes > 16) return 2;
  rfa_tissue table[16];
  for (int i = 0; i < n_classes; ++i) {
    double v[6];
    int32_t f[2];
    rd(v, 8, 6);
    rd(f, 4, 2);
    table[i].k = v[0];
    table[i].rho = v[1];
    table[i].c = v[2];
    table[i].h_perf = v[3];
    table[i].q_met = v[4];
    table[i].t_fixed = v[5];
    table[i].fixed = f[0];
    table[i].tissue = f[1];
  }
  const size_t n = (size_t)nx * ny * nz;
  uint8_t* labels = (uint8_t*)malloc(n);
  if (!labels) return 2;
  rd(labels, 1, n);
  rd(&n_tines, 4, 1);
  if (n_tines < 0 || n_tines > 64) return 2;
  int32_t* off = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tines + 1));
  rd(off, 4, (size_t)n_tines + 1);
  const int n_points = off[n_tines];
  double* pts = (double*)malloc(sizeof(double) * 3 * (size_t)(n_points > 0 ? n_points : 1));
  double* power = (double*)malloc(sizeof(double) * (size_t)(n_tines > 0 ? n_tines : 1));
  rd(pts, 8, 3 * (size_t)n_points);
  rd(power, 8, (size_t)n_tines);
  rd(&sigma, 8, 1);
  rd(&dt, 8, 1);
  rd(&n_steps, 4, 1);
  fclose(in);

  rfa_grid g = NULL;
  int bad = check(rfa_create_grid(nx, ny, nz, dx, dy, dz, &opt, &g), "rfa_create_grid");
  if (!bad) bad = check(rfa_set_tissue(g, labels, table, n_classes), "rfa_set_tissue");
  rfa_needle nd;
  nd.n_tines = n_tines;
  nd.pt_offset = off;
  nd.pts = pts;
  nd.power = power;
  nd.sigma = sigma;
  if (!bad) bad = check(rfa_set_needle(g, &nd), "rfa_set_needle");
  rfa_diag diag;
  if (!bad) bad = check(rfa_step(g, n_steps, dt, &diag), "rfa_step");
  double* t = (double*)malloc(sizeof(double) * n);
  uint8_t* mask = (uint8_t*)malloc(n);
  float* omega = (float*)malloc(sizeof(float) * n);
  if (!bad) bad = check(rfa_get_temperature(g, t, NULL, NULL), "rfa_get_temperature");
  if (!bad) bad = check(rfa_damage(g, mask, omega, NULL), "rfa_damage");
  if (!bad) {
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    const int64_t mono = diag.mono_violations;
    fwrite(t, sizeof(double), n, out);
    fwrite(mask, 1, n, out);
    fwrite(omega, sizeof(float), n, out);
    fwrite(&diag.energy_J, 8, 1, out);
    fwrite(&diag.injected_J, 8, 1, out);
    fwrite(&diag.residual_J, 8, 1, out);
    fwrite(&mono, 8, 1, out);
    fclose(out);
    printf("c driver: %dx%dx%d, %d steps, Tmax %.3f degC\n", nx, ny, nz, n_steps, diag.t_max_C);
  }
  if (g) rfa_destroy_grid(g);
  free(labels);
  free(off);
  free(pts);
  free(power);
  free(t);
  free(mask);
  free(omega);
  return bad;
}
