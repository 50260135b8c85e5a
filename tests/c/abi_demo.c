/* A plain C99 caller of the library: 2D harmonic-trap ground state, then real
 * time, through include/gpe.h only (no Python).  Prints one line of numbers:
 * status, steps, energy, mu, norm after 100 real-time steps. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "gpe.h"

int main(void) {
  gpe_desc d = {0};
  d.dim = 2;
  d.n[0] = 64;
  d.n[1] = 64;
  d.n[2] = 1;
  for (int j = 0; j < 2; ++j) {
    d.lo[j] = -8.0;
    d.hi[j] = 8.0;
  }
  d.g = 12.5484;
  d.precision = GPE_FP64;
  d.norm_target = 1.0;
  gpe_harmonic trap = {{1.0, 1.0, 0.0}};
  gpe_ctx *ctx = NULL;
  gpe_status st = gpe_create(&d, NULL, &trap, NULL, &ctx);
  if (st != GPE_OK) {
    printf("create %d %s\n", (int)st, gpe_last_error(NULL));
    return 1;
  }
  const int n = 64 * 64;
  double *psi = malloc(2 * (size_t)n * sizeof(double));
  const double h = 16.0 / 64;
  for (int i = 0; i < 64; ++i)
    for (int j = 0; j < 64; ++j) {
      const double x = -8.0 + i * h, y = -8.0 + j * h;
      psi[2 * (i * 64 + j)] = exp(-(x * x + y * y) / 2);
      psi[2 * (i * 64 + j) + 1] = 0.0;
    }
  st = gpe_set_state(ctx, psi);
  int64_t steps = 0;
  double energy = 0;
  if (st == GPE_OK) st = gpe_ground_state(ctx, 1e-3, 1e-10, 10, 100000, &steps, &energy);
  gpe_obs gs = {0}, rt = {0};
  if (st == GPE_OK) st = gpe_observables(ctx, &gs, NULL);
  if (st == GPE_OK) st = gpe_evolve(ctx, 1e-3, 100);
  if (st == GPE_OK) st = gpe_observables(ctx, &rt, NULL);
  printf("%d %lld %.12f %.12f %.15f\n", (int)st, (long long)steps, energy, gs.mu, rt.norm);
  free(psi);
  gpe_destroy(ctx);
  return st == GPE_OK ? 0 : 1;
}
