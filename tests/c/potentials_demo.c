/* A plain C99 caller of the potential and ground-state options: a 1D moving
 * harmonic trap through a time-dependent potential callback, the exact
 * imaginary-time substep, and a static optical lattice in 2D.  Prints:
 *   <x> at t = 2 in the moving trap, the closed form it should follow,
 *   mu of the 1D ground state (g = 10) with the exact substep,
 *   E of the 2D lattice ground state (g = 0). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gpe.h"

typedef struct {
  double amp, freq;
} trap_motion;

static void moving_trap(double t, gpe_separable *out, void *user) {
  const trap_motion *m = (const trap_motion *)user;
  memset(out, 0, sizeof *out);
  out->w[0] = 1.0;
  out->center[0] = m->amp * sin(m->freq * t);
}

static gpe_ctx *make(int dim, const int *n, const double *lo, const double *hi, double g) {
  gpe_desc d;
  memset(&d, 0, sizeof d);
  d.dim = dim;
  for (int j = 0; j < 3; ++j) d.n[j] = 1;
  for (int j = 0; j < dim; ++j) {
    d.n[j] = n[j];
    d.lo[j] = lo[j];
    d.hi[j] = hi[j];
  }
  d.g = g;
  d.precision = GPE_FP64;
  d.norm_target = 1.0;
  gpe_ctx *ctx = NULL;
  if (gpe_create(&d, NULL, NULL, NULL, &ctx) != GPE_OK) {
    printf("create failed: %s\n", gpe_last_error(NULL));
    exit(1);
  }
  return ctx;
}

static int check(gpe_ctx *ctx, gpe_status st, const char *what) {
  if (st == GPE_OK) return 0;
  printf("%s failed (%d): %s\n", what, (int)st, gpe_last_error(ctx));
  return 1;
}

int main(void) {
  /* 1D moving trap */
  const int n1[1] = {256};
  const double lo1[1] = {-10.0}, hi1[1] = {10.0};
  gpe_ctx *c1 = make(1, n1, lo1, hi1, 5.0);
  double *psi = calloc(2 * 256, sizeof(double));
  const double h = 20.0 / 256;
  for (int i = 0; i < 256; ++i) {
    const double x = -10.0 + i * h;
    psi[2 * i] = exp(-x * x / 2);
  }
  trap_motion m = {0.5, 2.0};
  int bad = check(c1, gpe_set_state(c1, psi), "set_state");
  bad |= check(c1, gpe_set_potential_fn(c1, moving_trap, &m), "set_potential_fn");
  bad |= check(c1, gpe_evolve(c1, 1e-3, 2000), "evolve");
  bad |= check(c1, gpe_get_state(c1, psi), "get_state");
  double t = 0, sx = 0, s0 = 0;
  bad |= check(c1, gpe_get_time(c1, &t), "get_time");
  for (int i = 0; i < 256; ++i) {
    const double x = -10.0 + i * h, r = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    sx += x * r;
    s0 += r;
  }
  const double W = m.freq;
  const double xk = m.amp / (1 - W * W) * (sin(W * t) - W * sin(t));
  printf("%.12f %.12f\n", sx / s0, xk);

  /* 1D ground state with the exact imaginary-time substep (a fresh context:
   * g = 10, trap w = 1) */
  gpe_ctx *c2 = make(1, (const int[]){128}, lo1, hi1, 10.0);
  gpe_harmonic trap = {{1.0, 0.0, 0.0}};
  const double h2 = 20.0 / 128;
  for (int i = 0; i < 128; ++i) {
    const double x = -10.0 + i * h2;
    psi[2 * i] = exp(-x * x / 2);
    psi[2 * i + 1] = 0;
  }
  int64_t steps = 0;
  double energy = 0;
  gpe_obs o;
  bad |= check(c2, gpe_set_potential(c2, NULL, &trap), "set_potential");
  bad |= check(c2, gpe_set_imag_method(c2, GPE_IMAG_EXACT), "set_imag_method");
  bad |= check(c2, gpe_set_state(c2, psi), "set_state");
  bad |= check(c2, gpe_ground_state(c2, 4e-3, 1e-15, 10, 400000, &steps, &energy), "ground");
  bad |= check(c2, gpe_observables(c2, &o, NULL), "observables");
  printf("%.12f\n", o.mu);

  /* 2D lattice s sin^2(x) on [0, 2 pi) x [-3, 3), g = 0 */
  const int n3[2] = {64, 16};
  const double lo3[2] = {0.0, -3.0}, hi3[2] = {6.283185307179586, 3.0};
  gpe_ctx *c3 = make(2, n3, lo3, hi3, 0.0);
  gpe_separable lat;
  memset(&lat, 0, sizeof lat);
  lat.lattice[0] = 2.0;
  lat.q[0] = 1.0;
  double *flat = calloc(2 * 64 * 16, sizeof(double));
  for (int i = 0; i < 64 * 16; ++i) flat[2 * i] = 1.0;
  bad |= check(c3, gpe_set_separable(c3, &lat), "set_separable");
  bad |= check(c3, gpe_set_state(c3, flat), "set_state");
  bad |= check(c3, gpe_ground_state(c3, 1e-3, 1e-14, 10, 200000, &steps, &energy), "ground");
  printf("%.12f\n", energy);

  free(psi);
  free(flat);
  gpe_destroy(c1);
  gpe_destroy(c2);
  gpe_destroy(c3);
  return bad;
}
