// Exercises every entry point of the CPU oracle on small grids (1D, 2D, 3D,
// odd boxes, all-zero and tiny states), built with the oracle's source by
// tests/test_sanitizers.py under the address and undefined-behaviour
// sanitizers: any out-of-bounds access, use after free, leak or undefined
// operation stops the program.  Prints "oracle sanitize OK" on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "oracle.h"

#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

static std::vector<double> state(long sites, unsigned seed) {
  std::vector<double> p(2 * sites);
  unsigned x = seed;
  for (auto &v : p) {
    x = x * 1664525u + 1013904223u;
    v = ((x >> 8) & 0xffff) / 65536.0 - 0.5;
  }
  return p;
}

static void one_grid(int dim, const int *n, const double *lo, const double *hi) {
  long sites = 1;
  for (int j = 0; j < dim; ++j) sites *= n[j];
  std::vector<double> V(sites);
  for (long s = 0; s < sites; ++s) V[s] = 0.01 * (double)(s % 7);
  std::vector<double> p = state(sites, 7u + (unsigned)sites);
  CHECK(orc_fft(p.data(), dim, n, 0) == 0);
  CHECK(orc_fft(p.data(), dim, n, 1) == 0);
  for (int ax = 0; ax < dim; ++ax) {
    CHECK(orc_fft_axis(p.data(), dim, n, ax, 0) == 0);
    CHECK(orc_fft_axis(p.data(), dim, n, ax, 1) == 0);
  }
  CHECK(orc_tssp_real(p.data(), dim, n, lo, hi, V.data(), 2.0, 1e-3, 3) == 0);
  CHECK(orc_tssp_real(p.data(), dim, n, lo, hi, nullptr, 2.0, -1e-3, 2) == 0);
  CHECK(orc_nonlinear_real(p.data(), dim, n, lo, hi, V.data(), 2.0, 5e-4) == 0);
  CHECK(orc_kinetic_real(p.data(), dim, n, lo, hi, 1e-3) == 0);
  for (int exact = 0; exact < 2; ++exact) {
    CHECK(orc_tssp_imag(p.data(), dim, n, lo, hi, V.data(), 3.0, 1e-3, 3, 1.0, exact) == 0);
    CHECK(orc_nonlinear_imag(p.data(), dim, n, lo, hi, V.data(), 3.0, 5e-4, exact) == 0);
    long steps = -1;
    double e = 0;
    const int rc = orc_ground_state(p.data(), dim, n, lo, hi, V.data(), 3.0, 1e-3, 1e-6, 2, 20,
                                    1.0, exact, &steps, &e);
    CHECK((rc == 0 || rc == 1) && steps >= 1 && steps <= 20 && std::isfinite(e));
  }
  double obs[10];
  CHECK(orc_observables(p.data(), dim, n, lo, hi, V.data(), 3.0, obs) == 0);
  for (double o : obs) CHECK(std::isfinite(o));
  double dk = 0;
  const int nb = orc_spectra_bins(dim, n, lo, hi, &dk);
  CHECK(nb > 0 && dk > 0);
  std::vector<double> a(nb), b(nb), c(nb), d(nb);
  CHECK(orc_spectra(p.data(), dim, n, lo, hi, nb, a.data(), b.data(), c.data(), d.data()) == 0);
  CHECK(orc_spectra(p.data(), dim, n, lo, hi, nb, nullptr, b.data(), nullptr, nullptr) == 0);
  // a state with zeros (the velocity guard) and the wrong bin count
  std::vector<double> z(2 * sites, 0.0);
  z[0] = 1.0;
  CHECK(orc_spectra(z.data(), dim, n, lo, hi, nb, a.data(), b.data(), c.data(), d.data()) == 0);
  CHECK(orc_spectra(z.data(), dim, n, lo, hi, nb + 1, a.data(), b.data(), c.data(), d.data()) < 0);
}

int main() {
  orc_set_threads(3);
  CHECK(orc_get_threads() == 3);
  const int n1[1] = {16};
  const double lo1[1] = {-4.0}, hi1[1] = {4.0};
  one_grid(1, n1, lo1, hi1);
  const int n2[2] = {8, 32};
  const double lo2[2] = {-3.0, -5.0}, hi2[2] = {3.0, 5.0};
  one_grid(2, n2, lo2, hi2);
  const int n3[3] = {4, 8, 16};
  const double lo3[3] = {0.0, -1.0, 2.0}, hi3[3] = {6.0, 1.0, 3.5};
  one_grid(3, n3, lo3, hi3);
  const int n2b[2] = {2, 2};
  const double lo2b[2] = {0.0, 0.0}, hi2b[2] = {1.0, 1.0};
  one_grid(2, n2b, lo2b, hi2b);
  // rejected arguments leave everything untouched
  std::vector<double> p = state(16, 3u);
  const int bad[1] = {12};
  CHECK(orc_fft(p.data(), 1, bad, 0) < 0);
  CHECK(orc_fft(nullptr, 1, n1, 0) < 0);
  CHECK(orc_tssp_imag(p.data(), 1, n1, lo1, hi1, nullptr, 1.0, 1e-3, 2, -1.0, 0) < 0);
  orc_set_threads(0);
  std::printf("oracle sanitize OK\n");
  return 0;
}
