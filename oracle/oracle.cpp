/*
 * Plain FP64 CPU oracle for the TSSP Gross-Pitaevskii solver.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark to check the GPU library.  It shares no
 * code with that library.  Everything here is written for obviousness, not
 * speed: an iterative radix-2 FFT with per-index libm twiddles, one site loop
 * per substep, no fusion.  The only concession to run time is std::thread over
 * independent FFT lines and over fixed chunks of sites (sums are taken per
 * fixed chunk and then added in chunk order, so results do not depend on the
 * thread count).
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * is silent the reading used is stated at the function.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <thread>
#include <vector>

namespace {

using cplx = std::complex<double>;
const double kPi = 3.14159265358979323846264338327950288;

int g_threads = 0;

int thread_count() {
  int t = g_threads;
  if (t <= 0) t = (int)std::thread::hardware_concurrency();
  return t <= 0 ? 1 : t;
}

/* Run f(i) for i in [0, count) over the host threads, static blocks.  Work
 * under 65536 sites runs on the calling thread. */
template <class F>
void parallel_for(long count, F f, long work) {
  int nt = thread_count();
  if (work < (1L << 16)) nt = 1;
  if (nt > count) nt = (int)std::max(1L, count);
  if (nt == 1) {
    for (long i = 0; i < count; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  long per = (count + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    long b = t * per, e = std::min(count, b + per);
    if (b >= e) break;
    pool.emplace_back([=, &f]() {
      for (long i = b; i < e; ++i) f(i);
    });
  }
  for (auto &th : pool) th.join();
}

struct Grid {
  int dim = 0;
  long n[3] = {1, 1, 1};
  long stride[3] = {1, 1, 1};
  long total = 1;
  double lo[3] = {0, 0, 0}, L[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  double dV = 1;
};

bool pow2(long v) { return v >= 2 && (v & (v - 1)) == 0; }

bool make_grid(int dim, const int *n, const double *lo, const double *hi,
               Grid &G) {
  if (dim < 1 || dim > 3 || !n) return false;
  G.dim = dim;
  G.total = 1;
  for (int j = 0; j < dim; ++j) {
    if (!pow2(n[j])) return false;
    G.n[j] = n[j];
    G.total *= n[j];
  }
  long s = 1;
  for (int j = dim - 1; j >= 0; --j) {
    G.stride[j] = s;
    s *= G.n[j];
  }
  G.dV = 1.0;
  for (int j = 0; j < dim; ++j) {
    double a = lo ? lo[j] : 0.0, b = hi ? hi[j] : 2 * kPi;
    if (!(b > a)) return false;
    G.lo[j] = a;
    G.L[j] = b - a;
    G.h[j] = G.L[j] / (double)G.n[j];
    G.dV *= G.h[j];
  }
  return true;
}

/* Index along axis j of flat site s. */
long axis_index(const Grid &G, long s, int j) { return (s / G.stride[j]) % G.n[j]; }

/* Signed integer wavenumber m for index i on an axis of n points. */
long signed_mode(long i, long n) { return i < n / 2 ? i : i - n; }

/* k_j = 2 pi m_j / L_j. */
double wavenumber(const Grid &G, long s, int j) {
  return 2 * kPi * (double)signed_mode(axis_index(G, s, j), G.n[j]) / G.L[j];
}

double coord(const Grid &G, long s, int j) {
  return G.lo[j] + (double)axis_index(G, s, j) * G.h[j];
}

double k_squared(const Grid &G, long s) {
  double k2 = 0;
  for (int j = 0; j < G.dim; ++j) {
    double k = wavenumber(G, s, j);
    k2 += k * k;
  }
  return k2;
}

/* ---------------------------------------------------------------------------
 * FFT.  The spectral method of the Numerical Scheme section needs the discrete
 * Fourier transform psi_hat(m) = sum_i psi(i) exp(-2 pi i m.i / n).  Textbook
 * iterative radix-2 decimation in time: bit-reversal permutation, then log2 n
 * butterfly levels.  Twiddles exp(sign 2 pi i j / m) are computed per index with
 * libm cos/sin (never by recurrence).
 * ------------------------------------------------------------------------- */
std::vector<cplx> twiddles(long m, int sign) {
  std::vector<cplx> w(m / 2);
  for (long j = 0; j < m / 2; ++j) {
    double a = 2 * kPi * (double)j / (double)m;
    w[j] = cplx(std::cos(a), sign * std::sin(a));
  }
  return w;
}

void fft_line(cplx *a, long m, const std::vector<cplx> &w) {
  /* bit reversal */
  for (long i = 1, j = 0; i < m; ++i) {
    long bit = m >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (long len = 2; len <= m; len <<= 1) {
    long half = len / 2, step = m / len;
    for (long b = 0; b < m; b += len) {
      for (long j = 0; j < half; ++j) {
        cplx t = w[j * step] * a[b + j + half];
        cplx u = a[b + j];
        a[b + j] = u + t;
        a[b + j + half] = u - t;
      }
    }
  }
}

/* One-dimensional transform of every line along axis `ax`. */
void fft_axis(cplx *psi, const Grid &G, int ax, bool inverse) {
  long m = G.n[ax], s = G.stride[ax];
  long lines = G.total / m;
  std::vector<cplx> w = twiddles(m, inverse ? +1 : -1);
  double scale = inverse ? 1.0 / (double)m : 1.0;
  int nt = G.total < (1L << 16) ? 1 : thread_count();
  long per = (lines + nt - 1) / nt;
  parallel_for(nt, [&](long t) {
    std::vector<cplx> buf(m);
    long b = t * per, e = std::min(lines, b + per);
    for (long l = b; l < e; ++l) {
      long outer = l / s, inner = l % s;
      cplx *base = psi + outer * m * s + inner;
      for (long i = 0; i < m; ++i) buf[i] = base[i * s];
      fft_line(buf.data(), m, w);
      for (long i = 0; i < m; ++i) base[i * s] = buf[i] * scale;
    }
  }, G.total);
}

void fft_all(cplx *psi, const Grid &G, bool inverse) {
  for (int ax = 0; ax < G.dim; ++ax) fft_axis(psi, G, ax, inverse);
}

/* Fixed chunking for sums: one chunk per line of the last axis. */
long chunk_len(const Grid &G) { return G.n[G.dim - 1]; }

/* sum_s f(s) with per-chunk partials added in chunk order. */
template <class F>
double chunked_sum(const Grid &G, F f) {
  long cl = chunk_len(G), nc = G.total / cl;
  std::vector<double> part(nc, 0.0);
  parallel_for(nc, [&](long c) {
    double acc = 0;
    for (long s = c * cl; s < (c + 1) * cl; ++s) acc += f(s);
    part[c] = acc;
  }, G.total);
  double tot = 0;
  for (double p : part) tot += p;
  return tot;
}

template <class F>
void for_sites(const Grid &G, F f) {
  long cl = chunk_len(G), nc = G.total / cl;
  parallel_for(nc, [&](long c) {
    for (long s = c * cl; s < (c + 1) * cl; ++s) f(s);
  }, G.total);
}

/* ---------------------------------------------------------------------------
 * TSSP substeps (Numerical Scheme section: the time-splitting spectral method
 * applied to Eq. 2; imaginary time replaces t by -i t).
 *
 * Reading (the paper does not print the splitting): Strang order
 * N(dt/2) K(dt) N(dt/2), after the TSSP scheme the paper cites.  The nonlinear
 * substep uses the density at the start of the substep (exact in real time,
 * where |psi| is unchanged by it; a frozen-density choice in imaginary time).
 * ------------------------------------------------------------------------- */

/* N(tau): psi <- exp(-i (V + g|psi|^2) tau) psi. */
void nonlinear_real(cplx *psi, const Grid &G, const double *V, double g,
                    double tau) {
  for_sites(G, [&](long s) {
    double rho = std::norm(psi[s]);
    double th = ((V ? V[s] : 0.0) + g * rho) * tau;
    psi[s] *= cplx(std::cos(th), -std::sin(th));
  });
}

/* K(dt) in Fourier space: psi_hat <- exp(-i |k|^2 dt / 2) psi_hat. */
void kinetic_real(cplx *psih, const Grid &G, double dt) {
  for_sites(G, [&](long s) {
    double ph = k_squared(G, s) * dt / 2;
    psih[s] *= cplx(std::cos(ph), -std::sin(ph));
  });
}

/* Imaginary-time N(tau): psi <- exp(-(V + g|psi|^2) tau) psi. */
void nonlinear_imag(cplx *psi, const Grid &G, const double *V, double g,
                    double tau) {
  for_sites(G, [&](long s) {
    double rho = std::norm(psi[s]);
    psi[s] *= std::exp(-((V ? V[s] : 0.0) + g * rho) * tau);
  });
}

/* Imaginary-time N(tau) solved exactly (the "exact" substep, an option: the
 * paper does not fix the substep) for the potential V - shift:
 * d psi/d tau = -(v + g|psi|^2) psi keeps the phase, and rho = |psi|^2 obeys
 * the Bernoulli equation
 *   d rho/d tau = -2 v rho - 2 g rho^2,
 * whose solution through 1/rho gives
 *   rho(tau) = rho0 e^{-2 v tau} / (1 + g rho0 (1 - e^{-2 v tau}) / v),
 * with (1 - e^{-2 v tau}) / v -> 2 tau at v = 0. */
void nonlinear_imag_exact(cplx *psi, const Grid &G, const double *V, double g,
                          double tau, double shift) {
  for_sites(G, [&](long s) {
    double rho = std::norm(psi[s]);
    double v = (V ? V[s] : 0.0) - shift;
    double e = v != 0.0 ? -std::expm1(-2.0 * v * tau) / v : 2.0 * tau;
    double rho_t = rho * std::exp(-2.0 * v * tau) / (1.0 + g * rho * e);
    psi[s] *= (rho > 0.0 ? std::sqrt(rho_t / rho) : 0.0);
  });
}

/* Imaginary-time K(dt): psi_hat <- exp(-|k|^2 dt / 2) psi_hat. */
void kinetic_imag(cplx *psih, const Grid &G, double dt) {
  for_sites(G, [&](long s) { psih[s] *= std::exp(-k_squared(G, s) * dt / 2); });
}

double norm_of(const cplx *psi, const Grid &G) {
  return G.dV * chunked_sum(G, [&](long s) { return std::norm(psi[s]); });
}

/* One real-time step: N(dt/2), forward FFT, K(dt), inverse FFT, N(dt/2). */
void real_step(cplx *psi, const Grid &G, const double *V, double g, double dt) {
  nonlinear_real(psi, G, V, g, dt / 2);
  fft_all(psi, G, false);
  kinetic_real(psi, G, dt);
  fft_all(psi, G, true);
  nonlinear_real(psi, G, V, g, dt / 2);
}

/* One imaginary-time step, then renormalisation to norm_target (the
 * wavefunction is normalised at every step of the ground-state method).
 * exact: the N substeps are solved exactly for V - mu, with mu a running
 * estimate of the chemical potential (0 at the first step of a run, then
 * mu += log(c) / dt from each step's renormalisation factor c): the norm then
 * stays near its target inside a step, so the second substep sees the
 * density of a normalised state; without the shift the state's decay within
 * the step biases mu at first order in dt. */
void imag_step(cplx *psi, const Grid &G, const double *V, double g, double dt,
               double norm_target, int exact, double *mu) {
  if (exact) {
    nonlinear_imag_exact(psi, G, V, g, dt / 2, *mu);
  } else {
    nonlinear_imag(psi, G, V, g, dt / 2);
  }
  fft_all(psi, G, false);
  kinetic_imag(psi, G, dt);
  fft_all(psi, G, true);
  if (exact) {
    nonlinear_imag_exact(psi, G, V, g, dt / 2, *mu);
  } else {
    nonlinear_imag(psi, G, V, g, dt / 2);
  }
  double c = std::sqrt(norm_target / norm_of(psi, G));
  for_sites(G, [&](long s) { psi[s] *= c; });
  if (exact) *mu += std::log(c) / dt;
}

/* ---------------------------------------------------------------------------
 * Observables.  r_rms is defined in the Results section (ground-state
 * validation); sigma_x/y/z are the axis rms sizes of the dynamics validation;
 * mu is the chemical potential of Table 1.  Reading (the paper prints neither
 * E nor mu): the energy functional whose variation gives Eq. 2,
 *   E = int 1/2 |grad psi|^2 + V |psi|^2 + g/2 |psi|^4,
 * and mu = (E_kin + E_pot + 2 E_int) / norm.  Sizes are measured from the
 * coordinate origin (uncentred), as the r_rms formula is written.
 * ------------------------------------------------------------------------- */
struct Obs {
  double norm, energy, mu, e_kin, e_pot, e_int, sigma[3], r_rms;
};

Obs observe(const cplx *psi, const Grid &G, const double *V, double g) {
  Obs o{};
  double s0 = chunked_sum(G, [&](long s) { return std::norm(psi[s]); });
  o.norm = G.dV * s0;
  o.e_pot = G.dV * chunked_sum(G, [&](long s) {
              return (V ? V[s] : 0.0) * std::norm(psi[s]);
            });
  o.e_int = 0.5 * g * G.dV * chunked_sum(G, [&](long s) {
              double r = std::norm(psi[s]);
              return r * r;
            });
  std::vector<cplx> ph(psi, psi + G.total);
  fft_all(ph.data(), G, false);
  o.e_kin = 0.5 * (G.dV / (double)G.total) *
            chunked_sum(G, [&](long s) { return k_squared(G, s) * std::norm(ph[s]); });
  o.energy = o.e_kin + o.e_pot + o.e_int;
  o.mu = (o.e_kin + o.e_pot + 2 * o.e_int) / o.norm;
  double r2 = 0;
  for (int j = 0; j < 3; ++j) {
    if (j >= G.dim) {
      o.sigma[j] = 0;
      continue;
    }
    double m2 = chunked_sum(G, [&](long s) {
      double x = coord(G, s, j);
      return x * x * std::norm(psi[s]);
    });
    o.sigma[j] = std::sqrt(m2 / s0);
    r2 += m2 / s0;
  }
  o.r_rms = std::sqrt(r2);
  return o;
}

/* ---------------------------------------------------------------------------
 * |k|-shell spectra (feature list: compressible and incompressible kinetic
 * energy spectra and the particle-number spectrum).  The paper names them
 * only.  Reading: the density-weighted velocity decomposition.  With
 * d_j psi = IDFT(i k_j psi_hat) and rho = |psi|^2,
 *   u_j = Im(conj(psi) d_j psi)/sqrt(rho),  w_j = Re(conj(psi) d_j psi)/sqrt(rho)
 * (both 0 where rho = 0), so |u|^2 + |w|^2 = |grad psi|^2 pointwise.  U = DFT(u)
 * splits into the compressible part k (k.U)/|k|^2 and the incompressible rest
 * (k = 0 goes to the incompressible part).  Shell sums, not densities:
 *   N(n)   = dV/N_tot  sum_{shell n} |psi_hat|^2
 *   E^c(n) = dV/(2 N_tot) sum |U^c|^2, E^i likewise, E^q from W = DFT(w).
 * Shell n of k: round(|k|/dk), dk = min_j 2 pi/L_j; for equal box lengths this
 * is taken in exact integer arithmetic on M = sum m_j^2.
 * ------------------------------------------------------------------------- */
bool equal_lengths(const Grid &G) {
  for (int j = 1; j < G.dim; ++j)
    if (std::fabs(G.L[j] - G.L[0]) > 1e-12 * G.L[0]) return false;
  return true;
}

double shell_width(const Grid &G) {
  double dk = 2 * kPi / G.L[0];
  for (int j = 1; j < G.dim; ++j) dk = std::min(dk, 2 * kPi / G.L[j]);
  return dk;
}

int shell_count(const Grid &G) {
  double dk = shell_width(G), q = 0;
  for (int j = 0; j < G.dim; ++j) {
    double kn = (double)(G.n[j] / 2) * (2 * kPi / G.L[j]) / dk;
    q += kn * kn;
  }
  return (int)std::floor(std::sqrt(q) + 0.5) + 1;
}

long shell_of(const Grid &G, long s, double dk) {
  if (equal_lengths(G)) {
    long M = 0;
    for (int j = 0; j < G.dim; ++j) {
      long m = signed_mode(axis_index(G, s, j), G.n[j]);
      M += m * m;
    }
    long r = (long)std::sqrt((double)M);
    while ((2 * r + 1) * (2 * r + 1) <= 4 * M) ++r;
    while (r > 0 && 4 * M < (2 * r - 1) * (2 * r - 1)) --r;
    return r;
  }
  return (long)std::floor(std::sqrt(k_squared(G, s)) / dk + 0.5);
}

}  // namespace

extern "C" {

void orc_set_threads(int nthreads) { g_threads = nthreads; }
int orc_get_threads(void) { return thread_count(); }

int orc_fft(double *psi, int dim, const int *n, int inverse) {
  Grid G;
  if (!psi || !make_grid(dim, n, nullptr, nullptr, G)) return -1;
  fft_all(reinterpret_cast<cplx *>(psi), G, inverse != 0);
  return 0;
}

int orc_fft_axis(double *psi, int dim, const int *n, int axis, int inverse) {
  Grid G;
  if (!psi || !make_grid(dim, n, nullptr, nullptr, G) || axis < 0 || axis >= dim)
    return -1;
  fft_axis(reinterpret_cast<cplx *>(psi), G, axis, inverse != 0);
  return 0;
}

int orc_tssp_real(double *psi, int dim, const int *n, const double *lo,
                  const double *hi, const double *V, double g, double dt,
                  long nsteps) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G) || nsteps < 0) return -1;
  cplx *p = reinterpret_cast<cplx *>(psi);
  for (long t = 0; t < nsteps; ++t) real_step(p, G, V, g, dt);
  return 0;
}

int orc_nonlinear_real(double *psi, int dim, const int *n, const double *lo,
                       const double *hi, const double *V, double g, double tau) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G)) return -1;
  nonlinear_real(reinterpret_cast<cplx *>(psi), G, V, g, tau);
  return 0;
}

int orc_kinetic_real(double *psi, int dim, const int *n, const double *lo,
                     const double *hi, double dt) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G)) return -1;
  cplx *p = reinterpret_cast<cplx *>(psi);
  fft_all(p, G, false);
  kinetic_real(p, G, dt);
  fft_all(p, G, true);
  return 0;
}

int orc_tssp_imag(double *psi, int dim, const int *n, const double *lo,
                  const double *hi, const double *V, double g, double dt,
                  long nsteps, double norm_target, int exact) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G) || nsteps < 0 || !(norm_target > 0))
    return -1;
  cplx *p = reinterpret_cast<cplx *>(psi);
  double mu = 0.0;
  for (long t = 0; t < nsteps; ++t) imag_step(p, G, V, g, dt, norm_target, exact, &mu);
  return 0;
}

int orc_nonlinear_imag(double *psi, int dim, const int *n, const double *lo,
                       const double *hi, const double *V, double g, double tau,
                       int exact) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G)) return -1;
  if (exact) {
    nonlinear_imag_exact(reinterpret_cast<cplx *>(psi), G, V, g, tau, 0.0);
  } else {
    nonlinear_imag(reinterpret_cast<cplx *>(psi), G, V, g, tau);
  }
  return 0;
}

int orc_ground_state(double *psi, int dim, const int *n, const double *lo,
                     const double *hi, const double *V, double g, double dt,
                     double tol, int check_every, long max_steps,
                     double norm_target, int exact, long *steps_done, double *energy) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G) || check_every < 1 || max_steps < 0 ||
      !(norm_target > 0))
    return -1;
  cplx *p = reinterpret_cast<cplx *>(psi);
  double e_prev = observe(p, G, V, g).energy;
  long t = 0;
  int rc = 1;
  double mu = 0.0;
  while (t < max_steps) {
    imag_step(p, G, V, g, dt, norm_target, exact, &mu);
    ++t;
    if (t % check_every == 0) {
      double e = observe(p, G, V, g).energy;
      bool done = std::fabs(e - e_prev) < tol;
      e_prev = e;
      if (done) {
        rc = 0;
        break;
      }
    }
  }
  if (steps_done) *steps_done = t;
  if (energy) *energy = observe(p, G, V, g).energy;
  return rc;
}

int orc_observables(const double *psi, int dim, const int *n, const double *lo,
                    const double *hi, const double *V, double g, double *out) {
  Grid G;
  if (!psi || !out || !make_grid(dim, n, lo, hi, G)) return -1;
  Obs o = observe(reinterpret_cast<const cplx *>(psi), G, V, g);
  out[0] = o.norm;
  out[1] = o.energy;
  out[2] = o.mu;
  out[3] = o.e_kin;
  out[4] = o.e_pot;
  out[5] = o.e_int;
  out[6] = o.sigma[0];
  out[7] = o.sigma[1];
  out[8] = o.sigma[2];
  out[9] = o.r_rms;
  return 0;
}

int orc_spectra_bins(int dim, const int *n, const double *lo, const double *hi,
                     double *dk) {
  Grid G;
  if (!make_grid(dim, n, lo, hi, G)) return -1;
  if (dk) *dk = shell_width(G);
  return shell_count(G);
}

int orc_spectra(const double *psi, int dim, const int *n, const double *lo,
                const double *hi, int nbins, double *n_k, double *e_comp,
                double *e_incomp, double *e_qp) {
  Grid G;
  if (!psi || !make_grid(dim, n, lo, hi, G)) return -1;
  if (nbins != shell_count(G)) return -2;
  const cplx *p = reinterpret_cast<const cplx *>(psi);
  const double dk = shell_width(G);
  const double w = G.dV / (double)G.total;
  std::vector<long> shell(G.total);
  for_sites(G, [&](long s) { shell[s] = shell_of(G, s, dk); });

  std::vector<cplx> ph(p, p + G.total);
  fft_all(ph.data(), G, false);
  std::vector<double> nk(nbins, 0.0), ec(nbins, 0.0), ei(nbins, 0.0), eq(nbins, 0.0);
  for (long s = 0; s < G.total; ++s) nk[shell[s]] += w * std::norm(ph[s]);

  /* U_j = DFT(u_j), W_j = DFT(w_j), one axis at a time. */
  std::vector<std::vector<cplx>> U(G.dim);
  for (int j = 0; j < G.dim; ++j) {
    std::vector<cplx> d(G.total);
    for_sites(G, [&](long s) { d[s] = cplx(0, wavenumber(G, s, j)) * ph[s]; });
    fft_all(d.data(), G, true);
    std::vector<cplx> u(G.total), wq(G.total);
    for_sites(G, [&](long s) {
      double rho = std::norm(p[s]);
      if (rho > 0) {
        cplx z = std::conj(p[s]) * d[s];
        double a = std::sqrt(rho);
        u[s] = cplx(z.imag() / a, 0);
        wq[s] = cplx(z.real() / a, 0);
      } else {
        u[s] = 0;
        wq[s] = 0;
      }
    });
    fft_all(u.data(), G, false);
    fft_all(wq.data(), G, false);
    for (long s = 0; s < G.total; ++s) eq[shell[s]] += 0.5 * w * std::norm(wq[s]);
    U[j] = std::move(u);
  }
  for (long s = 0; s < G.total; ++s) {
    double k[3] = {0, 0, 0}, k2 = 0;
    for (int j = 0; j < G.dim; ++j) {
      k[j] = wavenumber(G, s, j);
      k2 += k[j] * k[j];
    }
    double c_sum = 0, i_sum = 0;
    if (k2 > 0) {
      cplx kU = 0;
      for (int j = 0; j < G.dim; ++j) kU += k[j] * U[j][s];
      for (int j = 0; j < G.dim; ++j) {
        cplx uc = k[j] * kU / k2;
        c_sum += std::norm(uc);
        i_sum += std::norm(U[j][s] - uc);
      }
    } else {
      for (int j = 0; j < G.dim; ++j) i_sum += std::norm(U[j][s]);
    }
    ec[shell[s]] += 0.5 * w * c_sum;
    ei[shell[s]] += 0.5 * w * i_sum;
  }
  for (int b = 0; b < nbins; ++b) {
    if (n_k) n_k[b] = nk[b];
    if (e_comp) e_comp[b] = ec[b];
    if (e_incomp) e_incomp[b] = ei[b];
    if (e_qp) e_qp[b] = eq[b];
  }
  return 0;
}

}  // extern "C"
