/*
 * Plain FP64 CPU oracle for the time-splitting spectral (TSSP) solver of the
 * non-dimensional Gross-Pitaevskii equation (Numerical Scheme section, Eq. 2):
 *
 *     i d/dt psi = -1/2 lap psi + V psi + g |psi|^2 psi .
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (all functions):
 *   - psi is interleaved complex (re, im) FP64, row-major over n[0..dim-1],
 *     last axis contiguous.  dim is 1, 2 or 3; every n[j] is a power of two.
 *   - grid points x_{j,i} = lo[j] + i*h_j, h_j = (hi[j]-lo[j])/n[j]; periodic.
 *   - wavenumbers k_j = 2*pi*m_j/L_j with m_j = i (i < n/2) else i - n.
 *   - V is one FP64 value per site (NULL means V = 0).
 *   - Return value 0 on success, negative on bad arguments.
 *
 * Parity unpinned: none of the functions here (every function has a pin in
 * the CPU test suite).
 */
#ifndef GPE_ORACLE_H
#define GPE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Number of host threads used over independent FFT lines (<=0: all cores). */
void orc_set_threads(int nthreads);
int orc_get_threads(void);

/* Unnormalised forward DFT (sign -) or inverse DFT (sign +, times 1/N_tot)
 * over all axes, in place. */
int orc_fft(double *psi, int dim, const int *n, int inverse);

/* The same along one axis only (inverse carries 1/n[axis]). */
int orc_fft_axis(double *psi, int dim, const int *n, int axis, int inverse);

/* nsteps real-time Strang steps N(dt/2) K(dt) N(dt/2), unfused. */
int orc_tssp_real(double *psi, int dim, const int *n, const double *lo,
                  const double *hi, const double *V, double g, double dt,
                  long nsteps);

/* The two real-time substeps, for schedules built by the caller (the
 * time-dependent potential): N(tau) psi = exp(-i (V + g|psi|^2) tau) psi, and
 * K(dt) = forward transform, exp(-i |k|^2 dt / 2), inverse transform. */
int orc_nonlinear_real(double *psi, int dim, const int *n, const double *lo,
                       const double *hi, const double *V, double g, double tau);
int orc_kinetic_real(double *psi, int dim, const int *n, const double *lo,
                     const double *hi, double dt);

/* nsteps imaginary-time steps, each renormalised to norm_target.  exact = 0:
 * the N substeps hold the density at its start value (frozen); 1: they solve
 * d psi/d tau = -(V - mu + g|psi|^2) psi exactly, mu a running estimate of the
 * chemical potential (0 at the start of the call, then += log(c)/dt after
 * each step's renormalisation by c). */
int orc_tssp_imag(double *psi, int dim, const int *n, const double *lo,
                  const double *hi, const double *V, double g, double dt,
                  long nsteps, double norm_target, int exact);

/* One imaginary-time N(tau) substep (exact as above, with mu = 0). */
int orc_nonlinear_imag(double *psi, int dim, const int *n, const double *lo,
                       const double *hi, const double *V, double g, double tau,
                       int exact);

/* Imaginary-time ground state: step until the energy, evaluated every
 * check_every steps, changes by less than tol (absolute) from the previous
 * evaluation (the first evaluation compares against the initial state).
 * Returns 0 on convergence, 1 if max_steps was reached. */
int orc_ground_state(double *psi, int dim, const int *n, const double *lo,
                     const double *hi, const double *V, double g, double dt,
                     double tol, int check_every, long max_steps,
                     double norm_target, int exact, long *steps_done, double *energy);

/* out[0..10] = norm, energy, mu, e_kin, e_pot, e_int, sigma_0, sigma_1,
 * sigma_2, r_rms, (unused axes give sigma 0). */
int orc_observables(const double *psi, int dim, const int *n, const double *lo,
                    const double *hi, const double *V, double g, double *out);

/* Number of |k| shells and the shell width dk. */
int orc_spectra_bins(int dim, const int *n, const double *lo, const double *hi,
                     double *dk);

/* Shell sums of the particle number N(n), compressible, incompressible and
 * quantum-pressure kinetic energy.  Any output pointer may be NULL. */
int orc_spectra(const double *psi, int dim, const int *n, const double *lo,
                const double *hi, int nbins, double *n_k, double *e_comp,
                double *e_incomp, double *e_qp);

#ifdef __cplusplus
}
#endif
#endif
