/*
 * gpe.h -- C ABI of the MI355X time-splitting spectral (TSSP) solver for the
 * non-dimensional Gross-Pitaevskii equation (Numerical Scheme section, Eq. 2)
 *
 *     i d/dt psi = -1/2 lap psi + V psi + g |psi|^2 psi
 *
 * on a periodic box, in 1D, 2D or 3D, with real-time dynamics and the
 * imaginary-time ground-state method of the same section.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Grid: x_{j,i} = lo[j] + i*h_j, h_j = (hi[j]-lo[j])/n[j], periodic.  Every
 *    n[j] is a power of two in [8, 1024].  dim is 1, 2 or 3; only the first
 *    dim entries of n, lo and hi are read.
 *  - Layout: row-major over (n[0], n[1][, n[2]]), last axis contiguous,
 *    interleaved complex (re, im).  Host state buffers are FP64 whatever the
 *    context precision.
 *  - Wavenumbers: k_j = 2 pi m_j / L_j with m_j = i for i < n/2, else i - n.
 *  - Ownership: the library owns the context and all device memory it
 *    allocates.  Host pointers passed in are borrowed for the duration of the
 *    call and copied; outputs go to caller-owned buffers.
 *  - Streams: every call enqueues on the context stream (the one given to
 *    gpe_create, or a stream the library creates).  Calls that return host
 *    values synchronise that stream; gpe_evolve and gpe_set_state_device do
 *    not.
 *  - Errors: status codes only; nothing throws or aborts across the ABI.
 *    gpe_last_error() gives a message for the last failing call on a context.
 *  - Threads: a context is used by one host thread at a time.
 */
#ifndef GPE_H
#define GPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpe_ctx gpe_ctx; /* opaque, library-owned */

typedef enum {
  GPE_OK = 0,
  GPE_EINVAL = -1,       /* bad argument (shape, box, dt, null pointer) */
  GPE_ENOMEM = -2,       /* device allocation failed */
  GPE_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  GPE_ENOTCONV = -4,     /* ground state not converged within max_steps */
  GPE_ENONFINITE = -5,   /* a reduction met a NaN or Inf */
  GPE_EBUSY = -6,        /* result not ready */
  GPE_EUNSUPPORTED = -7, /* valid request outside what is built (e.g. n = 2048) */
  GPE_ECANCELED = -8     /* request cancelled before it finished */
} gpe_status;

typedef enum { GPE_FP64 = 0, GPE_FP32 = 1, GPE_FP32_STATE = 2 } gpe_precision;

/* Problem description (Eq. 2's grid, g and normalisation).  precision:
 * GPE_FP64; GPE_FP32, the state and the FFT in FP32 while phase arguments,
 * sums and the imaginary-time renormalisation stay FP64; GPE_FP32_STATE, the
 * state held in FP32 in device memory (half the bytes of FP64) and every
 * operation of a pass in FP64 (one FP32 rounding per pass, at the store).
 * norm_target is the value of dV * sum |psi|^2 that the ground-state method
 * renormalises to (1 when the particle number is absorbed in g). */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double lo[3], hi[3];
  double g;
  int32_t precision;
  double norm_target;
} gpe_desc;

/* Analytic harmonic trap V = 1/2 sum_j w_j^2 x_j^2 (the traps of the Results
 * section); costs no memory traffic. */
typedef struct {
  double w[3];
} gpe_harmonic;

/* Observables (Results section: r_rms and the axis rms sizes; Table 1: mu):
 *   norm  = dV sum |psi|^2
 *   e_kin = 1/2 dV/N sum |k|^2 |psi_hat|^2,  e_pot = dV sum V |psi|^2,
 *   e_int = g/2 dV sum |psi|^4,  energy = e_kin + e_pot + e_int,
 *   mu    = (e_kin + e_pot + 2 e_int) / norm,
 *   sigma[j]^2 = sum x_j^2 |psi|^2 / sum |psi|^2 (from the coordinate origin),
 *   r_rms^2 = sum_j sigma[j]^2. */
typedef struct {
  double norm, energy, mu, e_kin, e_pot, e_int, sigma[3], r_rms;
} gpe_obs;

/* |k|-shell spectra (feature list: particle-number, compressible and
 * incompressible kinetic-energy spectra).  Shell n collects the k with
 * round(|k|/dk) = n, dk = min_j 2 pi / L_j.  Values are shell sums:
 *   n_k[n]      = dV/N sum |psi_hat|^2
 *   e_comp[n]   = dV/(2N) sum |U^c|^2,  e_incomp[n] = dV/(2N) sum |U^i|^2,
 *   e_qp[n]     = dV/(2N) sum |W|^2,
 * with u = Im(conj(psi) grad psi)/|psi|, w = Re(conj(psi) grad psi)/|psi|,
 * U = DFT(u) split into k (k.U)/|k|^2 and the rest (k = 0 is incompressible).
 * The caller owns the arrays (nbins doubles each, any may be NULL); nbins must
 * equal gpe_spectra_bins(); dk is written by the library. */
typedef struct {
  int32_t nbins;
  double dk;
  double *n_k, *e_comp, *e_incomp, *e_qp;
} gpe_spectra;

/* Per-kernel-kind timing collected with HIP events while enabled.  A kind is
 * an operation on one axis ("step_x_fp64": fused TSSP pass along x; "fft_",
 * "obs_", "deriv_", "ifft_": the forward, read-only, derivative and inverse
 * passes used by observables, spectra and transforms). */
#define GPE_TIMING_KINDS 16
typedef struct {
  int32_t count;                       /* number of kinds reported */
  char name[GPE_TIMING_KINDS][32];     /* kind names */
  double total_ms[GPE_TIMING_KINDS];   /* summed event time */
  int64_t launches[GPE_TIMING_KINDS];  /* launches timed */
  double bytes[GPE_TIMING_KINDS];      /* algorithmic HBM bytes per launch */
} gpe_timing;

/* Create a context: validates desc, allocates the state and work buffers on
 * the current HIP device.  V_host (n sites of FP64, may be NULL) or V_an (may
 * be NULL) gives the potential; neither means V = 0; both is GPE_EINVAL.
 * hip_stream is a hipStream_t (NULL: the library creates its own).  The
 * state starts at zero.  On failure *out is NULL. */
gpe_status gpe_create(const gpe_desc *desc, const double *V_host,
                      const gpe_harmonic *V_an, void *hip_stream,
                      gpe_ctx **out);

/* Replace the potential (same rules as gpe_create).  Removes a separable or
 * time-dependent potential. */
gpe_status gpe_set_potential(gpe_ctx *ctx, const double *V_host,
                             const gpe_harmonic *V_an);

/* Separable analytic potential.  The feature list of the paper names
 * anharmonic traps, optical lattices and time-dependent potentials (the
 * V(r, t) of Eq. 2) without formulas; this is the family provided:
 *   V(r) = sum_j v_j(x_j),
 *   v_j(x) = 1/2 w_j^2 (x - c_j)^2 + a_j (x - c_j)^4 + s_j sin^2(q_j x + phi_j),
 * j < dim (later entries are ignored).  The passes read V as three per-axis
 * tables of n_j values: no per-site memory traffic. */
typedef struct {
  double w[3];        /* harmonic frequency w_j */
  double center[3];   /* trap centre c_j */
  double quartic[3];  /* anharmonic coefficient a_j */
  double lattice[3];  /* lattice depth s_j */
  double q[3];        /* lattice wavenumber q_j */
  double phase[3];    /* lattice phase phi_j */
} gpe_separable;

/* Static separable potential; replaces any earlier potential.  V NULL or a
 * non-finite entry: GPE_EINVAL. */
gpe_status gpe_set_separable(gpe_ctx *ctx, const gpe_separable *V);

/* Time-dependent separable potential V(r, t).  fn(t, out, user) fills the
 * parameters at time t; it runs on the calling host thread during library
 * calls and must not call the library for this context.  An N substep over
 * the time interval [ta, tb] applies exp(-i (V(r, (ta + tb)/2) + g|psi|^2)
 * (tb - ta)) (the midpoint rule keeps the splitting second order); two
 * fused half-steps apply the mean of their two midpoint potentials over the
 * full step, which equals the two half-steps applied one after the other.
 * Real time advances the context clock (gpe_evolve: t += nsteps dt); the
 * ground-state method and the observables use V at the current clock.
 * Non-finite parameters from fn stop the call with GPE_EINVAL.  fn = NULL
 * removes the potential (V = 0).  Replaces any earlier potential. */
typedef void (*gpe_potential_fn)(double t, gpe_separable *out, void *user);
gpe_status gpe_set_potential_fn(gpe_ctx *ctx, gpe_potential_fn fn, void *user);

/* The imaginary-time nonlinear substep of the ground-state method.  The
 * paper gives no formula; GPE_IMAG_FROZEN (the default) applies
 * exp(-(V + g|psi|^2) tau) with the density held at its value at the start
 * of the substep (this reproduces the paper's Table 1 values at its dt; the
 * chemical potential then carries an O(dt) bias).  GPE_IMAG_EXACT applies
 * the exact solution of d psi/d tau = -(V + g|psi|^2) psi, a Bernoulli
 * equation for |psi|^2:
 *   psi <- psi e^{-V tau} / sqrt(1 + g |psi|^2 (1 - e^{-2 V tau}) / V)
 * (2 tau in place of the fraction where V = 0), which leaves the splitting
 * error O(dt^2) in mu as well.  With g < 0 the exact substep has no solution
 * once g |psi|^2 (1 - e^{-2 V tau}) / V <= -1: the state turns non-finite.
 * Other values: GPE_EINVAL.  Batched server requests use the default. */
#define GPE_IMAG_FROZEN 0
#define GPE_IMAG_EXACT 1
gpe_status gpe_set_imag_method(gpe_ctx *ctx, int32_t method);

/* The context clock: 0 at creation; real-time steps advance it by dt.  It
 * only matters for a time-dependent potential. */
gpe_status gpe_set_time(gpe_ctx *ctx, double t);
gpe_status gpe_get_time(const gpe_ctx *ctx, double *t);

/* Copy a host FP64 state in (interleaved complex, n sites); synchronous. */
gpe_status gpe_set_state(gpe_ctx *ctx, const double *psi_host);

/* Copy a device state in from dptr (interleaved complex, src = GPE_FP64 for
 * FP64 or GPE_FP32 for FP32 values, n sites, device memory of the context's
 * device); enqueued on the stream. */
gpe_status gpe_set_state_device(gpe_ctx *ctx, const void *dptr, int32_t src);

/* Copy the state out to a host FP64 buffer (2 n doubles); synchronous. */
gpe_status gpe_get_state(gpe_ctx *ctx, double *psi_host_out);

/* Copy the state out to device memory as FP64 (dst = GPE_FP64) or FP32
 * (dst = GPE_FP32) values; enqueued. */
gpe_status gpe_get_state_device(gpe_ctx *ctx, void *dptr, int32_t dst);

/* Real-time TSSP (Numerical Scheme section): nsteps Strang steps
 * N(dt/2) K(dt) N(dt/2), with N(tau) psi = exp(-i (V + g|psi|^2) tau) psi in
 * real space and K(dt) = exp(-i |k|^2 dt / 2) in Fourier space.  Adjacent
 * half-steps N(dt/2) N(dt/2) are applied as one N(dt) (exact: N leaves |psi|
 * unchanged).  The state is a full-step state on return.  dt may be negative
 * (time reversal); dt = 0 or nsteps < 0 is GPE_EINVAL.  Asynchronous. */
gpe_status gpe_evolve(gpe_ctx *ctx, double dt, int64_t nsteps);

/* Real-time TSSP with an observable time series (the sigma(t), E(t) records
 * of the dynamics setups): nsteps steps in chunks of `every` (the last may be
 * shorter), and after each chunk the observables of the completed Strang step
 * in series[k], k < *count = ceil(nsteps/every).  The device never waits on
 * the host between chunks; one copy brings all records back at the end.  The
 * state equals that of gpe_evolve called once per chunk (a single
 * gpe_evolve over nsteps differs only by rounding: the chunk boundaries apply
 * N(dt/2) twice where it applies N(dt) once).  capacity: entries of series
 * (GPE_EINVAL if below ceil(nsteps/every)).  GPE_ENONFINITE if a record is
 * not finite (all records are still written). */
gpe_status gpe_evolve_record(gpe_ctx *ctx, double dt, int64_t nsteps, int32_t every,
                             gpe_obs *series, int64_t capacity, int64_t *count);

/* Imaginary-time ground state (Numerical Scheme section: t -> -i t with the
 * wavefunction normalised at every step).  Each step is
 * N_im(dt/2) K_im(dt) N_im(dt/2) followed by psi <- psi sqrt(norm_target /
 * (dV sum |psi|^2)), with N_im(tau) = exp(-(V + g|psi|^2) tau) (density taken
 * at the start of the substep) and K_im(dt) = exp(-|k|^2 dt / 2).  Every
 * check_every steps the energy is evaluated; the run stops at the first check
 * whose energy differs from the previous check (the first check: from the
 * starting state) by less than tol.  check_every = 0 runs exactly max_steps
 * steps with no checks and returns GPE_OK.  Otherwise returns GPE_OK on
 * convergence or GPE_ENOTCONV after max_steps.  steps_done and energy (the
 * last evaluated energy; NaN if none) may be NULL.  Synchronous. */
gpe_status gpe_ground_state(gpe_ctx *ctx, double dt, double tol,
                            int32_t check_every, int64_t max_steps,
                            int64_t *steps_done, double *energy);

/* Observables of the current state (see gpe_obs) and, if spec is not NULL,
 * the shell spectra (see gpe_spectra).  Synchronous.  GPE_ENONFINITE if a sum
 * is not finite.  With spec, the observables come out of the same sweep as
 * the spectra (E_kin from the full transform by Parseval's identity instead
 * of per-axis transforms), so they can differ from a call without spec in
 * the last bits (FP64), or by the FP32 rounding of the stored intermediate
 * transform (FP32 storage: about 1e-9 relative in E_kin). */
gpe_status gpe_observables(gpe_ctx *ctx, gpe_obs *out, gpe_spectra *spec);

/* Number of |k| shells for this context's grid. */
int32_t gpe_spectra_bins(const gpe_ctx *ctx);

/* Discrete Fourier transform of the state in place along the axes whose bit
 * is set in axis_mask (bit j = axis j): forward unnormalised (sign -), or
 * inverse with 1/n_j per axis (sign +).  The spectral building block of the
 * method, exposed for checking.  Asynchronous. */
gpe_status gpe_transform(gpe_ctx *ctx, int32_t axis_mask, int32_t inverse);

/* Wait for all work enqueued on the context stream. */
gpe_status gpe_synchronize(gpe_ctx *ctx);

/* Kernel timing with HIP events on the context stream: enable (1) or
 * disable (0) and reset; read the per-kind totals. */
gpe_status gpe_timing_enable(gpe_ctx *ctx, int32_t on);
gpe_status gpe_timing_read(gpe_ctx *ctx, gpe_timing *out);

/* Bytes of device memory the context holds. */
uint64_t gpe_device_bytes(const gpe_ctx *ctx);

/* HIP device ordinal the context was created on (the current device at
 * gpe_create); -1 for NULL.  Device pointers handed to the context
 * (gpe_set_state_device, gpe_get_state_device) must be on this device. */
int32_t gpe_device(const gpe_ctx *ctx);

/* The stream the context enqueues on (the caller's, or the private one the
 * library created when gpe_create got NULL). */
void *gpe_stream(const gpe_ctx *ctx);

/* Allocation-free steps, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  No context: psi_dev is the caller's device state (the layout
 * above, complex128 for GPE_FP64, complex64 for GPE_FP32 and
 * GPE_FP32_STATE; on the current HIP device), advanced in place on
 * hip_stream (NULL: the null stream), asynchronously.  imaginary = 0:
 * nsteps real-time steps, the same as gpe_evolve on a context of this desc
 * and trap (V = 0 if trap is NULL); imaginary = 1: nsteps renormalised
 * imaginary-time steps with the frozen-density substep, the same as
 * gpe_ground_state with check_every = 0.  The launch shapes are those of
 * the tuning table for desc, as for a new context.  The tables, partial sums
 * and renormalisation factor live in a device array of
 * GPE_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends; the call allocates nothing.  Calls on one
 * device share that array, so calls that overlap on one device (two host
 * threads, or two streams) race.  A grid whose buffers exceed the array
 * (imaginary time beyond about 512^3 sites) gets GPE_EUNSUPPORTED; bad
 * arguments GPE_EINVAL.  gpe_last_error(NULL) gives the message. */
#define GPE_NOALLOC_SCRATCH_BYTES (8u << 20)
gpe_status gpe_steps_noalloc(const gpe_desc *desc, const gpe_harmonic *trap, void *psi_dev,
                             int32_t imaginary, double dt, int64_t nsteps, void *hip_stream);

/* Message for the last failing call on ctx (ctx may be NULL: last failure of
 * gpe_create or gpe_steps_noalloc on this thread).  Never NULL. */
const char *gpe_last_error(const gpe_ctx *ctx);

void gpe_destroy(gpe_ctx *ctx);

/* ------------------------------------------------------------------------
 * Launch-shape tuning per shape class (dim, n, precision).  None of these
 * choices changes the arithmetic of a line, so results do not depend on them
 * except through the order of the axis passes (rounding only).  Contexts and
 * server classes created after an entry is set use it; earlier ones keep
 * their shapes.  The table is process-wide and thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t width[3];       /* strided axes (all but the last): columns per workgroup, 8 or 16,
                             for the step passes and transforms; the register-heavy
                             passes (closing phase, imaginary-time passes, batched
                             slots, spectral derivative) take 8 where 16 would put
                             1024 threads in a workgroup with FP64 arithmetic.  With
                             FP32 storage (GPE_FP32, GPE_FP32_STATE) and in-place
                             passes also 32: the plain step passes take tiles of 32
                             columns that go through the LDS as two 16-column halves
                             (the other passes take 16); with transpose = 1 also 4
                             (4-line tiles, axes of 128 points or more) */
  int32_t xcd_remap[3];   /* strided axes: 1 = each XCD takes a contiguous run of tiles */
  int32_t pass_order[3];  /* the axes (0 = slowest) in the order a step visits them */
  int32_t plan[3];        /* radix plan per axis: 0 default; 1 the alternative (1024
                             points only: stages 8, 8, 8, 2 with 8 points per thread
                             instead of 16, 8, 8 with 16) */
  int32_t stream[3];      /* per axis, the step passes' non-temporal (streaming)
                             cache policy: bit 0 loads, bit 1 stores (0..3) */
  int32_t transpose;      /* 3D grids of more than 2^20 sites: 1 = the step passes
                             rotate the grid.  Each reads whole lines of its axis and
                             writes them, as rows of width[axis] sites, to a second
                             state array (allocated on first use) in the layout the
                             next pass reads; the axes go in the order 2, 0, 1, so
                             that every step starts and ends in the stored layout.
                             width, xcd_remap and stream then describe the rotating
                             passes on all three axes; the read-only passes
                             (observables, transforms, spectra) take the class's
                             defaults, in pass_order.  0 = in-place passes */
  double ms_per_step;     /* measured real-time step (gpe_autotune), else 0 */
} gpe_tuning;             /* entries beyond dim (and width/xcd_remap of the last axis
                             unless transpose) are 0 */

/* Time the real-time step of this shape class on the current device: per
 * axis every radix plan x width x tile order x streaming policy, then every
 * pass order, then the per-axis choices again (coordinate descent from the
 * current entry or the defaults; `steps` timed
 * steps per candidate, the minimum of three runs; a candidate must be more
 * than 1% faster than the incumbent to replace it), record the result in the
 * table and copy it to *out (nullable).  On 3D grids of more than 2^20 sites
 * the rotating step passes (transpose = 1) are searched the same way from
 * 8-column tiles and kept when faster.  With GPE_TUNE_VERBOSE=1 in the
 * environment every candidate and its time go to stderr.  Allocates a scratch context of the
 * class for the duration of the call.  g, box and norm_target of desc are not
 * used. */
gpe_status gpe_autotune(const gpe_desc *desc, int32_t steps, gpe_tuning *out);

/* Set (validated; GPE_EINVAL on a bad entry) or read the entry of a class.
 * gpe_tuning_get returns the defaults with *found = 0 when there is none. */
gpe_status gpe_tuning_set(const gpe_desc *desc, const gpe_tuning *t);
gpe_status gpe_tuning_get(const gpe_desc *desc, gpe_tuning *out, int32_t *found);
void gpe_tuning_clear(void);

/* Save the table as JSON / merge a saved table into it (all entries are
 * validated before any is applied; GPE_EINVAL on a malformed file). */
gpe_status gpe_tuning_save(const char *path);
gpe_status gpe_tuning_load(const char *path);

/* ------------------------------------------------------------------------
 * Serving: a request scheduler over one GPU (no counterpart in the paper,
 * which solves one problem per run).  Independent solves of the problems
 * above are submitted from any host thread; a scheduler thread admits them in
 * arrival order while the HBM budget allows and a slot of their shape class
 * (dim, n, precision, box, dt, real or imaginary time) is free, and runs in rounds: each round gives
 * every shape class with running requests one chunk of batched steps (all its
 * slots in the same launches), sized so that each running request receives
 * about the same GPU time per round (1 ms), and finishes the requests that
 * the previous round completed while the GPU runs the current one.  Requests
 * of any size mix; each one's arithmetic does not depend on what else runs,
 * nor on how its steps are cut into chunks.  Requests of 2^23 grid points or
 * more (the heavy tier) run first come, first served among themselves, one
 * at a time, beside the lighter requests: a heavy request waiting for the
 * tier does not hold back the requests queued behind it.  Environment
 * settings read at gpe_server_create: GPE_SERVER_HEAVY_SITES (tier
 * threshold, 0 turns the tier off), GPE_SERVER_HEAVY_ACTIVE (heavy requests
 * running at once), GPE_SERVER_HEAVY_WEIGHT (GPU time per round of a heavy
 * request, in light-request quanta; default 1), GPE_SERVER_HEAVY_SHARE
 * (0 <= f < 1: the heavy tier keeps at least that fraction of each round;
 * default 0), GPE_SERVER_QUANTUM_MS (GPU time per running request per
 * round; default 1), GPE_SERVER_HEAVY_BESIDE (1, the default: heavy
 * requests run on a stream of their own, concurrently with the lighter
 * classes, each chunk lasting about as long as the lighter classes' round;
 * 0: they take their quanta in turn with the others), GPE_SERVER_ONCHIP
 * (0 routes no class to the on-chip kernel) and GPE_SERVER_ONCHIP_MAX_N
 * (largest square 2D edge routed there, default 64; the kernel itself holds
 * up to 64 in FP64 and 128 in FP32).
 *
 * Beyond the request/poll/cancel calls a plain submit-and-wait interface
 * needs, this interface adds: max_active and chunk_steps at creation,
 * keep_state in a request (a result carries observables; the final state
 * only when asked for), the final state as a separate poll argument
 * (caller-owned, so a result record holds no pointer), release of finished
 * records, wait_idle, statistics, and gpe_request_bytes for capacity
 * planning.
 * ---------------------------------------------------------------------- */
typedef struct gpe_server gpe_server; /* opaque, library-owned */

typedef struct {
  gpe_desc desc;          /* grid, box, g, precision, norm_target */
  gpe_harmonic trap;      /* analytic harmonic potential (all zero: V = 0) */
  const double *psi0;     /* initial state, host FP64 (copied at submit) */
  int32_t mode;           /* 0: real-time evolution, 1: imaginary time */
  double dt;              /* > 0 */
  int64_t nsteps;         /* steps to run (imaginary time: fixed count, renormalised each step) */
  int32_t keep_state;     /* 1: keep the final state for gpe_server_poll */
} gpe_request;

typedef struct {
  gpe_status status;      /* GPE_OK, GPE_ENONFINITE, GPE_ECANCELED, GPE_ENOMEM, ... */
  gpe_obs obs;            /* observables of the final state */
  double t_submit, t_start, t_done;  /* seconds on the server's clock */
  int64_t steps_done;
} gpe_result;

typedef struct {
  int64_t submitted, completed, running, queued;
  double busy_seconds;            /* wall time with at least one request running */
  double site_steps;              /* sum over completed requests of sites x steps */
  uint64_t bytes_in_use;          /* HBM held for admitted requests */
} gpe_server_stats;

/* Create a server on the current HIP device.  hbm_budget_bytes caps the
 * device memory of admitted requests (0: the device's free memory);
 * max_slots is the slot count of each shape class (1..256, else
 * GPE_EUNSUPPORTED); max_active caps the requests running at once over all
 * classes (0: no cap; 1: one at a time); chunk_steps (>= 1) is the length of
 * the step graph replayed for small grids, whose chunks are whole replays. */
gpe_status gpe_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t max_active,
                             int32_t chunk_steps, gpe_server **out);

/* Queue a request (validated now; GPE_EINVAL etc. on bad input, GPE_ENOMEM if
 * it could never fit the budget, GPE_EUNSUPPORTED for dim = 1: the batched
 * classes are 2D and 3D).  The initial state is copied.  *id names it. */
gpe_status gpe_server_submit(gpe_server *srv, const gpe_request *req, uint64_t *id);

/* GPE_EBUSY while the request is queued or running; otherwise fills *out and,
 * if psi_out is not NULL and the request kept its state, copies the final
 * state (host FP64).  A finished request can be polled any number of times. */
gpe_status gpe_server_poll(gpe_server *srv, uint64_t id, gpe_result *out, double *psi_out);

/* Cancel a queued or running request (finishes with GPE_ECANCELED, without
 * observables or final state). */
gpe_status gpe_server_cancel(gpe_server *srv, uint64_t id);

/* Drop the record of a finished request, with its stored final state (a
 * server keeps every finished request until it is released or the server is
 * destroyed).  GPE_EBUSY while the request is queued or running, GPE_EINVAL
 * for an unknown id. */
gpe_status gpe_server_release(gpe_server *srv, uint64_t id);
/* Block until no request is queued or running. */
gpe_status gpe_server_wait_idle(gpe_server *srv);

gpe_status gpe_server_stats_read(gpe_server *srv, gpe_server_stats *out);

/* Device bytes the server charges against its budget for a request of this
 * shape: *class_b once per shape class (server created with max_slots), and
 * *slot_b per running request (its state, partials and tables). */
gpe_status gpe_request_bytes(const gpe_desc *desc, int32_t max_slots, uint64_t *class_b,
                             uint64_t *slot_b);

/* Stop the scheduler (requests still queued or running are cancelled). */
void gpe_server_destroy(gpe_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GPE_H */
