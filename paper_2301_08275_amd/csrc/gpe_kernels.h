// Internal interface between the host runtime (gpe.cpp) and the HIP kernels
// (axis_pass.hip, reduce.hip, spectra.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gpe {

// What an axis pass does before its forward transform (pre), between the
// transforms (mid) and after the inverse transform (post).
enum PhaseOp : int {
  PH_NONE = 0,
  PH_REAL = 1,  // psi <- exp(-i (V + g|psi|^2) tau) psi
  PH_IMAG = 2,  // psi <- exp(-(V + g|psi|^2) tau) psi   (pre: after psi <- c psi)
  PH_DERIV = 3, // post only: d = result, p = src at the site:
                //   out = (Im(conj(p) d) + i Re(conj(p) d)) / |p|  (0 where p = 0)
  PH_IMAG_EXACT = 4,  // the exact solution of d psi/d tau = -(V + g|psi|^2) psi:
                      //   psi <- psi e^{-V tau} / sqrt(1 + g|psi|^2 E),
                      //   E = (1 - e^{-2 V tau}) / V  (2 tau at V = 0)
};

enum MidOp : int {
  MID_NONE = 0,   // forward and inverse with nothing in between (identity)
  MID_TABLE = 1,  // multiply the spectrum by a per-frequency complex table
};

// Reduction slots written per workgroup when the matching flag is set.
enum RedFlag : int {
  RED_NONE = 0,
  RED_NORM_OUT = 1,  // sum |psi_out|^2                           (1 value)
  RED_KIN = 2,       // sum w[f] |psi_hat|^2 after the forward FFT (1 value)
  RED_REAL = 4,      // sums over the (pre-op) input: |psi|^2, V|psi|^2, |psi|^4,
                     // x0^2|psi|^2, x1^2|psi|^2, x2^2|psi|^2     (6 values)
};
constexpr int kRedSlots = 8;  // partial[wg * kRedSlots + slot]
constexpr int kSlotNormOut = 0, kSlotKin = 1, kSlotReal = 2;

enum VKind : int { V_NONE = 0, V_ARRAY = 1, V_HARMONIC = 2, V_TABLES = 3 };

// One request of a batched shape class (device-resident).  Batched passes
// launch one grid row (blockIdx.y) per slot; a slot whose mode is SLOT_FREE or
// whose steps are done costs its blocks an early return, so slots can be
// filled and emptied without changing the launch.
enum SlotMode : int { SLOT_FREE = 0, SLOT_REAL = 1, SLOT_IMAG = 2 };
struct Slot {
  void *psi;          // state (class precision)
  double g;
  double hv[3];       // analytic potential V = sum_j hv[j] x_j^2 (3D view)
  int mode;           // SlotMode
  int steps_total;
  int steps_done;     // advanced once per step by the slot update kernel
  int pad;
  double scale;       // imaginary time: renormalisation factor for the next step
  double norm_target;
};
// slot_pass bits for batched passes: first pass of a step, last pass of a step.
constexpr int SLOT_PASS_FIRST = 1, SLOT_PASS_LAST = 2;

struct PassArgs {
  const void *src;  // complex T, whole grid
  void *dst;        // complex T, whole grid (may equal src)
  int n[3];         // grid as 3D (2D problems use n[0] = 1)
  int axis;         // transformed axis (0, 1 or 2)
  int forward;      // 1: run forward stages on input; 0: input is a spectrum
  int inverse;      // 1: run inverse stages; 0: store the spectrum (natural order)
  int store;        // 0: read-only pass (reductions only)
  int refwd;        // 1 (generic mode): after the post op, transform forward again along
                    // the axis and store that spectrum (natural order)
  int pre, post, mid, red;
  double tau_pre, tau_post, g;
  int vkind;          // V_NONE, V_ARRAY (V below) or V_HARMONIC (hv below)
  int wreq;           // columns per workgroup requested for a strided axis (8 or 16)
  int plan;           // radix plan of the axis (0 default, 1 alternative)
  int xcd_remap;      // strided axes: give each XCD a contiguous run of tiles
  int trans;          // 1: rotating pass (3D; src and dst distinct): the input holds
                      // the grid as [b][c][a] (a = axis, b = (a+1)%3, c = (a+2)%3,
                      // last index fastest), the output as [c][a][b]; a tile is W
                      // whole lines at consecutive b, written as rows of W sites
  const double *V;    // FP64 potential per site, or null
  double hv[3];       // analytic V = sum_j hv[j] x_j^2 when V is null
  const double *vtab; // V_TABLES: V = t[j0] + t[n0 + j1] + t[n0 + n1 + j2] (view axes)
  const double *vtab_post;  // V_TABLES tables of the post phase when it differs from
                            // the pre phase's in the same pass (null: vtab)
  double lo[3], h[3]; // coordinates x_j = lo[j] + i h[j] (3D indexing)
  const void *tw;     // twiddles exp(-2 pi i j / N), j < N, complex T
  const void *mtab;   // mid table (complex T, N entries) for MID_TABLE
  const double *kw;   // RED_KIN weights per frequency (N doubles)
  const double *scale;  // PH_IMAG pre: psi <- (*scale) psi (null: 1)
  const double *mu_shift;  // PH_IMAG_EXACT: the substeps use V - *mu_shift (null: 0)
  int stream;         // step passes: non-temporal loads (bit 0) and stores (bit 1), tuned per axis
  double *partial;      // reductions, kRedSlots doubles per workgroup
  // batched shape class (MODE_SLOTS): per-slot state and operations
  Slot *slots;
  const int *slot_map;  // grid row -> slot index (null: row = slot)
  int nslots;           // grid rows (blockIdx.y) of a batched launch
  int slot_pass;        // SLOT_PASS_FIRST | SLOT_PASS_LAST bits
  int slot_step;        // step of this launch within the chunk: slot step = steps_done + slot_step
  int slot_imag;        // class mode: 0 real time, 1 imaginary time
  double dt;
  const void *mtab_imag;  // imaginary-time kinetic table of the class
};

struct PassShape {
  int N;        // axis length
  bool strided; // tiles of W columns (the axis is not the contiguous one, or the pass rotates)
  int W;        // lines (contiguous) or columns (strided) per workgroup
  int threads;  // workgroup size
  long long blocks;
};

// Launch geometry the kernels are built for (must match the template choice).
// plan: 0 the default radix plan of the axis length, 1 the alternative
// (only 1024 points has one; elsewhere 1 means 0).
// wreq: columns (or rotating lines) per tile, 8 or 16; 32 gives the plain
// in-place step pass of an FP32-storage strided axis tiles of two 16-column
// halves (PassShape::W = 32; other passes use 16); 4 gives rotating passes on
// axes of 128 points or more 4-line tiles.
// narrow: the pass runs one of the register-heavy operation sets (closing
// real-time phase, imaginary-time pre and post passes, batched slots, the
// spectral derivative, generic; also the exact imaginary-time pre pass, which
// is compute-bound there).  Where a 16-column strided tile would take
// 1024 threads (128 VGPRs each) with FP64 arithmetic or 16 points per thread,
// those kernels take 8-column tiles (measured faster; the generic and
// derivative sets would also spill).  Block counts with narrow = true are
// never smaller than without.
// trans: the rotating form of the pass (PassArgs::trans; 3D only): tiles of
// W whole lines of the axis at consecutive positions of the next axis.
PassShape pass_shape(int precision, const int n[3], int axis, int wreq, int plan = 0,
                     bool narrow = false, bool trans = false);
// The shape launch_axis_pass uses for these arguments; the partial sums of a
// reducing pass have one row per block of this shape.
PassShape launch_shape(int precision, const PassArgs &a);
inline bool plan_available(int n, int plan) { return plan == 0 || (plan == 1 && n == 1024); }

// Launch one axis pass; precision 0 = FP64, 1 = FP32, 2 = FP32 state.
hipError_t launch_axis_pass(int precision, const PassArgs &a, hipStream_t s);

// Sum `count` partial blocks of kRedSlots doubles in fixed order into
// out[kRedSlots] (device), optionally deriving the imaginary-time scale:
// if scale_out != null: scale_out[0] = c = sqrt(norm_target / (dV * sum slot 0)),
// and if shift_dt != 0 also scale_out[1] += log(c) / shift_dt (the running
// chemical-potential shift of the exact imaginary-time substep).
// With scratch (>= kFinBlocks * kRedSlots doubles, device) and many blocks,
// the sum runs in two fixed-order stages (kFinBlocks workgroups over fixed
// row ranges, then one over their results): same determinism, less latency.
constexpr int kFinBlocks = 64;
hipError_t launch_finalize(const double *partial, long long count, double *out,
                           double *scale_out, double norm_target, double dV,
                           hipStream_t s, double *scratch = nullptr, double shift_dt = 0.0);

// psi <- c psi (c read from device), precision 0/1; sets *c = 1 afterwards.
hipError_t launch_scale(int precision, void *psi, long long sites, double *c,
                        hipStream_t s);

// |k|-shell sums.  kind 0: n_k from the spectrum f[0]; kind 1: compressible,
// incompressible and quantum-pressure energies from the spectra f[j] of
// Z_j = u_j + i w_j.  Partial histograms of 4 x nbins doubles per workgroup.
struct ShellArgs {
  int kind;
  const void *f[3];  // complex T fields on the 3D view grid
  int n[3];          // 3D view (2D: n[0] = 1)
  double kscale[3];  // 2 pi / L_j per view axis (0 for a missing axis)
  double dk;         // shell width
  int integer_shells;  // equal box lengths: shells from the integer sum of m_j^2
  int nbins;
  double w;          // dV / N_tot
  double wk;         // 1 / N_tot (kind 0: the |k|^2 |psi_hat|^2 sums)
  double *partial;   // [gridDim][4][nbins]
};
// Workgroups of a shell launch of this kind on the current device (at most
// kShellMaxBlocks; the partial histograms need that many rows at most).
constexpr int kShellMaxBlocks = 1024;
int shell_blocks(int precision, int kind, long long sites, int nbins);
hipError_t launch_shells(int precision, const ShellArgs &a, int blocks, hipStream_t s);
// out[i] = sum_b partial[b * len + i] for i < len, b < count, fixed order.
hipError_t launch_sum_columns(const double *partial, long long count, int len, double *out,
                              hipStream_t s);

// After the last pass of step `step` of a chunk (imaginary-time classes): per
// slot that ran it, form the renormalisation factor from the slot's norm
// partials in fixed order.
hipError_t launch_slot_update(Slot *slots, int nslots, const double *partial,
                              long long blocks_per_grid, double dV, int step, hipStream_t s);
// After a chunk of `steps` steps: steps_done of every slot advances by
// `steps`, clamped to steps_total (slot step counts change once per chunk;
// within a chunk a launch names its step).
hipError_t launch_slot_advance(Slot *slots, int nslots, int steps, hipStream_t s);

// On-chip batched class: one workgroup holds a whole square 2D grid in LDS
// and runs several steps of its slot without touching HBM in between.
struct OnchipArgs {
  Slot *slots;
  const int *slot_map;  // grid row -> slot index
  int steps;            // steps per launch (each slot runs min(steps, remaining))
  int rows_first;       // 1: a step starts with the lines along the last axis
  int n;                // grid is n x n
  double dt, dV;
  double lo[3], h[3];   // 3D view coordinates (view axis 0 unused)
  const void *tw_row, *tw_col;  // twiddles along the last / first axis
  const void *kr_row, *kr_col;  // real-time kinetic factors per axis
  const void *ki_row, *ki_col;  // imaginary-time kinetic factors per axis
};
// Square 2D grids whose state fits one workgroup's LDS: n <= 64 in FP64,
// n <= 128 in FP32.
bool onchip_supported(int precision, int n);
hipError_t launch_onchip(int precision, const OnchipArgs &a, int rows, hipStream_t s);

// Precision codes of a context: 0 FP64; 1 FP32 state and arithmetic; 2 FP32
// state with FP64 arithmetic.
inline bool state_f32(int precision) { return precision != 0; }
inline bool math_f32(int precision) { return precision == 1; }

// Most slots a shape class holds (the active-slot map travels as a kernel
// argument).
constexpr int kMaxSlots = 256;
struct SlotMap {
  int n;
  int idx[kMaxSlots];
};
// Stream-ordered writes of one slot-table entry and of the active-slot map.
// The values travel as kernel arguments, so no host buffer has to outlive the
// call.
hipError_t launch_slot_write(Slot *dst, const Slot &value, hipStream_t s);
hipError_t launch_map_write(int *dst, const SlotMap &m, hipStream_t s);

// Fill a state with index-hashed values in [-1, 1) (for timing runs).
hipError_t launch_fill_noise(int precision, void *psi, long long sites, hipStream_t s);

// Parameters of a separable analytic potential on the 3D view axes:
// v_j(x) = hw[j] (x - c[j])^2 + a[j] (x - c[j])^4 + s[j] sin^2(q[j] x + ph[j]).
struct SepParams {
  double hw[3], c[3], a[3], s[3], q[3], ph[3];
};
// out[off_j + i] = wA v_j(x_{j,i}; A) + wB v_j(x_{j,i}; B) for every view axis j
// and i < n[j] (off_0 = 0, off_1 = n[0], off_2 = n[0] + n[1]),
// x_{j,i} = lo[j] + i h[j].
hipError_t launch_vtables(const SepParams &A, double wA, const SepParams &B, double wB,
                          const int n[3], const double lo[3], const double h[3], double *out,
                          hipStream_t s);

// Precision conversion copies (device to device).
hipError_t launch_convert(int src_prec, const void *src, int dst_prec, void *dst,
                          long long sites, hipStream_t s);

}  // namespace gpe
