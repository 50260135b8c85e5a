// Internal: the context behind the opaque gpe_ctx handle and the host helpers
// shared by the C ABI (gpe.cpp) and the serving scheduler (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "gpe.h"
#include "gpe_kernels.h"

namespace gpe_host {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Kinds of per-frequency tables along one axis.
enum TableKind { TB_KREAL = 0, TB_KIMAG = 1, TB_DERIV = 2, TB_INVN = 3 };

// Launch shapes of the rotating step passes (3D; see gpe_tuning.transpose):
// on = 1 runs the step passes in their rotating form, with these widths, tile
// orders and streaming flags per view axis; the context's in-place shapes then
// serve the read-only passes (observables, transforms, spectra).
struct RotShape {
  int on = 0;
  int wreq[3] = {8, 8, 8};
  int xcd[3] = {1, 1, 1};
  int stream[3] = {0, 0, 0};
};

struct TimedKind {
  std::string name;
  double total_ms = 0;
  long long launches = 0;
  double bytes = 0;
};

}  // namespace gpe_host

struct gpe_ctx {
  gpe_desc desc{};
  int dim = 0;
  int n3[3] = {1, 1, 1};     // 3D view (2D problems: n3[0] = 1)
  double lo3[3] = {0, 0, 0}, h3[3] = {0, 0, 0}, L3[3] = {1, 1, 1};
  long long sites = 0;
  int prec = 0;
  size_t esize = 16;  // bytes per complex site
  double dV = 1;

  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  void *psi = nullptr;
  // Second state array of the rotating passes (allocated on first use); the
  // two swap roles after every pass, and psi always names the current state.
  void *psi_alt = nullptr;
  void *work[3] = {nullptr, nullptr, nullptr};  // spectra work fields (allocated on demand)
  double *hist_partial = nullptr;  // shell histograms per workgroup
  double *hist = nullptr;          // 8 x nbins finalized shell sums
  double *V = nullptr;         // FP64 potential array (device) or null
  double hv[3] = {0, 0, 0};    // analytic V coefficients (3D view)
  // Separable potential: per-view-axis tables (n3[0] + n3[1] + n3[2] doubles)
  // of v_j, or, for a time-dependent potential, of its mean over the
  // midpoints of the N substep about to run (rewritten before each use).
  double *vtab = nullptr;
  bool vtab_on = false;
  gpe_potential_fn vfn = nullptr;
  void *vfn_user = nullptr;
  double time = 0.0;           // context clock (real time)
  int imag_method = GPE_IMAG_FROZEN;  // imaginary-time N substep
  double *partial = nullptr;   // per-workgroup partials, 3 regions
  long long partial_region = 0;  // doubles per region
  double *sums = nullptr;      // finalized sums, 4 x kRedSlots
  double *scale = nullptr;     // imaginary-time c
  double *fin = nullptr;       // two-stage finalize scratch, kFinBlocks x kRedSlots
  void *tw[3] = {nullptr, nullptr, nullptr};  // per axis (3D view) twiddles
  double *kw[3] = {nullptr, nullptr, nullptr};  // k^2/N weights per axis
  std::map<std::pair<int, std::pair<int, double>>, void *> tables;  // (axis,(kind,dt))
  // Small grids: steady-state steps replayed from HIP graphs, per
  // (mode 0 real / 1 imaginary, dt, steps per graph); rebuilt when the
  // potential changes.
  std::map<std::tuple<int, double, int>, hipGraphExec_t> step_graphs;
  size_t dev_bytes = 0;

  bool timing = false;
  std::vector<gpe_host::TimedKind> kinds;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;

  std::string err;
  int pass_order[3] = {2, 1, 0};
  // Strided columns per workgroup, per view axis (axis 2 is contiguous).  The
  // slowest axis prefers 256-byte rows in both precisions; the middle axis is
  // fastest with 128-byte rows in FP64 and 64-byte rows of 16 columns in FP32
  // (measured at 512^3 on MI355X).
  int wreq[3] = {16, 8, 8};
  // Strided passes hand each XCD a contiguous run of tiles (measured: a few
  // percent faster at 512^3 than the default round-robin order).
  int xcd_remap[3] = {1, 1, 0};
  // Radix plan per view axis (0 default, 1 the alternative plan where one
  // exists).
  int plan[3] = {0, 0, 0};
  // Streaming (non-temporal) loads (bit 0) and stores (bit 1) in the step
  // passes, per view axis.
  int streaming[3] = {0, 0, 0};
  // 3D: the step passes in their rotating form (axes in the order 2, 0, 1;
  // pass_order then applies to the read-only passes only).
  gpe_host::RotShape rot;
};


namespace gpe_host {

gpe_status fail(gpe_ctx *c, gpe_status st, const std::string &msg);
gpe_status hipfail(gpe_ctx *c, hipError_t e, const char *what);
gpe_status get_table(gpe_ctx *c, int vaxis, int kind, double dt, void **out);
gpe::PassArgs base_args(gpe_ctx *c, int vaxis);
gpe_status launch_pass(gpe_ctx *c, const gpe::PassArgs &a);
gpe_status set_potential(gpe_ctx *c, const double *V_host, const gpe_harmonic *V_an);
// Times and weights of a time-dependent potential's table: wa V(ta) + wb V(tb).
struct VAt {
  double ta, wa, tb, wb;
};
// Writes table region `region` (0 or 1, each n3[0] + n3[1] + n3[2] doubles).
gpe_status vtables_at(gpe_ctx *c, const VAt &at, int region = 0);
inline long long vtab_len(const gpe_ctx *c) { return c->n3[0] + c->n3[1] + c->n3[2]; }
void drop_step_graphs(gpe_ctx *c);
// Steps per step graph unless convergence checks set the length.
constexpr int kGraphSteps = 32;
// n identical steady-state steps (mode 0: real time with N(dt) first and no
// closing phase; 1: imaginary time), from graphs of len steps where allowed.
gpe_status steady_steps(gpe_ctx *c, int mode, double dt, int64_t n, int len, void *const K[3]);
gpe_status compute_obs(gpe_ctx *c, const double *scale, gpe_obs *o);
// One real-time step (opening phase N(tau_pre), the kinetic factor K on every
// axis, closing phase N(tau_post) if nonzero; pre/post: time-dependent
// potential times, or null) and one imaginary-time step; direct launches.
gpe_status real_step(gpe_ctx *c, void *const K[3], double tau_pre, double tau_post,
                     const VAt *pre, const VAt *post);
gpe_status imag_step(gpe_ctx *c, void *const K[3], double dt);
int n_axes(const gpe_ctx *c);
int order_axis(const gpe_ctx *c, int i);
int view_axis(const gpe_ctx *c, int user_axis);
gpe_status validate_desc(const gpe_desc *d, std::string &msg);
// Launch shapes a new context of this class uses (view axes): the tuning
// table's entry, else the defaults.
void effective_tuning(const gpe_desc &d, int wreq[3], int xcd[3], int order[3], int plan[3],
                      int stream[3], RotShape *rot = nullptr);
// The step passes of this context rotate the grid (3D, tuned so, and not
// replayed from graphs).
bool use_trans(const gpe_ctx *c);
// Device bytes of a context (with_state: including the state array).
uint64_t context_bytes(const gpe_desc &d, bool with_state = true);
// gpe_create, optionally without the state array (a holder of the tables of
// a shape class, used only for its geometry, twiddles and weights).
gpe_status create_context(const gpe_desc *desc, const double *V_host, const gpe_harmonic *V_an,
                          void *hip_stream, bool with_state, gpe_ctx **out);

}  // namespace gpe_host
