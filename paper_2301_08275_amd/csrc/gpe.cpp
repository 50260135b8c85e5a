// Host runtime behind the C ABI of include/gpe.h: context and buffers, the
// FP64 host tables (twiddles, kinetic factors), the real- and imaginary-time
// step schedules built from fused axis passes, observables and timing.
#include "gpe.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "gpe_ctx.h"
#include "gpe_kernels.h"

namespace {
thread_local std::string g_create_error;
}  // namespace

namespace gpe_host {

gpe_status fail(gpe_ctx *c, gpe_status st, const std::string &msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return st;
}

gpe_status hipfail(gpe_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? GPE_ENOMEM : GPE_EDEVICE, m);
}

#define HIPCHK(ctx, call, what)                  \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hipfail(ctx, e_, what); \
  } while (0)

bool pow2_in_range(int v) { return v >= 8 && v <= 1024 && (v & (v - 1)) == 0; }

gpe_status dalloc(gpe_ctx *c, void **p, size_t bytes, const char *what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hipfail(c, e, what);
  }
  c->dev_bytes += bytes;
  return GPE_OK;
}

int view_axis(const gpe_ctx *c, int user_axis) { return user_axis + (3 - c->dim); }

// Signed integer mode of index i on an axis of n points.
long signed_mode(long i, long n) { return i < n / 2 ? i : i - n; }

double wavenumber(const gpe_ctx *c, int vaxis, long i) {
  return 2 * kPi * (double)signed_mode(i, c->n3[vaxis]) / c->L3[vaxis];
}

// Host FP64 tables uploaded in the state precision, 16 bytes per entry either
// way: FP64 (re, im), or FP32 (re_hi, im_hi, re_lo, im_lo) with hi the FP32
// rounding of the FP64 value and lo the FP32 rounding of the remainder.
gpe_status upload_complex(gpe_ctx *c, void **dst, const std::vector<double> &re,
                          const std::vector<double> &im) {
  const size_t n = re.size();
  std::vector<double> d(2 * n);
  std::vector<float> f(4 * n);
  for (size_t i = 0; i < n; ++i) {
    d[2 * i] = re[i];
    d[2 * i + 1] = im[i];
    const float rh = (float)re[i], ih = (float)im[i];
    f[4 * i] = rh;
    f[4 * i + 1] = ih;
    f[4 * i + 2] = (float)(re[i] - (double)rh);
    f[4 * i + 3] = (float)(im[i] - (double)ih);
  }
  gpe_status st = dalloc(c, dst, n * 16, "table allocation");
  if (st != GPE_OK) return st;
  HIPCHK(c, hipMemcpy(*dst, c->prec == 1 ? (void *)f.data() : (void *)d.data(), n * 16,
                      hipMemcpyHostToDevice), "table upload");
  return GPE_OK;
}

// exp(-2 pi i j / N), j < N, each entry computed directly from its index.
gpe_status make_twiddles(gpe_ctx *c, int vaxis) {
  const int N = c->n3[vaxis];
  std::vector<double> re(N), im(N);
  for (int j = 0; j < N; ++j) {
    const double a = 2 * kPi * (double)j / (double)N;
    re[j] = std::cos(a);
    im[j] = -std::sin(a);
  }
  return upload_complex(c, &c->tw[vaxis], re, im);
}

gpe_status make_kin_weights(gpe_ctx *c, int vaxis) {
  const int N = c->n3[vaxis];
  std::vector<double> w(N);
  for (int j = 0; j < N; ++j) {
    const double k = wavenumber(c, vaxis, j);
    w[j] = k * k / (double)N;
  }
  gpe_status st = dalloc(c, (void **)&c->kw[vaxis], N * sizeof(double), "table allocation");
  if (st != GPE_OK) return st;
  HIPCHK(c, hipMemcpy(c->kw[vaxis], w.data(), N * sizeof(double), hipMemcpyHostToDevice),
         "table upload");
  return GPE_OK;
}

// Per-frequency factor along one axis, 1/N folded in:
//   TB_KREAL exp(-i k^2 dt/2)/N, TB_KIMAG exp(-k^2 dt/2)/N, TB_DERIV i k/N,
//   TB_INVN 1/N.  Arguments in FP64.
gpe_status get_table(gpe_ctx *c, int vaxis, int kind, double dt, void **out) {
  auto key = std::make_pair(vaxis, std::make_pair(kind, dt));
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    *out = it->second;
    return GPE_OK;
  }
  if (c->tables.size() > 64) {
    // Bounded cache.  One operation fetches tables of a single (kind, dt) for
    // its axes, so those are kept: the caller may hold pointers to them.
    // Graphs of cached steps refer to tables and go too.
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
    drop_step_graphs(c);
    for (auto t = c->tables.begin(); t != c->tables.end();) {
      if (t->first.second == key.second) {
        ++t;
        continue;
      }
      (void)hipFree(t->second);
      t = c->tables.erase(t);
    }
  }
  const int N = c->n3[vaxis];
  std::vector<double> re(N), im(N);
  for (int j = 0; j < N; ++j) {
    const double k = wavenumber(c, vaxis, j);
    const double inv = 1.0 / (double)N;
    if (kind == TB_KREAL) {
      const double ph = k * k * dt / 2;
      re[j] = std::cos(ph) * inv;
      im[j] = -std::sin(ph) * inv;
    } else if (kind == TB_KIMAG) {
      re[j] = std::exp(-k * k * dt / 2) * inv;
      im[j] = 0;
    } else if (kind == TB_DERIV) {
      re[j] = 0;
      im[j] = k * inv;
    } else {
      re[j] = inv;
      im[j] = 0;
    }
  }
  void *p = nullptr;
  gpe_status st = upload_complex(c, &p, re, im);
  if (st != GPE_OK) return st;
  c->tables[key] = p;
  *out = p;
  return GPE_OK;
}

gpe::PassArgs base_args(gpe_ctx *c, int vaxis) {
  gpe::PassArgs a{};
  a.src = c->psi;
  a.dst = c->psi;
  for (int j = 0; j < 3; ++j) {
    a.n[j] = c->n3[j];
    a.hv[j] = c->hv[j];
    a.lo[j] = c->lo3[j];
    a.h[j] = c->h3[j];
  }
  a.axis = vaxis;
  a.wreq = c->wreq[vaxis];
  a.plan = c->plan[vaxis];
  a.stream = c->streaming[vaxis];
  a.xcd_remap = (vaxis != 2 && c->xcd_remap[vaxis]) ? 1 : 0;
  a.vkind = c->V ? gpe::V_ARRAY
                 : c->vtab_on ? gpe::V_TABLES
                 : ((c->hv[0] != 0 || c->hv[1] != 0 || c->hv[2] != 0) ? gpe::V_HARMONIC
                                                                      : gpe::V_NONE);
  a.vtab = c->vtab;
  a.forward = 1;
  a.inverse = 1;
  a.store = 1;
  a.g = c->desc.g;
  a.V = c->V;
  a.tw = c->tw[vaxis];
  return a;
}

// Timing kind: operation, axis of the 3D view, precision.
std::string kind_name(int prec, const gpe::PassArgs &a) {
  const char *op = "step";
  if (!a.forward) op = "ifft";
  else if (!a.store) op = "obs";
  else if (!a.inverse) op = "fft";
  else if (a.post == gpe::PH_DERIV) op = "deriv";
  static const char ax[3] = {'x', 'y', 'z'};
  return std::string(op) + "_" + ax[a.axis] + (prec == 1 ? "_fp32" : prec == 2 ? "_fp32s" : "_fp64");
}

gpe_status launch_pass(gpe_ctx *c, const gpe::PassArgs &a) {
  int kind = -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    // kinds: one per axis of the 3D view; bytes = algorithmic HBM traffic
    const std::string nm = kind_name(c->prec, a);
    for (size_t i = 0; i < c->kinds.size(); ++i)
      if (c->kinds[i].name == nm) kind = (int)i;
    if (kind < 0) {
      TimedKind k;
      k.name = nm;
      c->kinds.push_back(k);
      kind = (int)c->kinds.size() - 1;
    }
    double bytes = (double)c->sites * c->esize;  // every pass reads the state once
    bytes += a.store ? (double)c->sites * c->esize : 0;
    // (the derivative pass combines with the state it loaded: no second read)
    if (c->V && (a.pre != gpe::PH_NONE || a.post != gpe::PH_NONE)) bytes += 8.0 * c->sites;
    c->kinds[kind].bytes = bytes;
    if (!c->event_pool.empty()) {
      e0 = c->event_pool.back().first;
      e1 = c->event_pool.back().second;
      c->event_pool.pop_back();
    } else {
      HIPCHK(c, hipEventCreate(&e0), "event create");
      HIPCHK(c, hipEventCreate(&e1), "event create");
    }
    HIPCHK(c, hipEventRecord(e0, c->stream), "event record");
  }
  hipError_t e = gpe::launch_axis_pass(c->prec, a, c->stream);
  if (e != hipSuccess) return hipfail(c, e, "axis pass launch");
  if (c->timing) {
    HIPCHK(c, hipEventRecord(e1, c->stream), "event record");
    c->pending.push_back({kind, {e0, e1}});
    if (c->pending.size() >= 256) {
      // drain: events complete in order on the stream
      HIPCHK(c, hipEventSynchronize(c->pending.back().second.second), "event sync");
      for (auto &pe : c->pending) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, pe.second.first, pe.second.second);
        c->kinds[pe.first].total_ms += ms;
        c->kinds[pe.first].launches += 1;
        c->event_pool.push_back(pe.second);
      }
      c->pending.clear();
    }
  }
  return GPE_OK;
}

gpe_status drain_timing(gpe_ctx *c) {
  if (c->pending.empty()) return GPE_OK;
  HIPCHK(c, hipEventSynchronize(c->pending.back().second.second), "event sync");
  for (auto &pe : c->pending) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, pe.second.first, pe.second.second);
    c->kinds[pe.first].total_ms += ms;
    c->kinds[pe.first].launches += 1;
    c->event_pool.push_back(pe.second);
  }
  c->pending.clear();
  return GPE_OK;
}

int n_axes(const gpe_ctx *c) { return c->dim; }
int order_axis(const gpe_ctx *c, int i) {
  // pass order over the view axes that exist (skip axis 0 in 2D)
  int k = 0;
  for (int j = 0; j < 3; ++j) {
    int ax = c->pass_order[j];
    if (ax < 3 - c->dim) continue;
    if (k == i) return ax;
    ++k;
  }
  return -1;
}

gpe_status validate_desc(const gpe_desc *d, std::string &msg) {
  if (!d) { msg = "desc is NULL"; return GPE_EINVAL; }
  if (d->dim < 1 || d->dim > 3) {
    msg = "dim must be 1, 2 or 3";
    return GPE_EINVAL;
  }
  for (int j = 0; j < d->dim; ++j) {
    if (d->n[j] < 1 || (d->n[j] & (d->n[j] - 1)) != 0) {
      msg = "n[j] must be a power of two";
      return GPE_EINVAL;
    }
    if (!pow2_in_range(d->n[j])) {
      msg = "n[j] must be in [8, 1024]";
      return GPE_EUNSUPPORTED;
    }
    if (!(std::isfinite(d->lo[j]) && std::isfinite(d->hi[j]) && d->hi[j] > d->lo[j])) {
      msg = "need finite lo[j] < hi[j]";
      return GPE_EINVAL;
    }
  }
  if (!std::isfinite(d->g)) { msg = "g must be finite"; return GPE_EINVAL; }
  if (d->precision != GPE_FP64 && d->precision != GPE_FP32 && d->precision != GPE_FP32_STATE) {
    msg = "precision must be GPE_FP64, GPE_FP32 or GPE_FP32_STATE";
    return GPE_EINVAL;
  }
  if (!(d->norm_target > 0) || !std::isfinite(d->norm_target)) {
    msg = "norm_target must be positive";
    return GPE_EINVAL;
  }
  return GPE_OK;
}

gpe_status set_potential(gpe_ctx *c, const double *V_host, const gpe_harmonic *V_an) {
  if (V_host && V_an) return fail(c, GPE_EINVAL, "give V_host or V_an, not both");
  drop_step_graphs(c);  // their launches carry the old potential
  for (int j = 0; j < 3; ++j) c->hv[j] = 0;
  c->vtab_on = false;
  c->vfn = nullptr;
  c->vfn_user = nullptr;
  if (V_an) {
    for (int j = 0; j < c->dim; ++j) {
      if (!std::isfinite(V_an->w[j])) return fail(c, GPE_EINVAL, "trap frequency not finite");
      c->hv[view_axis(c, j)] = 0.5 * V_an->w[j] * V_an->w[j];
    }
  }
  if (V_host) {
    if (!c->V) {
      gpe_status st = dalloc(c, (void **)&c->V, c->sites * sizeof(double), "V allocation");
      if (st != GPE_OK) return st;
    }
    HIPCHK(c, hipMemcpy(c->V, V_host, c->sites * sizeof(double), hipMemcpyHostToDevice),
           "V upload");
  } else if (c->V) {
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
    (void)hipFree(c->V);
    c->dev_bytes -= c->sites * sizeof(double);
    c->V = nullptr;
  }
  return GPE_OK;
}

// Separable potential parameters on the view axes (hw = w^2 / 2); false if
// any used entry is not finite.
bool sep_params(const gpe_ctx *c, const gpe_separable &u, gpe::SepParams *P) {
  *P = gpe::SepParams{};
  for (int j = 0; j < c->dim; ++j) {
    const int v = view_axis(c, j);
    const double vals[6] = {u.w[j], u.center[j], u.quartic[j], u.lattice[j], u.q[j], u.phase[j]};
    for (double x : vals)
      if (!std::isfinite(x)) return false;
    P->hw[v] = 0.5 * u.w[j] * u.w[j];
    P->c[v] = u.center[j];
    P->a[v] = u.quartic[j];
    P->s[v] = u.lattice[j];
    P->q[v] = u.q[j];
    P->ph[v] = u.phase[j];
  }
  return true;
}

// Two regions of per-axis tables: the second holds the closing phase's
// potential when one pass carries both phases (a 1D grid).
gpe_status alloc_vtab(gpe_ctx *c) {
  if (c->vtab) return GPE_OK;
  return dalloc(c, (void **)&c->vtab, 2 * vtab_len(c) * sizeof(double),
                "potential table allocation");
}

// Rewrite the tables of a time-dependent potential with the weighted sum of
// V(ta) (weight wa) and V(tb) (weight wb; skipped when 0); a static
// potential needs nothing.  Enqueued on the context stream, so passes
// already enqueued read the previous tables.
gpe_status vtables_at(gpe_ctx *c, const VAt &at, int region) {
  if (!c->vfn) return GPE_OK;
  gpe_separable u[2] = {};
  gpe::SepParams P[2];
  c->vfn(at.ta, &u[0], c->vfn_user);
  if (at.wb != 0) c->vfn(at.tb, &u[1], c->vfn_user);
  if (!sep_params(c, u[0], &P[0]) || (at.wb != 0 && !sep_params(c, u[1], &P[1])))
    return fail(c, GPE_EINVAL, "the potential callback returned a non-finite parameter");
  if (at.wb == 0) P[1] = P[0];
  HIPCHK(c, gpe::launch_vtables(P[0], at.wa, P[1], at.wb, c->n3, c->lo3, c->h3,
                                c->vtab + region * vtab_len(c), c->stream),
         "potential table launch");
  return GPE_OK;
}

// Read-only observation passes: per axis a forward transform with the
// kinetic-weight sum; the first also takes the real-space sums.  scale (device,
// nullable) multiplies the state on the fly.  Enqueues the finalized sums,
// 3 x kRedSlots doubles, at sums_dev (device); no host wait.
gpe_status enqueue_observe(gpe_ctx *c, const double *scale, double *sums_dev) {
  gpe_status vst = vtables_at(c, VAt{c->time, 1.0, 0.0, 0.0});  // E_pot at the clock
  if (vst != GPE_OK) return vst;
  for (int i = 0; i < n_axes(c); ++i) {
    const int ax = order_axis(c, i);
    gpe::PassArgs a = base_args(c, ax);
    a.inverse = 0;
    a.store = 0;
    a.red = gpe::RED_KIN | (i == 0 ? gpe::RED_REAL : 0);
    a.kw = c->kw[ax];
    a.scale = scale;
    a.partial = c->partial + i * c->partial_region;
    gpe_status st = launch_pass(c, a);
    if (st != GPE_OK) return st;
    const gpe::PassShape sh = gpe::launch_shape(c->prec, a);
    HIPCHK(c, gpe::launch_finalize(a.partial, sh.blocks, sums_dev + i * gpe::kRedSlots,
                                   nullptr, 0, 1, c->stream, c->fin), "finalize launch");
  }
  return GPE_OK;
}

// The observables of one record of finalized sums (3 x kRedSlots, pass order).
gpe_status obs_from_sums(gpe_ctx *c, const double *sums, gpe_obs *o) {
  double s[3][gpe::kRedSlots];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < gpe::kRedSlots; ++k)
      s[i][k] = i < n_axes(c) ? sums[i * gpe::kRedSlots + k] : 0;
  const double *r = &s[0][gpe::kSlotReal];
  double kin = 0;
  for (int i = 0; i < n_axes(c); ++i) kin += s[i][gpe::kSlotKin];
  gpe_obs out{};
  out.norm = c->dV * r[0];
  out.e_pot = c->dV * r[1];
  out.e_int = 0.5 * c->desc.g * c->dV * r[2];
  out.e_kin = 0.5 * c->dV * kin;
  out.energy = out.e_kin + out.e_pot + out.e_int;
  out.mu = (out.e_kin + out.e_pot + 2 * out.e_int) / out.norm;
  double r2 = 0;
  for (int j = 0; j < 3; ++j) {
    if (j < c->dim) {
      const double m2 = r[3 + view_axis(c, j)] / r[0];
      out.sigma[j] = std::sqrt(m2);
      r2 += m2;
    } else {
      out.sigma[j] = 0;
    }
  }
  out.r_rms = std::sqrt(r2);
  *o = out;
  bool finite = std::isfinite(out.norm) && std::isfinite(out.energy) && std::isfinite(r2);
  if (!finite) return fail(c, GPE_ENONFINITE, "observables are not finite");
  return GPE_OK;
}

gpe_status compute_obs(gpe_ctx *c, const double *scale, gpe_obs *o) {
  gpe_status st = enqueue_observe(c, scale, c->sums);
  if (st != GPE_OK) return st;
  std::vector<double> h(3 * gpe::kRedSlots, 0.0);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->sums, 3 * gpe::kRedSlots * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream), "sums download");
  HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  return obs_from_sums(c, h.data(), o);
}

bool equal_lengths(const gpe_ctx *c) {
  const int off = 3 - c->dim;
  for (int j = off + 1; j < 3; ++j)
    if (std::fabs(c->L3[j] - c->L3[off]) > 1e-12 * c->L3[off]) return false;
  return true;
}

double shell_width(const gpe_ctx *c) {
  double dk = 2 * kPi / c->L3[3 - c->dim];
  for (int j = 3 - c->dim; j < 3; ++j) dk = std::fmin(dk, 2 * kPi / c->L3[j]);
  return dk;
}

int shell_count(const gpe_ctx *c) {
  const double dk = shell_width(c);
  double q = 0;
  for (int j = 3 - c->dim; j < 3; ++j) {
    const double kn = (double)(c->n3[j] / 2) * (2 * kPi / c->L3[j]) / dk;
    q += kn * kn;
  }
  return (int)std::floor(std::sqrt(q) + 0.5) + 1;
}

// Forward transform of src into dst (then in place on dst) along every axis
// but view axis `skip` (-1: none); with real_sums, the first pass also takes
// the real-space sums of src (finalized into real_sums, kRedSlots doubles).
gpe_status forward_all(gpe_ctx *c, const void *src, void *dst, int skip = -1,
                       double *real_sums = nullptr) {
  bool first = true;
  for (int i = 0; i < n_axes(c); ++i) {
    const int ax = order_axis(c, i);
    if (ax == skip) continue;
    gpe::PassArgs a = base_args(c, ax);
    a.src = first ? src : dst;
    a.dst = dst;
    a.inverse = 0;
    if (first && real_sums) {
      a.red = gpe::RED_REAL;
      a.partial = c->partial;
    }
    gpe_status st = launch_pass(c, a);
    if (st != GPE_OK) return st;
    if (first && real_sums) {
      const gpe::PassShape sh = gpe::launch_shape(c->prec, a);
      HIPCHK(c, gpe::launch_finalize(a.partial, sh.blocks, real_sums, nullptr, 0, 1, c->stream,
                                     c->fin), "finalize launch");
    }
    first = false;
  }
  return GPE_OK;
}

// Shell spectra of the current state (see gpe_spectra); with obs, also the
// observables: the first pass of the transform behind N(n) takes the
// real-space sums and the particle-number shell kernel sums
// |k|^2 |psi_hat|^2 / N_tot over the grid, the kinetic sum by Parseval's
// identity on the whole grid, so the read-only observable passes do not run.
gpe_status compute_spectra(gpe_ctx *c, gpe_spectra *spec, gpe_obs *obs = nullptr) {
  const int nb = shell_count(c);
  if (spec->nbins != nb) return fail(c, GPE_EINVAL, "spec->nbins must equal gpe_spectra_bins()");
  for (int j = 0; j < c->dim; ++j) {
    if (!c->work[j]) {
      gpe_status st = dalloc(c, &c->work[j], c->sites * c->esize, "spectra work allocation");
      if (st != GPE_OK) return st;
    }
  }
  const int blocks0 = gpe::shell_blocks(c->prec, 0, c->sites, nb);
  const int blocks1 = gpe::shell_blocks(c->prec, 1, c->sites, nb);
  if (!c->hist_partial) {
    gpe_status st = dalloc(c, (void **)&c->hist_partial,
                           (size_t)gpe::kShellMaxBlocks * 4 * nb * sizeof(double),
                           "histogram allocation");
    if (st != GPE_OK) return st;
    st = dalloc(c, (void **)&c->hist, 8 * (size_t)nb * sizeof(double), "histogram allocation");
    if (st != GPE_OK) return st;
  }
  gpe::ShellArgs sa{};
  for (int j = 0; j < 3; ++j) {
    sa.n[j] = c->n3[j];
    sa.kscale[j] = j >= 3 - c->dim ? 2 * kPi / c->L3[j] : 0.0;
  }
  sa.dk = shell_width(c);
  sa.integer_shells = equal_lengths(c) ? 1 : 0;
  sa.nbins = nb;
  sa.w = c->dV / (double)c->sites;
  sa.wk = 1.0 / (double)c->sites;
  sa.partial = c->hist_partial;
  if (obs) {
    gpe_status vst = vtables_at(c, VAt{c->time, 1.0, 0.0, 0.0});  // E_pot at the clock
    if (vst != GPE_OK) return vst;
  }
  // particle-number spectrum from the transform of psi
  gpe_status st = forward_all(c, c->psi, c->work[0], -1, obs ? c->sums : nullptr);
  if (st != GPE_OK) return st;
  sa.kind = 0;
  sa.f[0] = c->work[0];
  HIPCHK(c, gpe::launch_shells(c->prec, sa, blocks0, c->stream), "shell launch");
  HIPCHK(c, gpe::launch_sum_columns(c->hist_partial, blocks0, 4 * nb, c->hist, c->stream),
         "histogram sum");
  // Z_j = u_j + i w_j from the spectral derivative along each axis, transformed
  void *deriv_tab[3] = {nullptr, nullptr, nullptr};
  for (int j = 0; j < c->dim; ++j) {
    const int ax = view_axis(c, j);
    st = get_table(c, ax, TB_DERIV, 0.0, &deriv_tab[ax]);
    if (st != GPE_OK) return st;
    gpe::PassArgs a = base_args(c, ax);
    a.src = c->psi;
    a.dst = c->work[j];
    a.mid = gpe::MID_TABLE;
    a.mtab = deriv_tab[ax];
    a.post = gpe::PH_DERIV;
    a.refwd = 1;  // Z_j leaves this pass already transformed along axis j
    st = launch_pass(c, a);
    if (st != GPE_OK) return st;
    st = forward_all(c, c->work[j], c->work[j], ax);
    if (st != GPE_OK) return st;
  }
  sa.kind = 1;
  for (int j = 0; j < 3; ++j) sa.f[j] = nullptr;
  for (int j = 0; j < c->dim; ++j) sa.f[view_axis(c, j)] = c->work[j];
  HIPCHK(c, gpe::launch_shells(c->prec, sa, blocks1, c->stream), "shell launch");
  HIPCHK(c, gpe::launch_sum_columns(c->hist_partial, blocks1, 4 * nb, c->hist + 4 * nb, c->stream),
         "histogram sum");
  std::vector<double> h(8 * (size_t)nb);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream), "histogram download");
  std::vector<double> sums(3 * gpe::kRedSlots, 0.0);
  if (obs)
    HIPCHK(c, hipMemcpyAsync(sums.data(), c->sums, gpe::kRedSlots * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream), "sums download");
  HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  if (obs) {
    sums[gpe::kSlotKin] = h[nb];  // the shell kernel's |k|^2 sum
    gpe_status ost = obs_from_sums(c, sums.data(), obs);
    if (ost != GPE_OK) return ost;
  }
  for (int b = 0; b < nb; ++b) {
    if (spec->n_k) spec->n_k[b] = h[b];
    if (spec->e_comp) spec->e_comp[b] = h[4 * nb + nb + b];
    if (spec->e_incomp) spec->e_incomp[b] = h[4 * nb + 2 * nb + b];
    if (spec->e_qp) spec->e_qp[b] = h[4 * nb + 3 * nb + b];
  }
  spec->dk = shell_width(c);
  for (double x : h)
    if (!std::isfinite(x)) return fail(c, GPE_ENONFINITE, "spectra are not finite");
  return GPE_OK;
}

// Device bytes gpe_create allocates for desc (state, partials, sums, scale,
// twiddles and E_kin weights per axis); must follow gpe_create.
uint64_t context_bytes(const gpe_desc &d, bool with_state) {
  int n3[3] = {1, 1, 1};
  const int off = 3 - d.dim;
  long long sites = 1;
  for (int j = 0; j < d.dim; ++j) {
    n3[j + off] = d.n[j];
    sites *= d.n[j];
  }
  const uint64_t es = gpe::state_f32(d.precision) ? 8 : 16;
  int wdef[3], xcd[3], order[3], plan[3], stream[3];
  effective_tuning(d, wdef, xcd, order, plan, stream);
  long long maxb = 1;
  uint64_t tables = 0;
  for (int ax = off; ax < 3; ++ax) {
    const gpe::PassShape sh = gpe::pass_shape(d.precision, n3, ax, wdef[ax], plan[ax], true);
    if (sh.blocks > maxb) maxb = sh.blocks;
    if (d.dim == 3) {
      const gpe::PassShape st = gpe::pass_shape(d.precision, n3, ax, 8, plan[ax], true, true);
      if (st.blocks > maxb) maxb = st.blocks;
    }
    tables += (uint64_t)n3[ax] * (16 + sizeof(double));
  }
  return (with_state ? (uint64_t)sites * es : 0) +
         (uint64_t)gpe::kFinBlocks * gpe::kRedSlots * sizeof(double) + 3 * (uint64_t)maxb * gpe::kRedSlots * sizeof(double) +
         4 * gpe::kRedSlots * sizeof(double) + 2 * sizeof(double) + tables;
}

}  // namespace gpe_host

using namespace gpe_host;

extern "C" {

gpe_status gpe_create(const gpe_desc *desc, const double *V_host, const gpe_harmonic *V_an,
                      void *hip_stream, gpe_ctx **out) {
  return create_context(desc, V_host, V_an, hip_stream, true, out);
}

}  // extern "C"

namespace gpe_host {

gpe_status create_context(const gpe_desc *desc, const double *V_host, const gpe_harmonic *V_an,
                          void *hip_stream, bool with_state, gpe_ctx **out) {
  if (!out) return fail(nullptr, GPE_EINVAL, "out is NULL");
  *out = nullptr;
  std::string msg;
  gpe_status st = validate_desc(desc, msg);
  if (st != GPE_OK) return fail(nullptr, st, msg);
  if (V_host && V_an) return fail(nullptr, GPE_EINVAL, "give V_host or V_an, not both");

  gpe_ctx *c = new gpe_ctx();
  c->desc = *desc;
  c->dim = desc->dim;
  c->prec = desc->precision;
  c->esize = gpe::state_f32(c->prec) ? 8 : 16;
  effective_tuning(*desc, c->wreq, c->xcd_remap, c->pass_order, c->plan, c->streaming,
                   &c->rot);
  const int off = 3 - c->dim;
  c->sites = 1;
  c->dV = 1;
  for (int j = 0; j < 3; ++j) {
    c->n3[j] = 1;
    c->lo3[j] = 0;
    c->h3[j] = 0;
    c->L3[j] = 1;
  }
  for (int j = 0; j < c->dim; ++j) {
    c->n3[j + off] = desc->n[j];
    c->lo3[j + off] = desc->lo[j];
    c->L3[j + off] = desc->hi[j] - desc->lo[j];
    c->h3[j + off] = c->L3[j + off] / desc->n[j];
    c->sites *= desc->n[j];
    c->dV *= c->h3[j + off];
  }
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, GPE_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, GPE_EDEVICE, "stream creation failed");
    }
    c->own_stream = true;
  }
  auto bail = [&](gpe_status s) {
    g_create_error = c->err;
    gpe_destroy(c);
    return s;
  };
  if (with_state) {
    if ((st = dalloc(c, &c->psi, c->sites * c->esize, "state allocation")) != GPE_OK)
      return bail(st);
    if (hipMemset(c->psi, 0, c->sites * c->esize) != hipSuccess)
      return bail(fail(c, GPE_EDEVICE, "state clear"));
  }
  // Tuning overrides for experiments: strided workgroup widths per axis.
  if (const char *w = std::getenv("GPE_TUNE_WX")) c->wreq[0] = std::atoi(w);
  if (const char *w = std::getenv("GPE_TUNE_WY")) c->wreq[1] = std::atoi(w);
  if (const char *w = std::getenv("GPE_TUNE_XCD")) c->xcd_remap[0] = c->xcd_remap[1] = std::atoi(w);
  long long maxb = 1;
  for (int ax = 3 - c->dim; ax < 3; ++ax) {
    // (narrow shapes have the most blocks: room for every pass's partials,
    // in either form of the step passes)
    const gpe::PassShape sh = gpe::pass_shape(c->prec, c->n3, ax, c->wreq[ax], c->plan[ax], true);
    if (sh.blocks > maxb) maxb = sh.blocks;
    if (c->dim == 3) {
      const gpe::PassShape st = gpe::pass_shape(c->prec, c->n3, ax, 8, c->plan[ax], true, true);
      if (st.blocks > maxb) maxb = st.blocks;
    }
  }
  c->partial_region = maxb * gpe::kRedSlots;
  if ((st = dalloc(c, (void **)&c->partial, 3 * c->partial_region * sizeof(double),
                   "partials allocation")) != GPE_OK) return bail(st);
  if ((st = dalloc(c, (void **)&c->sums, 4 * gpe::kRedSlots * sizeof(double),
                   "sums allocation")) != GPE_OK) return bail(st);
  if ((st = dalloc(c, (void **)&c->scale, 2 * sizeof(double), "scale allocation")) != GPE_OK)
    return bail(st);
  if ((st = dalloc(c, (void **)&c->fin, gpe::kFinBlocks * gpe::kRedSlots * sizeof(double),
                   "finalize scratch allocation")) != GPE_OK)
    return bail(st);
  const double one = 1.0;
  if (hipMemcpy(c->scale, &one, sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(c, GPE_EDEVICE, "scale init"));
  for (int ax = 3 - c->dim; ax < 3; ++ax) {
    if ((st = make_twiddles(c, ax)) != GPE_OK) return bail(st);
    if ((st = make_kin_weights(c, ax)) != GPE_OK) return bail(st);
  }
  if ((st = set_potential(c, V_host, V_an)) != GPE_OK) return bail(st);
  if (const char *ord = std::getenv("GPE_PASS_ORDER")) {
    if (std::strlen(ord) == 3) {
      for (int j = 0; j < 3; ++j) c->pass_order[j] = ord[j] - '0';
    }
  }
  *out = c;
  return GPE_OK;
}

}  // namespace gpe_host

extern "C" {

gpe_status gpe_set_potential(gpe_ctx *c, const double *V_host, const gpe_harmonic *V_an) {
  if (!c) return GPE_EINVAL;
  return set_potential(c, V_host, V_an);
}

gpe_status gpe_set_separable(gpe_ctx *c, const gpe_separable *V) {
  if (!c) return GPE_EINVAL;
  if (!V) return fail(c, GPE_EINVAL, "V is NULL");
  gpe::SepParams P;
  if (!sep_params(c, *V, &P)) return fail(c, GPE_EINVAL, "potential parameter not finite");
  gpe_status st = set_potential(c, nullptr, nullptr);
  if (st == GPE_OK) st = alloc_vtab(c);
  if (st != GPE_OK) return st;
  HIPCHK(c, gpe::launch_vtables(P, 1.0, P, 0.0, c->n3, c->lo3, c->h3, c->vtab, c->stream),
         "potential table launch");
  c->vtab_on = true;
  return GPE_OK;
}

gpe_status gpe_set_potential_fn(gpe_ctx *c, gpe_potential_fn fn, void *user) {
  if (!c) return GPE_EINVAL;
  gpe_status st = set_potential(c, nullptr, nullptr);
  if (st != GPE_OK || !fn) return st;
  if ((st = alloc_vtab(c)) != GPE_OK) return st;
  c->vfn = fn;
  c->vfn_user = user;
  c->vtab_on = true;
  return GPE_OK;
}

gpe_status gpe_set_imag_method(gpe_ctx *c, int32_t method) {
  if (!c) return GPE_EINVAL;
  if (method != GPE_IMAG_FROZEN && method != GPE_IMAG_EXACT)
    return fail(c, GPE_EINVAL, "method must be GPE_IMAG_FROZEN or GPE_IMAG_EXACT");
  drop_step_graphs(c);  // cached imaginary-time graphs hold the other substep
  c->imag_method = method;
  return GPE_OK;
}

gpe_status gpe_set_time(gpe_ctx *c, double t) {
  if (!c) return GPE_EINVAL;
  if (!std::isfinite(t)) return fail(c, GPE_EINVAL, "t must be finite");
  c->time = t;
  return GPE_OK;
}

gpe_status gpe_get_time(const gpe_ctx *c, double *t) {
  if (!c || !t) return GPE_EINVAL;
  *t = c->time;
  return GPE_OK;
}

gpe_status gpe_set_state(gpe_ctx *c, const double *psi_host) {
  if (!c) return GPE_EINVAL;
  if (!psi_host) return fail(c, GPE_EINVAL, "psi_host is NULL");
  if (c->prec == GPE_FP64) {
    HIPCHK(c, hipMemcpyAsync(c->psi, psi_host, c->sites * 16, hipMemcpyHostToDevice, c->stream),
           "state upload");
  } else {
    std::vector<float> f(2 * c->sites);
    for (long long i = 0; i < 2 * c->sites; ++i) f[i] = (float)psi_host[i];
    HIPCHK(c, hipMemcpyAsync(c->psi, f.data(), c->sites * 8, hipMemcpyHostToDevice, c->stream),
           "state upload");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  return GPE_OK;
}

gpe_status gpe_set_state_device(gpe_ctx *c, const void *dptr, int32_t src) {
  if (!c) return GPE_EINVAL;
  if (!dptr) return fail(c, GPE_EINVAL, "dptr is NULL");
  if (src != GPE_FP64 && src != GPE_FP32) return fail(c, GPE_EINVAL, "bad precision");
  HIPCHK(c, gpe::launch_convert(src, dptr, c->prec, c->psi, c->sites, c->stream),
         "state convert");
  return GPE_OK;
}

gpe_status gpe_get_state(gpe_ctx *c, double *psi_host_out) {
  if (!c) return GPE_EINVAL;
  if (!psi_host_out) return fail(c, GPE_EINVAL, "psi_host_out is NULL");
  if (c->prec == GPE_FP64) {
    HIPCHK(c, hipMemcpyAsync(psi_host_out, c->psi, c->sites * 16, hipMemcpyDeviceToHost,
                             c->stream), "state download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  } else {
    std::vector<float> f(2 * c->sites);
    HIPCHK(c, hipMemcpyAsync(f.data(), c->psi, c->sites * 8, hipMemcpyDeviceToHost, c->stream),
           "state download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
    for (long long i = 0; i < 2 * c->sites; ++i) psi_host_out[i] = f[i];
  }
  return GPE_OK;
}

gpe_status gpe_get_state_device(gpe_ctx *c, void *dptr, int32_t dst) {
  if (!c) return GPE_EINVAL;
  if (!dptr) return fail(c, GPE_EINVAL, "dptr is NULL");
  if (dst != GPE_FP64 && dst != GPE_FP32) return fail(c, GPE_EINVAL, "bad precision");
  HIPCHK(c, gpe::launch_convert(c->prec, c->psi, dst, dptr, c->sites, c->stream),
         "state convert");
  return GPE_OK;
}

}  // extern "C"

namespace gpe_host {

// Small grids are launch-bound: runs of identical steps replay from graphs.
constexpr long long kGraphSites = 1LL << 20;
constexpr size_t kMaxStepGraphs = 8;   // graphs kept per context

// One real-time step: phase N(tau_pre) before the first pass, the kinetic
// factor K in every pass, and a closing phase N(dt/2) after the last pass of
// the last step of a call.
// (never on graph-sized grids: a graph would replay the rotating passes from
// the arrays that were current when it was captured)
bool use_trans(const gpe_ctx *c) {
  return c->rot.on && c->dim == 3 && c->sites > kGraphSites;
}

// The rotating passes visit the axes in this order: the first reads the grid
// as stored ([0][1][2]) and each writes the layout the next one reads, the
// last one the stored layout again.
constexpr int kTransOrder[3] = {2, 0, 1};

gpe_status ensure_alt(gpe_ctx *c) {
  if (c->psi_alt) return GPE_OK;
  return dalloc(c, &c->psi_alt, c->sites * c->esize, "second state allocation");
}

// Point a step pass at the current state; a rotating pass writes the other
// array, which then becomes the current state.
void route(gpe_ctx *c, gpe::PassArgs &a, bool trans) {
  a.src = c->psi;
  a.dst = trans ? c->psi_alt : c->psi;
  a.trans = trans ? 1 : 0;
  if (trans) {
    a.wreq = c->rot.wreq[a.axis];
    a.xcd_remap = c->rot.xcd[a.axis];
    a.stream = c->rot.stream[a.axis];
  }
}

void after_pass(gpe_ctx *c, bool trans) {
  if (trans) std::swap(c->psi, c->psi_alt);
}

gpe_status real_step(gpe_ctx *c, void *const K[3], double tau_pre, double tau_post,
                     const VAt *pre, const VAt *post) {
  const int na = n_axes(c);
  const bool trans = use_trans(c);
  if (trans) {
    gpe_status ast = ensure_alt(c);
    if (ast != GPE_OK) return ast;
  }
  for (int i = 0; i < na; ++i) {
    const int ax = trans ? kTransOrder[i] : order_axis(c, i);
    // The closing phase's potential goes to the second table region when the
    // same pass also opens the step (one axis), else over the opening one
    // (stream order: the first pass has read it by then).
    const bool closing = i == na - 1 && tau_post != 0 && post;
    const int post_region = (i == 0 && pre) ? 1 : 0;
    gpe_status vst = GPE_OK;
    if (i == 0 && pre) vst = vtables_at(c, *pre, 0);
    if (vst == GPE_OK && closing) vst = vtables_at(c, *post, post_region);
    if (vst != GPE_OK) return vst;
    gpe::PassArgs a = base_args(c, ax);
    if (closing && post_region == 1) a.vtab_post = c->vtab + vtab_len(c);
    a.mid = gpe::MID_TABLE;
    a.mtab = K[ax];
    if (i == 0) {
      a.pre = gpe::PH_REAL;
      a.tau_pre = tau_pre;
    }
    if (i == na - 1 && tau_post != 0) {
      a.post = gpe::PH_REAL;
      a.tau_post = tau_post;
    }
    route(c, a, trans);
    gpe_status st = launch_pass(c, a);
    if (st != GPE_OK) return st;
    after_pass(c, trans);
  }
  return GPE_OK;
}

// One imaginary-time step: the pending scale and N(dt/2) before the first
// pass, N(dt/2) and the norm reduction after the last; the finalize kernel
// turns the reduction into the next scale.  The axes go in the reverse of the
// real-time order, so that the closing pass, whose phase and reduction need
// the most registers, is the contiguous-axis pass (on a strided axis it
// spills at 16 columns and runs on 8): 2.94 instead of 3.42 ms per step at
// 512^3 FP64 when this was chosen, 0.301 instead of 0.327 at 256^3.
gpe_status imag_step(gpe_ctx *c, void *const K[3], double dt) {
  const int na = n_axes(c);
  const bool trans = use_trans(c);
  if (trans) {
    gpe_status ast = ensure_alt(c);
    if (ast != GPE_OK) return ast;
  }
  for (int i = 0; i < na; ++i) {
    const int ax = trans ? kTransOrder[i] : order_axis(c, na - 1 - i);
    gpe::PassArgs a = base_args(c, ax);
    a.mid = gpe::MID_TABLE;
    a.mtab = K[ax];
    const bool exact = c->imag_method == GPE_IMAG_EXACT;
    const int op = exact ? gpe::PH_IMAG_EXACT : gpe::PH_IMAG;
    if (exact) a.mu_shift = c->scale + 1;
    if (i == 0) {
      a.scale = c->scale;
      a.pre = op;
      a.tau_pre = dt / 2;
    }
    if (i == na - 1) {
      a.post = op;
      a.tau_post = dt / 2;
      a.red = gpe::RED_NORM_OUT;
      a.partial = c->partial;
    }
    route(c, a, trans);
    gpe_status st = launch_pass(c, a);
    if (st != GPE_OK) return st;
    after_pass(c, trans);
    if (i == na - 1) {
      const gpe::PassShape sh = gpe::launch_shape(c->prec, a);
      HIPCHK(c, gpe::launch_finalize(c->partial, sh.blocks, c->sums + 3 * gpe::kRedSlots,
                                     c->scale, c->desc.norm_target, c->dV, c->stream, c->fin,
                                     exact ? dt : 0.0),
             "finalize launch");
    }
  }
  return GPE_OK;
}

bool graphs_allowed(const gpe_ctx *c) { return !c->timing && c->sites <= kGraphSites; }

// A graph of len identical steady-state steps (real: N(dt) first, no closing
// phase; imaginary: every step), cached per (mode, dt, len).  Null if the
// context stream cannot be captured; the caller then launches directly.
hipGraphExec_t step_graph(gpe_ctx *c, int mode, double dt, int len, void *const K[3]) {
  const auto key = std::make_tuple(mode, dt, len);
  auto it = c->step_graphs.find(key);
  if (it != c->step_graphs.end()) return it->second;
  if (c->step_graphs.size() >= kMaxStepGraphs) drop_step_graphs(c);
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  const std::string err = c->err;  // a failed capture leaves no error behind
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  bool ok = true;
  for (int s = 0; s < len && ok; ++s)
    ok = (mode == 0 ? real_step(c, K, dt, 0.0, nullptr, nullptr) : imag_step(c, K, dt)) == GPE_OK;
  const bool ended = hipStreamEndCapture(c->stream, &g) == hipSuccess;
  if (ok && ended && g) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!(ok && ended) || !ge) {
    (void)hipGetLastError();
    c->err = err;
    return nullptr;
  }
  c->step_graphs[key] = ge;
  return ge;
}

// Run n steady-state steps: whole graphs of len steps where they fit and
// graphs are allowed, single launches for the rest.
gpe_status steady_steps(gpe_ctx *c, int mode, double dt, int64_t n, int len, void *const K[3]) {
  if (graphs_allowed(c) && n >= len && len >= 2) {
    if (hipGraphExec_t ge = step_graph(c, mode, dt, len, K)) {
      for (; n >= len; n -= len) HIPCHK(c, hipGraphLaunch(ge, c->stream), "step graph launch");
    }
  }
  for (; n > 0; --n) {
    gpe_status st = mode == 0 ? real_step(c, K, dt, 0.0, nullptr, nullptr) : imag_step(c, K, dt);
    if (st != GPE_OK) return st;
  }
  return GPE_OK;
}

void drop_step_graphs(gpe_ctx *c) {
  if (c->step_graphs.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto &kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
  c->step_graphs.clear();
}

}  // namespace gpe_host

extern "C" {

gpe_status gpe_evolve(gpe_ctx *c, double dt, int64_t nsteps) {
  if (!c) return GPE_EINVAL;
  if (!std::isfinite(dt) || dt == 0) return fail(c, GPE_EINVAL, "dt must be finite and nonzero");
  if (nsteps < 0) return fail(c, GPE_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return GPE_OK;
  void *K[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < n_axes(c); ++i) {
    const int ax = order_axis(c, i);
    gpe_status st = get_table(c, ax, TB_KREAL, dt, &K[ax]);
    if (st != GPE_OK) return st;
  }
  // Adjacent half-steps of N are fused: the first step opens with N(dt/2),
  // the others with N(dt), and the last closes with N(dt/2).
  const double t0 = c->time;
  gpe_status st = GPE_OK;
  if (c->vfn) {
    // Time-dependent potential: step s covers [t_s, t_s + dt]; its N
    // half-steps take V at the midpoints t_s + dt/4 and t_s + 3 dt/4, and a
    // fused N(dt) the mean of the two midpoints it joins.
    const VAt close{t0 + nsteps * dt - dt / 4, 1.0, 0.0, 0.0};
    for (int64_t s = 0; s < nsteps && st == GPE_OK; ++s) {
      const double ts = t0 + s * dt;
      const VAt open = s == 0 ? VAt{t0 + dt / 4, 1.0, 0.0, 0.0}
                              : VAt{ts - dt / 4, 0.5, ts + dt / 4, 0.5};
      st = real_step(c, K, s == 0 ? dt / 2 : dt, s == nsteps - 1 ? dt / 2 : 0.0, &open, &close);
    }
  } else if (nsteps == 1) {
    st = real_step(c, K, dt / 2, dt / 2, nullptr, nullptr);
  } else {
    st = real_step(c, K, dt / 2, 0.0, nullptr, nullptr);
    if (st == GPE_OK) st = steady_steps(c, 0, dt, nsteps - 2, kGraphSteps, K);
    if (st == GPE_OK) st = real_step(c, K, dt, dt / 2, nullptr, nullptr);
  }
  if (st == GPE_OK) c->time = t0 + nsteps * dt;
  return st;
}

gpe_status gpe_evolve_record(gpe_ctx *c, double dt, int64_t nsteps, int32_t every,
                             gpe_obs *series, int64_t capacity, int64_t *count) {
  if (!c) return GPE_EINVAL;
  if (!series || !count) return fail(c, GPE_EINVAL, "series or count is NULL");
  if (every < 1) return fail(c, GPE_EINVAL, "every must be >= 1");
  if (nsteps < 0) return fail(c, GPE_EINVAL, "nsteps must be >= 0");
  const int64_t need = (nsteps + every - 1) / every;
  *count = 0;
  if (capacity < need) return fail(c, GPE_EINVAL, "series capacity is below ceil(nsteps/every)");
  if (need == 0) return GPE_OK;
  const size_t rec = 3 * gpe::kRedSlots;
  double *dev = nullptr;
  gpe_status st = dalloc(c, (void **)&dev, need * rec * sizeof(double), "series allocation");
  if (st != GPE_OK) return st;
  int64_t k = 0;
  for (int64_t done = 0; done < nsteps && st == GPE_OK; ++k) {
    const int64_t n = std::min<int64_t>(every, nsteps - done);
    st = gpe_evolve(c, dt, n);
    if (st == GPE_OK) st = enqueue_observe(c, nullptr, dev + k * rec);
    done += n;
  }
  std::vector<double> h(need * rec, 0.0);
  if (st == GPE_OK) {
    hipError_t e = hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = hipfail(c, e, "series download");
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(dev);
  c->dev_bytes -= need * rec * sizeof(double);
  if (st != GPE_OK) return st;
  gpe_status first_bad = GPE_OK;
  for (int64_t j = 0; j < need; ++j) {
    const gpe_status sj = obs_from_sums(c, &h[j * rec], &series[j]);
    if (sj != GPE_OK && first_bad == GPE_OK) first_bad = sj;
  }
  *count = need;
  return first_bad;
}

gpe_status gpe_ground_state(gpe_ctx *c, double dt, double tol, int32_t check_every,
                            int64_t max_steps, int64_t *steps_done, double *energy) {
  if (!c) return GPE_EINVAL;
  if (!(std::isfinite(dt) && dt > 0)) return fail(c, GPE_EINVAL, "dt must be positive");
  if (check_every < 0 || max_steps < 0) return fail(c, GPE_EINVAL, "negative count");
  if (check_every > 0 && !(tol >= 0)) return fail(c, GPE_EINVAL, "tol must be >= 0");
  void *K[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < n_axes(c); ++i) {
    const int ax = order_axis(c, i);
    gpe_status st = get_table(c, ax, TB_KIMAG, dt, &K[ax]);
    if (st != GPE_OK) return st;
  }
  // a time-dependent potential enters at the current clock (imaginary time
  // does not advance it)
  gpe_status vst = vtables_at(c, VAt{c->time, 1.0, 0.0, 0.0});
  if (vst != GPE_OK) return vst;
  // scale c = 1 and, for the exact substep, the chemical-potential shift 0
  const double init[2] = {1.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(c->scale, init, sizeof(init), hipMemcpyHostToDevice, c->stream),
         "scale reset");
  double e_prev = NAN, e_last = NAN;
  if (check_every > 0) {
    gpe_obs o;
    gpe_status st = compute_obs(c, nullptr, &o);
    if (st != GPE_OK) return st;
    e_prev = o.energy;
  }
  gpe_status result = check_every > 0 ? GPE_ENOTCONV : GPE_OK;
  // Steps between two checks are identical; on small grids they replay from
  // a graph of check_every steps (32 without checks or when checks are rare).
  const int len = (check_every >= 2 && check_every <= 64) ? check_every : kGraphSteps;
  int64_t s = 0;
  while (s < max_steps) {
    int64_t run = max_steps - s;
    if (check_every > 0) run = std::min<int64_t>(run, check_every - s % check_every);
    gpe_status st = steady_steps(c, 1, dt, run, len, K);
    if (st != GPE_OK) return st;
    s += run;
    if (check_every > 0 && s % check_every == 0) {
      gpe_obs o;
      st = compute_obs(c, c->scale, &o);
      if (st != GPE_OK) return st;
      e_last = o.energy;
      const bool done = std::fabs(o.energy - e_prev) < tol;
      e_prev = o.energy;
      if (done) {
        result = GPE_OK;
        break;
      }
    }
  }
  HIPCHK(c, gpe::launch_scale(c->prec, c->psi, c->sites, c->scale, c->stream), "scale launch");
  HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  if (steps_done) *steps_done = s;
  if (energy) *energy = e_last;
  if (result == GPE_ENOTCONV) return fail(c, GPE_ENOTCONV, "ground state did not converge");
  return result;
}

gpe_status gpe_observables(gpe_ctx *c, gpe_obs *out, gpe_spectra *spec) {
  if (!c) return GPE_EINVAL;
  if (!out) return fail(c, GPE_EINVAL, "out is NULL");
  if (!spec) return compute_obs(c, nullptr, out);
  return compute_spectra(c, spec, out);
}

int32_t gpe_spectra_bins(const gpe_ctx *c) {
  if (!c) return -1;
  return shell_count(c);
}

gpe_status gpe_transform(gpe_ctx *c, int32_t axis_mask, int32_t inverse) {
  if (!c) return GPE_EINVAL;
  if (axis_mask & ~((1 << c->dim) - 1)) return fail(c, GPE_EINVAL, "axis_mask names a missing axis");
  for (int j = 0; j < c->dim; ++j) {
    if (!(axis_mask & (1 << j))) continue;
    const int ax = view_axis(c, j);
    gpe::PassArgs a = base_args(c, ax);
    if (inverse) {
      void *tab = nullptr;
      gpe_status st = get_table(c, ax, TB_INVN, 0.0, &tab);
      if (st != GPE_OK) return st;
      a.forward = 0;
      a.mid = gpe::MID_TABLE;
      a.mtab = tab;
    } else {
      a.inverse = 0;
    }
    gpe_status st = launch_pass(c, a);
    if (st != GPE_OK) return st;
  }
  return GPE_OK;
}

gpe_status gpe_synchronize(gpe_ctx *c) {
  if (!c) return GPE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "stream sync");
  return GPE_OK;
}

gpe_status gpe_timing_enable(gpe_ctx *c, int32_t on) {
  if (!c) return GPE_EINVAL;
  gpe_status st = drain_timing(c);
  if (st != GPE_OK) return st;
  c->kinds.clear();
  c->timing = on != 0;
  return GPE_OK;
}

gpe_status gpe_timing_read(gpe_ctx *c, gpe_timing *out) {
  if (!c || !out) return GPE_EINVAL;
  gpe_status st = drain_timing(c);
  if (st != GPE_OK) return st;
  std::memset(out, 0, sizeof(*out));
  out->count = (int32_t)std::min<size_t>(GPE_TIMING_KINDS, c->kinds.size());
  for (int i = 0; i < out->count; ++i) {
    std::snprintf(out->name[i], sizeof(out->name[i]), "%s", c->kinds[i].name.c_str());
    out->total_ms[i] = c->kinds[i].total_ms;
    out->launches[i] = c->kinds[i].launches;
    out->bytes[i] = c->kinds[i].bytes;
  }
  return GPE_OK;
}

uint64_t gpe_device_bytes(const gpe_ctx *c) { return c ? c->dev_bytes : 0; }

int32_t gpe_device(const gpe_ctx *c) { return c ? c->device : -1; }

void *gpe_stream(const gpe_ctx *c) { return c ? static_cast<void *>(c->stream) : nullptr; }

const char *gpe_last_error(const gpe_ctx *c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void gpe_destroy(gpe_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &pe : c->pending) c->event_pool.push_back(pe.second);
  for (auto &ev : c->event_pool) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  for (auto &kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : c->tables) (void)hipFree(kv.second);
  for (int j = 0; j < 3; ++j) {
    if (c->tw[j]) (void)hipFree(c->tw[j]);
    if (c->kw[j]) (void)hipFree(c->kw[j]);
  }
  if (c->psi) (void)hipFree(c->psi);
  if (c->psi_alt) (void)hipFree(c->psi_alt);
  for (int j = 0; j < 3; ++j)
    if (c->work[j]) (void)hipFree(c->work[j]);
  if (c->hist_partial) (void)hipFree(c->hist_partial);
  if (c->hist) (void)hipFree(c->hist);
  if (c->V) (void)hipFree(c->V);
  if (c->vtab) (void)hipFree(c->vtab);
  if (c->partial) (void)hipFree(c->partial);
  if (c->sums) (void)hipFree(c->sums);
  if (c->scale) (void)hipFree(c->scale);
  if (c->fin) (void)hipFree(c->fin);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
