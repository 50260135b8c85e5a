// Allocation-free TSSP steps on a caller-owned device state.
//
// The same fused axis passes, finalize and scale kernels as gpe_evolve and
// gpe_ground_state, with every buffer they need beyond the state -- the
// twiddle and kinetic-factor tables, the per-workgroup partial sums, the
// finalized sums and the renormalisation factor -- placed in one file-scope
// device array instead of memory the library allocates.  Nothing here calls
// hipMalloc or hipFree: for callers that cannot allocate device memory.
//
// Each device holds its own copy of `scratch` for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in, not a
// device address).  Calls on one device share that copy: calls that overlap
// on one device race.  Nothing in it is assumed to start at any value: every
// call rewrites the tables and the factor before its first pass, and every
// partial sum is written before it is read.
#include "gpe.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "gpe_ctx.h"
#include "gpe_kernels.h"

namespace {

constexpr size_t kScratchBytes = GPE_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current).
gpe_status scratch_of(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return GPE_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return GPE_EDEVICE;
    }
    g_scratch[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch[dev];
  return GPE_OK;
}

struct TableArgs {
  int n[3];        // 3D view
  double L[3];     // box lengths (view axes)
  double dt;
  int imag;        // kinetic factor exp(-k^2 dt/2)/N (1) or exp(-i k^2 dt/2)/N (0)
  int fp32_pairs;  // entries as FP32 hi + lo pairs (the FP32 form)
  void *tw[3];     // exp(-2 pi i j / N), N entries of 16 bytes
  void *kin[3];    // kinetic factor per frequency index, N entries of 16 bytes
  double *scale;   // renormalisation factor (1) and chemical-potential shift (0)
};

__device__ void put(void *tab, int i, double re, double im, int fp32_pairs) {
  if (fp32_pairs) {
    const float rh = (float)re, ih = (float)im;
    reinterpret_cast<float4 *>(tab)[i] =
        make_float4(rh, ih, (float)(re - (double)rh), (float)(im - (double)ih));
  } else {
    reinterpret_cast<double2 *>(tab)[i] = make_double2(re, im);
  }
}

// One thread per (axis, index): twiddles and kinetic factors, each entry
// computed from its own index in FP64.
__global__ void __launch_bounds__(256) tables_kernel(const TableArgs a) {
  const double pi = 3.14159265358979323846264338327950288;
  const int j = blockIdx.x * blockDim.x + threadIdx.x, ax = blockIdx.y;
  if (ax == 0 && j == 0 && a.scale) {
    a.scale[0] = 1.0;
    a.scale[1] = 0.0;
  }
  const int N = a.n[ax];
  if (!a.tw[ax] || j >= N) return;
  const double ang = 2 * pi * (double)j / (double)N;
  put(a.tw[ax], j, cos(ang), -sin(ang), a.fp32_pairs);
  const int m = j < N / 2 ? j : j - N;
  const double k = 2 * pi * (double)m / a.L[ax], inv = 1.0 / (double)N;
  const double ph = k * k * a.dt / 2;
  if (a.imag) put(a.kin[ax], j, exp(-ph) * inv, 0.0, a.fp32_pairs);
  else put(a.kin[ax], j, cos(ph) * inv, -sin(ph) * inv, a.fp32_pairs);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

using namespace gpe_host;

extern "C" gpe_status gpe_steps_noalloc(const gpe_desc *desc, const gpe_harmonic *trap,
                                        void *psi_dev, int32_t imaginary, double dt,
                                        int64_t nsteps, void *hip_stream) {
  std::string msg;
  if (!desc || !psi_dev) return fail(nullptr, GPE_EINVAL, "desc or psi_dev is NULL");
  gpe_status st = validate_desc(desc, msg);
  if (st != GPE_OK) return fail(nullptr, st, msg);
  if (imaginary != 0 && imaginary != 1) return fail(nullptr, GPE_EINVAL, "imaginary must be 0 or 1");
  if (!std::isfinite(dt) || dt == 0 || (imaginary && dt < 0))
    return fail(nullptr, GPE_EINVAL, "dt must be finite and nonzero (positive in imaginary time)");
  if (nsteps < 0) return fail(nullptr, GPE_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return GPE_OK;

  // A context on the stack that owns nothing: the caller's state and stream,
  // the launch shapes of its shape class, and pointers into the scratch.
  gpe_ctx c;
  c.desc = *desc;
  c.dim = desc->dim;
  c.prec = desc->precision;
  c.esize = gpe::state_f32(c.prec) ? 8 : 16;
  c.sites = 1;
  c.dV = 1;
  effective_tuning(*desc, c.wreq, c.xcd_remap, c.pass_order, c.plan, c.streaming);
  const int off = 3 - c.dim;
  for (int j = 0; j < c.dim; ++j) {
    c.n3[j + off] = desc->n[j];
    c.lo3[j + off] = desc->lo[j];
    c.L3[j + off] = desc->hi[j] - desc->lo[j];
    c.h3[j + off] = c.L3[j + off] / desc->n[j];
    c.sites *= desc->n[j];
    c.dV *= c.h3[j + off];
  }
  if (trap) {
    for (int j = 0; j < c.dim; ++j) {
      if (!std::isfinite(trap->w[j])) return fail(nullptr, GPE_EINVAL, "trap frequency not finite");
      c.hv[j + off] = 0.5 * trap->w[j] * trap->w[j];
    }
  }
  if (hipGetDevice(&c.device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, GPE_EDEVICE, "no current HIP device");
  }
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.psi = psi_dev;

  // Scratch layout: per axis the twiddles and the kinetic factor (16 bytes
  // per entry); imaginary time adds the factor, the finalized sums, the
  // two-stage finalize rows and one region of per-workgroup partials.
  size_t need = 0;
  size_t tw_off[3] = {0, 0, 0}, kin_off[3] = {0, 0, 0};
  for (int ax = off; ax < 3; ++ax) {
    tw_off[ax] = need;
    need = align256(need + (size_t)c.n3[ax] * 16);
    kin_off[ax] = need;
    need = align256(need + (size_t)c.n3[ax] * 16);
  }
  size_t scale_off = 0, sums_off = 0, fin_off = 0, part_off = 0;
  if (imaginary) {
    long long maxb = 1;
    for (int ax = off; ax < 3; ++ax) {
      const gpe::PassShape sh = gpe::pass_shape(c.prec, c.n3, ax, c.wreq[ax], c.plan[ax], true);
      if (sh.blocks > maxb) maxb = sh.blocks;
    }
    c.partial_region = maxb * gpe::kRedSlots;
    scale_off = need;
    need = align256(need + 2 * sizeof(double));
    sums_off = need;
    need = align256(need + 4 * gpe::kRedSlots * sizeof(double));
    fin_off = need;
    need = align256(need + gpe::kFinBlocks * gpe::kRedSlots * sizeof(double));
    part_off = need;
    need = align256(need + (size_t)c.partial_region * sizeof(double));
  }
  if (need > kScratchBytes)
    return fail(nullptr, GPE_EUNSUPPORTED,
                "grid needs " + std::to_string(need) + " bytes of scratch, above the " +
                    std::to_string(kScratchBytes) + " of the allocation-free path");
  unsigned char *base = nullptr;
  if ((st = scratch_of(c.device, &base)) != GPE_OK)
    return fail(nullptr, st, "scratch lookup failed on device " + std::to_string(c.device));

  TableArgs ta{};
  void *K[3] = {nullptr, nullptr, nullptr};
  for (int ax = 0; ax < 3; ++ax) {
    ta.n[ax] = c.n3[ax];
    ta.L[ax] = c.L3[ax];
    if (ax >= off) {
      c.tw[ax] = base + tw_off[ax];
      K[ax] = base + kin_off[ax];
      ta.tw[ax] = c.tw[ax];
      ta.kin[ax] = K[ax];
    }
  }
  ta.dt = dt;
  ta.imag = imaginary;
  ta.fp32_pairs = c.prec == GPE_FP32 ? 1 : 0;
  if (imaginary) {
    c.scale = reinterpret_cast<double *>(base + scale_off);
    c.sums = reinterpret_cast<double *>(base + sums_off);
    c.fin = reinterpret_cast<double *>(base + fin_off);
    c.partial = reinterpret_cast<double *>(base + part_off);
    ta.scale = c.scale;
  }
  int nmax = 1;
  for (int ax = 0; ax < 3; ++ax) nmax = c.n3[ax] > nmax ? c.n3[ax] : nmax;
  hipLaunchKernelGGL(tables_kernel, dim3((nmax + 255) / 256, 3), dim3(256), 0, c.stream, ta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, GPE_EDEVICE, std::string("table launch: ") + hipGetErrorString(e));

  if (!imaginary) {
    // as gpe_evolve: the opening N(dt/2), fused N(dt) between steps, the closing N(dt/2)
    if (nsteps == 1) {
      st = real_step(&c, K, dt / 2, dt / 2, nullptr, nullptr);
    } else {
      st = real_step(&c, K, dt / 2, 0.0, nullptr, nullptr);
      for (int64_t s = 1; s + 1 < nsteps && st == GPE_OK; ++s)
        st = real_step(&c, K, dt, 0.0, nullptr, nullptr);
      if (st == GPE_OK) st = real_step(&c, K, dt, dt / 2, nullptr, nullptr);
    }
  } else {
    // as gpe_ground_state with check_every = 0: renormalised steps, the last
    // factor applied at the end
    for (int64_t s = 0; s < nsteps && st == GPE_OK; ++s) st = imag_step(&c, K, dt);
    if (st == GPE_OK) {
      e = gpe::launch_scale(c.prec, c.psi, c.sites, c.scale, c.stream);
      if (e != hipSuccess) st = fail(&c, GPE_EDEVICE, std::string("scale launch: ") + hipGetErrorString(e));
    }
  }
  if (st != GPE_OK) return fail(nullptr, st, c.err);
  return GPE_OK;
}
