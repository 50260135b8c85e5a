// On-chip batched TSSP steps for small square 2D grids.
//
// A grid of n x n sites whose state fits one workgroup's LDS (n <= 64 in
// FP64, n <= 128 in FP32) is loaded once, advanced by several steps of the
// Strang splitting (Numerical Scheme section) entirely in LDS, and stored
// once: no HBM traffic and no launch between the steps.  One workgroup per
// slot of a batched shape class, so a launch advances every request of the
// class.  Each step is two axis passes over the LDS-resident grid: the lines
// along one axis (real-space phase, forward DFT, kinetic factor, inverse
// DFT), then the lines along the other (the same, then the closing phase).
// The per-line arithmetic is that of the HBM-streaming axis pass: same plans,
// stages, tables, phase and potential code, so both paths give the same
// result up to the order of the norm sum of the imaginary-time method.
#include "axis_pass.h"

namespace gpe {
namespace pass {
namespace {

template <typename T, int N>
struct OC {
  using PL = typename PlanFor<N>::type;
  static constexpr int E = PL::E, TPL = PL::TPL;
  // threads: one per E points, at most 512 (two waves per SIMD, so the
  // kernel may use up to 256 VGPRs and keeps its registers)
  static constexpr int TH = (N * N / E) < 512 ? (N * N / E) : 512;
  static constexpr int LR = TH / TPL;                                  // lines per round
  static constexpr int ROUNDS = N / LR;
  // Row stride: one padding slot per eight points plus four, so that the rows
  // a wavefront touches start on different banks.
  static constexpr int RS = N + N / 8 + 4;
  static constexpr int SIZE = N * RS;
  static_assert(LR * ROUNDS == N, "rounds must cover the lines");
  static_assert(2 * SIZE * sizeof(T) + 64 * sizeof(double) <= 160 * 1024, "fits LDS");
};

// An opaque zero.  Every quantity of a pass derived from it (LDS addresses,
// coordinates, table pointers) is recomputed in each round and step instead
// of being hoisted out of the step loop and held in registers for all of it,
// which would double the register use and spill.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Move the registers of one line from the stage-A to the stage-B layout
// through the line's own LDS locations.
template <class PL, int A, int B, typename T, typename F>
__device__ __forceinline__ void oc_exchange(cx<T> *v, int t, T *lre, T *lim, F at, bool first) {
  constexpr int RA = PL::rad(A), RB = PL::rad(B), E = PL::E, TPL = PL::TPL;
  if (!first) __syncthreads();
#pragma unroll
  for (int b = 0; b < E / RA; ++b)
#pragma unroll
    for (int d = 0; d < RA; ++d) {
      const int i = at(PL::pos(A, t + TPL * b, d));
      lre[i] = v[b * RA + d].x;
      lim[i] = v[b * RA + d].y;
    }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < E / RB; ++b)
#pragma unroll
    for (int d = 0; d < RB; ++d) {
      const int i = at(PL::pos(B, t + TPL * b, d));
      v[b * RB + d].x = lre[i];
      v[b * RB + d].y = lim[i];
    }
}

// One axis pass over the LDS-resident grid: ROWS = lines along the last axis
// (view axis 2), else along the first (view axis 1).  The closing phase of an
// imaginary-time step also accumulates sum |psi|^2 into nacc.
template <typename T, int N, bool ROWS>
__device__ __forceinline__ void oc_pass(T *lre, T *lim, const tab_t<T> *__restrict__ tw,
                                        const tab_t<T> *__restrict__ kt, int pre, double tau_pre,
                                        int post, double tau_post, double g,
                                        const double (&hv)[3], int vkind,
                                        const double (&lo)[3], const double (&h)[3],
                                        double &nacc) {
  using C = OC<T, N>;
  using PL = typename C::PL;
  constexpr int E = PL::E, TPL = PL::TPL, R0 = PL::rad(0), RL = PL::rad(PL::M - 1);
  const int tid = threadIdx.x;
  const int c0 = ROWS ? tid / TPL : tid % C::LR;
  const int t = ROWS ? tid % TPL : tid / C::LR;
  for (int r = 0; r < C::ROUNDS; ++r) {
    const int z = opaque_zero();
    const int c = r * C::LR + c0 + z;
    const tab_t<T> *__restrict__ twz = tw + z;
    const tab_t<T> *__restrict__ ktz = kt + z;
    const int tz = t + z;
    auto at = [c](int p) {
      return ROWS ? c * C::RS + p + (p >> 3) : p * C::RS + c + (c >> 3);
    };
    cx<T> v[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const int p = PL::pos(0, tz + TPL * b, d);
        const int i = at(p);
        cx<T> u{lre[i], lim[i]};
        if (pre != PH_NONE) {
          const double V = vkind == V_HARMONIC
                               ? harmonic_potential(lo, h, hv, 0, ROWS ? c : p, ROWS ? p : c)
                               : 0.0;
          u = apply_phase(pre, u, V, g, tau_pre);
        }
        v[b * R0 + d] = u;
      }
    stage<PL, 0, -1>(v, tz, twz);
    if constexpr (PL::M > 1) {
      oc_exchange<PL, 0, 1>(v, tz, lre, lim, at, true);
      stage<PL, 1, -1>(v, tz, twz);
    }
    if constexpr (PL::M > 2) {
      oc_exchange<PL, 1, 2>(v, tz, lre, lim, at, false);
      stage<PL, 2, -1>(v, tz, twz);
    }
    if constexpr (PL::M > 3) {
      oc_exchange<PL, 2, 3>(v, tz, lre, lim, at, false);
      stage<PL, 3, -1>(v, tz, twz);
    }
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int d = 0; d < RL; ++d) {
        const int f = PL::freq(PL::pos(PL::M - 1, tz + TPL * b, d));
        v[b * RL + d] = table_mul(v[b * RL + d], ktz[f]);
      }
    if constexpr (PL::M > 3) {
      stage<PL, 3, +1>(v, tz, twz);
      oc_exchange<PL, 3, 2>(v, tz, lre, lim, at, false);
    }
    if constexpr (PL::M > 2) {
      stage<PL, 2, +1>(v, tz, twz);
      oc_exchange<PL, 2, 1>(v, tz, lre, lim, at, false);
    }
    if constexpr (PL::M > 1) {
      stage<PL, 1, +1>(v, tz, twz);
      oc_exchange<PL, 1, 0>(v, tz, lre, lim, at, false);
    }
    stage<PL, 0, +1>(v, tz, twz);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const int p = PL::pos(0, tz + TPL * b, d);
        cx<T> u = v[b * R0 + d];
        if (post != PH_NONE) {
          const double V = vkind == V_HARMONIC
                               ? harmonic_potential(lo, h, hv, 0, ROWS ? c : p, ROWS ? p : c)
                               : 0.0;
          u = apply_phase(post, u, V, g, tau_post);
          if (post == PH_IMAG) nacc += (double)u.x * u.x + (double)u.y * u.y;
        }
        const int i = at(p);
        lre[i] = u.x;
        lim[i] = u.y;
      }
  }
}

template <typename T, int N, bool ROWS_FIRST>
__global__ void __launch_bounds__((OC<T, N>::TH)) onchip_kernel(const OnchipArgs a) {
  using C = OC<T, N>;
  __shared__ T lre[C::SIZE], lim[C::SIZE];
  __shared__ double red[64];
  __shared__ double bcast;
  Slot &sl = a.slots[a.slot_map[blockIdx.x]];
  const int mode = sl.mode, total = sl.steps_total, done0 = sl.steps_done;
  if (mode == SLOT_FREE || done0 >= total) return;
  const int K = min(a.steps, total - done0);
  const bool im = mode == SLOT_IMAG;
  const double g = sl.g, norm_target = sl.norm_target;
  const double hv[3] = {sl.hv[0], sl.hv[1], sl.hv[2]};
  // (copied: references into the kernel arguments would move them to
  // private memory)
  const double lo[3] = {a.lo[0], a.lo[1], a.lo[2]}, h[3] = {a.h[0], a.h[1], a.h[2]};
  const int vkind = (hv[0] != 0 || hv[1] != 0 || hv[2] != 0) ? V_HARMONIC : V_NONE;
  cx<T> *psi = static_cast<cx<T> *>(sl.psi);
  const tab_t<T> *tw_row = static_cast<const tab_t<T> *>(a.tw_row);
  const tab_t<T> *tw_col = static_cast<const tab_t<T> *>(a.tw_col);
  const tab_t<T> *k_row = static_cast<const tab_t<T> *>(im ? a.ki_row : a.kr_row);
  const tab_t<T> *k_col = static_cast<const tab_t<T> *>(im ? a.ki_col : a.kr_col);
  const int tid = threadIdx.x;

  // Load, with the imaginary-time factor still pending from a previous launch.
  const double sc0 = im ? sl.scale : 1.0;
  for (int i = tid; i < N * N; i += C::TH) {
    const int r = i / N, q = i % N;
    cx<T> u = psi[i];
    if (im) u = {(T)(sc0 * (double)u.x), (T)(sc0 * (double)u.y)};
    lre[r * C::RS + q + (q >> 3)] = u.x;
    lim[r * C::RS + q + (q >> 3)] = u.y;
  }
  __syncthreads();

  for (int s = 0; s < K; ++s) {
    const int step = done0 + s;
    // Real time: adjacent half-step phases fuse into one of dt, except at the
    // first and last step of the request.  Imaginary time: dt/2 on both sides.
    const int ph = im ? PH_IMAG : PH_REAL;
    const double tau_pre = (im || step == 0) ? 0.5 * a.dt : a.dt;
    const int post = (im || step == total - 1) ? ph : PH_NONE;
    const double tau_post = 0.5 * a.dt;
    double nacc = 0;
    if constexpr (ROWS_FIRST) {
      oc_pass<T, N, true>(lre, lim, tw_row, k_row, ph, tau_pre, PH_NONE, 0.0, g, hv, vkind, lo, h,
                          nacc);
      __syncthreads();
      oc_pass<T, N, false>(lre, lim, tw_col, k_col, PH_NONE, 0.0, post, tau_post, g, hv, vkind,
                           lo, h, nacc);
    } else {
      oc_pass<T, N, false>(lre, lim, tw_col, k_col, ph, tau_pre, PH_NONE, 0.0, g, hv, vkind, lo,
                           h, nacc);
      __syncthreads();
      oc_pass<T, N, true>(lre, lim, tw_row, k_row, PH_NONE, 0.0, post, tau_post, g, hv, vkind, lo,
                          h, nacc);
    }
    __syncthreads();
    if (im) {
      // Renormalise: fixed-order block sum of |psi|^2, then c applied in LDS.
      if constexpr (C::TH >= 64) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) nacc += __shfl_xor(nacc, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = nacc;
      } else {
        red[tid] = nacc;
      }
      __syncthreads();
      if (tid == 0) {
        const int nr = C::TH >= 64 ? C::TH / 64 : C::TH;
        double sum = 0;
        for (int w = 0; w < nr; ++w) sum += red[w];
        bcast = sqrt(norm_target / (a.dV * sum));
      }
      __syncthreads();
      const double sc = bcast;
      for (int i = tid; i < N * N; i += C::TH) {
        const int r = i / N, q = i % N;
        const int j = r * C::RS + q + (q >> 3);
        lre[j] = (T)(sc * (double)lre[j]);
        lim[j] = (T)(sc * (double)lim[j]);
      }
      __syncthreads();
    }
  }

  for (int i = tid; i < N * N; i += C::TH) {
    const int r = i / N, q = i % N;
    psi[i] = cx<T>{lre[r * C::RS + q + (q >> 3)], lim[r * C::RS + q + (q >> 3)]};
  }
  if (tid == 0) {
    sl.steps_done = done0 + K;
    sl.scale = 1.0;
  }
}

template <typename T, int N>
hipError_t launch_oc(const OnchipArgs &a, int rows, hipStream_t s) {
  if (a.rows_first)
    hipLaunchKernelGGL((onchip_kernel<T, N, true>), dim3((unsigned)rows), dim3(OC<T, N>::TH), 0,
                       s, a);
  else
    hipLaunchKernelGGL((onchip_kernel<T, N, false>), dim3((unsigned)rows), dim3(OC<T, N>::TH),
                       0, s, a);
  return hipGetLastError();
}

}  // namespace
}  // namespace pass

bool onchip_supported(int precision, int n) {
  if (precision != 0 && precision != 1) return false;
  const int nmax = precision == 1 ? 128 : 64;
  return n >= 8 && n <= nmax && (n & (n - 1)) == 0;
}

hipError_t launch_onchip(int precision, const OnchipArgs &a, int rows, hipStream_t s) {
  using namespace pass;
  if (rows < 1 || a.steps < 1 || !a.slot_map || !onchip_supported(precision, a.n))
    return hipErrorInvalidValue;
  if (precision == 1) {
    switch (a.n) {
      case 8: return launch_oc<float, 8>(a, rows, s);
      case 16: return launch_oc<float, 16>(a, rows, s);
      case 32: return launch_oc<float, 32>(a, rows, s);
      case 64: return launch_oc<float, 64>(a, rows, s);
      case 128: return launch_oc<float, 128>(a, rows, s);
    }
  } else {
    switch (a.n) {
      case 8: return launch_oc<double, 8>(a, rows, s);
      case 16: return launch_oc<double, 16>(a, rows, s);
      case 32: return launch_oc<double, 32>(a, rows, s);
      case 64: return launch_oc<double, 64>(a, rows, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace gpe
