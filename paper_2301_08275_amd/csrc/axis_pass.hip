// Fused per-axis TSSP pass for gfx950.
//
// The spectral step of the method (Numerical Scheme section: the kinetic
// substep exp(-i |k|^2 dt/2) applied between a forward and an inverse DFT)
// factors over axes because |k|^2 = sum_j k_j^2 and the d-dimensional DFT is
// the product of one-dimensional DFTs along each axis.  One launch therefore
// treats one axis completely: each workgroup loads whole lines along that
// axis from HBM, optionally applies the real-space nonlinear/potential phase
// (pre), runs the forward DFT of every line through registers and LDS,
// multiplies by a per-frequency table (kinetic factor with 1/N, a spectral
// derivative, ...), runs the inverse DFT, optionally applies the phase again
// (post) and accumulates sums, and stores the lines back.  A 3D real-time step
// is three such launches: 32 bytes of HBM traffic per site per launch in FP64.
//
// FFT: mixed-radix (2/4/8/16) Cooley-Tukey, decimation in frequency for the
// forward transform (digit-reversed spectrum, never reordered) and the exact
// reverse for the inverse, so the spectrum is used in place.  Each thread
// holds E elements of one line; stages exchange through LDS.  Twiddles come
// from an FP64-accurate table exp(-2 pi i j/N) built on the host per index.
#include "gpe_kernels.h"

#include <cmath>

namespace gpe {
namespace {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// v * exp(SIGN * 2 pi i k / 16); k is a constant once loops are unrolled.
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot16(cx<T> v, int k) {
  const T r = T(0.70710678118654752440);
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  switch (k) {
    case 0: return v;
    case 1: return cmul(v, cx<T>{c1, SIGN * s1});
    case 2: return {r * (v.x - SIGN * v.y), r * (v.y + SIGN * v.x)};
    case 3: return cmul(v, cx<T>{s1, SIGN * c1});
    case 4: return {-SIGN * v.y, SIGN * v.x};
    case 5: return cmul(v, cx<T>{-s1, SIGN * c1});
    case 6: return {-r * (v.x + SIGN * v.y), r * (SIGN * v.x - v.y)};
    default: return cmul(v, cx<T>{-c1, SIGN * s1});
  }
}

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of R <= 16 points, natural order in and out:
// X[k] = sum_n x[n] exp(SIGN 2 pi i n k / R).  Radix-2 decimation in frequency.
template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft(cx<T> *v) {
#pragma unroll
  for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int b = 0; b < R; b += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        cx<T> a = v[b + j], c = v[b + j + h];
        v[b + j] = cadd(a, c);
        v[b + j + h] = rot16<SIGN>(csub(a, c), j * (16 / (2 * h)));
      }
    }
  }
  cx<T> t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] = v[i];
#pragma unroll
  for (int i = 0; i < R; ++i) v[bitrev<R>(i)] = t[i];
}

// Plan: N = R0 R1 R2 R3 points per line, E elements per thread, every radix
// divides E.  Stage s combines the elements whose position digit s differs:
// positions p = (q mod st) + (q / st) st R + d st, st = N / (P(s) R(s)),
// for butterfly q in [0, N/R) and digit d in [0, R).
template <int N_, int E_, int R0, int R1 = 1, int R2 = 1, int R3 = 1>
struct Plan {
  static constexpr int N = N_, E = E_, TPL = N_ / E_;
  static constexpr int M = (R1 == 1 ? 1 : (R2 == 1 ? 2 : (R3 == 1 ? 3 : 4)));
  __host__ __device__ static constexpr int rad(int s) {
    return s == 0 ? R0 : s == 1 ? R1 : s == 2 ? R2 : R3;
  }
  __host__ __device__ static constexpr int P(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= rad(i);
    return p;
  }
  __host__ __device__ static constexpr int stride(int s) { return N / (P(s) * rad(s)); }
  __host__ __device__ static constexpr int pos(int s, int q, int d) {
    return (q % stride(s)) + (q / stride(s)) * stride(s) * rad(s) + d * stride(s);
  }
  // Frequency held at position p after all forward stages (digit reversal).
  __host__ __device__ static constexpr int freq(int p) {
    int f = 0;
    for (int s = 0; s < M; ++s) f += ((p / stride(s)) % rad(s)) * P(s);
    return f;
  }
  static_assert(R0 * R1 * R2 * R3 == N_, "radices must multiply to N");
  static_assert(E_ % R0 == 0 && E_ % R1 == 0 && E_ % R2 == 0 && E_ % R3 == 0,
                "every radix divides E");
};

template <int N> struct PlanFor;
template <> struct PlanFor<8> { using type = Plan<8, 8, 8>; };
template <> struct PlanFor<16> { using type = Plan<16, 8, 8, 2>; };
template <> struct PlanFor<32> { using type = Plan<32, 8, 8, 4>; };
template <> struct PlanFor<64> { using type = Plan<64, 8, 8, 8>; };
template <> struct PlanFor<128> { using type = Plan<128, 8, 8, 8, 2>; };
template <> struct PlanFor<256> { using type = Plan<256, 8, 8, 8, 4>; };
template <> struct PlanFor<512> { using type = Plan<512, 8, 8, 8, 8>; };
template <> struct PlanFor<1024> { using type = Plan<1024, 16, 16, 8, 8>; };

// LDS layout of a tile of W lines of N points (separate re and im planes).
template <int N, int W, bool STRIDED>
struct Lds {
  // strided: rows of W columns, one pad slot per row; contiguous: one line
  // after the other, one pad slot per 16 points.
  static constexpr int size = STRIDED ? N * (W + 1) : W * (N + N / 16);
  __device__ static __forceinline__ int idx(int p, int c) {
    return STRIDED ? p * (W + 1) + c : c * (N + N / 16) + p + (p >> 4);
  }
};

// One forward (SIGN = -1: DFT then twiddle) or inverse (SIGN = +1: conjugate
// twiddle then DFT) stage S on the thread's E registers.
template <class PL, int S, int SIGN, typename T>
__device__ __forceinline__ void stage(cx<T> *v, int t, const cx<T> *__restrict__ tw) {
  constexpr int R = PL::rad(S), B = PL::E / R, ST = PL::stride(S), P = PL::P(S);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int q = t + PL::TPL * b;
    cx<T> *u = v + b * R;
    const int tb = P * (q % ST);
    if (SIGN < 0) {
      dft<R, -1>(u);
      if (ST > 1) {
#pragma unroll
        for (int d = 1; d < R; ++d) u[d] = cmul(u[d], tw[tb * d]);
      }
    } else {
      if (ST > 1) {
#pragma unroll
        for (int d = 1; d < R; ++d) u[d] = cmulc(u[d], tw[tb * d]);
      }
      dft<R, +1>(u);
    }
  }
}

// Move the E registers from the stage-A layout to the stage-B layout.
template <class PL, int W, bool STRIDED, int A, int B, typename T>
__device__ __forceinline__ void exchange(cx<T> *v, int t, int c, T *lre, T *lim,
                                         bool first) {
  using L = Lds<PL::N, W, STRIDED>;
  constexpr int RA = PL::rad(A), RB = PL::rad(B);
  if (!first) __syncthreads();
#pragma unroll
  for (int b = 0; b < PL::E / RA; ++b)
#pragma unroll
    for (int d = 0; d < RA; ++d) {
      const int i = L::idx(PL::pos(A, t + PL::TPL * b, d), c);
      lre[i] = v[b * RA + d].x;
      lim[i] = v[b * RA + d].y;
    }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < PL::E / RB; ++b)
#pragma unroll
    for (int d = 0; d < RB; ++d) {
      const int i = L::idx(PL::pos(B, t + PL::TPL * b, d), c);
      v[b * RB + d].x = lre[i];
      v[b * RB + d].y = lim[i];
    }
}

template <class PL, int W, bool STRIDED, typename T>
__device__ __forceinline__ void forward_fft(cx<T> *v, int t, int c, T *lre, T *lim,
                                            const cx<T> *tw) {
  stage<PL, 0, -1>(v, t, tw);
  if constexpr (PL::M > 1) {
    exchange<PL, W, STRIDED, 0, 1>(v, t, c, lre, lim, true);
    stage<PL, 1, -1>(v, t, tw);
  }
  if constexpr (PL::M > 2) {
    exchange<PL, W, STRIDED, 1, 2>(v, t, c, lre, lim, false);
    stage<PL, 2, -1>(v, t, tw);
  }
  if constexpr (PL::M > 3) {
    exchange<PL, W, STRIDED, 2, 3>(v, t, c, lre, lim, false);
    stage<PL, 3, -1>(v, t, tw);
  }
}

template <class PL, int W, bool STRIDED, typename T>
__device__ __forceinline__ void inverse_fft(cx<T> *v, int t, int c, T *lre, T *lim,
                                            const cx<T> *tw, bool first) {
  if constexpr (PL::M > 3) {
    stage<PL, 3, +1>(v, t, tw);
    exchange<PL, W, STRIDED, 3, 2>(v, t, c, lre, lim, first);
    first = false;
  }
  if constexpr (PL::M > 2) {
    stage<PL, 2, +1>(v, t, tw);
    exchange<PL, W, STRIDED, 2, 1>(v, t, c, lre, lim, first);
    first = false;
  }
  if constexpr (PL::M > 1) {
    stage<PL, 1, +1>(v, t, tw);
    exchange<PL, W, STRIDED, 1, 0>(v, t, c, lre, lim, first);
  }
  stage<PL, 0, +1>(v, t, tw);
}

__device__ __forceinline__ double site_potential(const PassArgs &a, int j0, int j1, int j2) {
  if (a.V) return a.V[((long long)j0 * a.n[1] + j1) * a.n[2] + j2];
  const double x0 = a.lo[0] + j0 * a.h[0], x1 = a.lo[1] + j1 * a.h[1],
               x2 = a.lo[2] + j2 * a.h[2];
  return a.hv[0] * x0 * x0 + a.hv[1] * x1 * x1 + a.hv[2] * x2 * x2;
}

// Nonlinear/potential phase in FP64 whatever the state precision.
template <typename T>
__device__ __forceinline__ cx<T> apply_phase(int op, cx<T> v, double V, double g,
                                             double tau) {
  const double re = (double)v.x, im = (double)v.y;
  const double th = (V + g * (re * re + im * im)) * tau;
  if (op == PH_REAL) {
    double s, c;
    sincos(th, &s, &c);
    return {(T)(re * c + im * s), (T)(im * c - re * s)};
  }
  const double f = exp(-th);
  return {(T)(re * f), (T)(im * f)};
}

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double *out,
                                                   int slot0) {
  __shared__ double red[16][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = acc[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    acc[k] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0;
    for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
    out[(long long)blockIdx.x * kRedSlots + slot0 + threadIdx.x] = s;
  }
}

template <typename T, class PL, int W, bool STRIDED>
__global__ void __launch_bounds__(PL::TPL * W)
axis_pass_kernel(const PassArgs a) {
  constexpr int N = PL::N, E = PL::E, TPL = PL::TPL;
  using L = Lds<N, W, STRIDED>;
  __shared__ T lre[PL::M > 1 ? L::size : 1], lim[PL::M > 1 ? L::size : 1];

  const int tid = threadIdx.x;
  const int c = STRIDED ? (tid % W) : (tid / TPL);
  const int t = STRIDED ? (tid / W) : (tid % TPL);
  const int n1 = a.n[1], n2 = a.n[2];

  // Line geometry: element p of this thread's line sits at base + p * S; its
  // site coordinates are (j0, j1, j2) with the axis coordinate replaced by p.
  long long base, S;
  int j0 = 0, j1 = 0, j2 = 0;
  bool valid = true;
  if (!STRIDED) {
    const long long line = (long long)blockIdx.x * W + c;
    valid = line < (long long)a.n[0] * n1;
    j0 = (int)(line / n1);
    j1 = (int)(line % n1);
    base = line * N;
    S = 1;
  } else {
    const int ct = n2 / W;
    const int outer = blockIdx.x / ct;
    j2 = (blockIdx.x % ct) * W + c;
    if (a.axis == 1) {
      j0 = outer;
      base = (long long)outer * n1 * n2 + j2;
      S = n2;
    } else {
      j1 = outer;
      base = (long long)outer * n2 + j2;
      S = (long long)n1 * n2;
    }
  }
  const int axis = STRIDED ? a.axis : 2;

  const cx<T> *__restrict__ src = static_cast<const cx<T> *>(a.src);
  cx<T> *__restrict__ dst = static_cast<cx<T> *>(a.dst);
  const cx<T> *__restrict__ tw = static_cast<const cx<T> *>(a.tw);
  const cx<T> *__restrict__ mtab = static_cast<const cx<T> *>(a.mtab);
  constexpr int R0 = PL::rad(0), RL = PL::rad(PL::M - 1);

  double acc[kRedSlots];
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;

  cx<T> v[E];
  if (a.forward) {
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const int p = PL::pos(0, t + TPL * b, d);
        v[b * R0 + d] = valid ? src[base + p * S] : cx<T>{0, 0};
      }
    if (a.scale || a.pre != PH_NONE || (a.red & RED_REAL)) {
      const double sc = a.scale ? *a.scale : 1.0;
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          const int k0 = axis == 0 ? p : j0, k1 = axis == 1 ? p : j1, k2 = axis == 2 ? p : j2;
          cx<T> u = v[b * R0 + d];
          if (a.scale) u = {(T)(sc * (double)u.x), (T)(sc * (double)u.y)};
          const double V = (a.pre != PH_NONE || (a.red & RED_REAL)) && valid
                               ? site_potential(a, k0, k1, k2) : 0.0;
          if (a.red & RED_REAL) {
            const double rho = (double)u.x * u.x + (double)u.y * u.y;
            const double x0 = a.lo[0] + k0 * a.h[0], x1 = a.lo[1] + k1 * a.h[1],
                         x2 = a.lo[2] + k2 * a.h[2];
            acc[kSlotReal + 0] += rho;
            acc[kSlotReal + 1] += V * rho;
            acc[kSlotReal + 2] += rho * rho;
            acc[kSlotReal + 3] += x0 * x0 * rho;
            acc[kSlotReal + 4] += x1 * x1 * rho;
            acc[kSlotReal + 5] += x2 * x2 * rho;
          }
          if (a.pre != PH_NONE) u = apply_phase(a.pre, u, V, a.g, a.tau_pre);
          v[b * R0 + d] = u;
        }
    }
    forward_fft<PL, W, STRIDED>(v, t, c, lre, lim, tw);
  } else {
    // Input is a spectrum in natural order: load it in the digit-reversed
    // layout the inverse stages start from.
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int d = 0; d < RL; ++d) {
        const int p = PL::pos(PL::M - 1, t + TPL * b, d);
        v[b * RL + d] = valid ? src[base + PL::freq(p) * S] : cx<T>{0, 0};
      }
  }

  // Spectrum of this line: element (b, d) holds frequency freq(pos(M-1, q, d)).
  if ((a.red & RED_KIN) || a.mid == MID_TABLE || !a.inverse) {
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int d = 0; d < RL; ++d) {
        const int f = PL::freq(PL::pos(PL::M - 1, t + TPL * b, d));
        cx<T> u = v[b * RL + d];
        if (a.red & RED_KIN) acc[kSlotKin] += a.kw[f] * ((double)u.x * u.x + (double)u.y * u.y);
        if (a.mid == MID_TABLE) u = cmul(u, mtab[f]);
        v[b * RL + d] = u;
        if (!a.inverse && a.store && valid) dst[base + f * S] = u;
      }
  }

  if (a.inverse) {
    inverse_fft<PL, W, STRIDED>(v, t, c, lre, lim, tw, !a.forward);
    if (a.post != PH_NONE || (a.red & RED_NORM_OUT)) {
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          cx<T> u = v[b * R0 + d];
          if (a.post != PH_NONE) {
            const int k0 = axis == 0 ? p : j0, k1 = axis == 1 ? p : j1, k2 = axis == 2 ? p : j2;
            const double V = valid ? site_potential(a, k0, k1, k2) : 0.0;
            u = apply_phase(a.post, u, V, a.g, a.tau_post);
          }
          if (a.red & RED_NORM_OUT) acc[kSlotNormOut] += (double)u.x * u.x + (double)u.y * u.y;
          v[b * R0 + d] = u;
        }
    }
    if (a.store && valid) {
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          dst[base + p * S] = v[b * R0 + d];
        }
    }
  }

  if (a.red) {
    if (!valid) {
#pragma unroll
      for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;
    }
    block_reduce_store(acc, a.partial, 0);
  }
}

template <typename T, int N>
constexpr int contig_lines() {
  return PlanFor<N>::type::TPL >= 256 ? 1 : 256 / PlanFor<N>::type::TPL;
}

template <typename T, int N>
hipError_t launch_n(const PassArgs &a, const PassShape &sh, hipStream_t s) {
  using PL = typename PlanFor<N>::type;
  const dim3 grid((unsigned)sh.blocks), block((unsigned)sh.threads);
  if (!sh.strided) {
    constexpr int W = contig_lines<T, N>();
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, false>), grid, block, 0, s, a);
  } else if (sh.W == 16) {
    if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, 16, true>), grid, block, 0, s, a);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, 8, true>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const PassArgs &a, const PassShape &sh, hipStream_t s) {
  switch (sh.N) {
    case 8: return launch_n<T, 8>(a, sh, s);
    case 16: return launch_n<T, 16>(a, sh, s);
    case 32: return launch_n<T, 32>(a, sh, s);
    case 64: return launch_n<T, 64>(a, sh, s);
    case 128: return launch_n<T, 128>(a, sh, s);
    case 256: return launch_n<T, 256>(a, sh, s);
    case 512: return launch_n<T, 512>(a, sh, s);
    case 1024: return launch_n<T, 1024>(a, sh, s);
    default: return hipErrorInvalidValue;
  }
}

int tpl_of(int N) {
  switch (N) {
    case 8: return PlanFor<8>::type::TPL;
    case 16: return PlanFor<16>::type::TPL;
    case 32: return PlanFor<32>::type::TPL;
    case 64: return PlanFor<64>::type::TPL;
    case 128: return PlanFor<128>::type::TPL;
    case 256: return PlanFor<256>::type::TPL;
    case 512: return PlanFor<512>::type::TPL;
    case 1024: return PlanFor<1024>::type::TPL;
    default: return 0;
  }
}

}  // namespace

PassShape pass_shape(int precision, const int n[3], int axis) {
  PassShape sh{};
  sh.N = n[axis];
  sh.strided = axis != 2;
  const int tpl = tpl_of(sh.N);
  if (tpl == 0) return sh;
  if (!sh.strided) {
    sh.W = tpl >= 256 ? 1 : 256 / tpl;
    sh.threads = tpl * sh.W;
    const long long lines = (long long)n[0] * n[1];
    sh.blocks = (lines + sh.W - 1) / sh.W;
  } else {
    sh.W = (precision == 1 && n[2] >= 16) ? 16 : 8;
    sh.threads = tpl * sh.W;
    const long long outer = axis == 1 ? n[0] : n[1];
    sh.blocks = outer * (n[2] / sh.W);
  }
  return sh;
}

hipError_t launch_axis_pass(int precision, const PassArgs &a, hipStream_t s) {
  const PassShape sh = pass_shape(precision, a.n, a.axis);
  if (sh.threads == 0 || (sh.strided && a.n[2] < sh.W)) return hipErrorInvalidValue;
  return precision == 1 ? launch_t<float>(a, sh, s) : launch_t<double>(a, sh, s);
}

}  // namespace gpe
