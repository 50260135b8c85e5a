// Fused per-axis TSSP pass for gfx950 (templates shared by the FP64 and FP32
// translation units).
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
// (post) and accumulates sums, and stores the lines back (or, in the rotating
// form, into a second array in the layout the next pass reads).  A 3D
// real-time step is three such launches: 32 bytes of HBM traffic per site per
// launch in FP64.
//
// FFT: mixed-radix (2/4/8/16) Cooley-Tukey, decimation in frequency for the
// forward transform (digit-reversed spectrum, never reordered) and the exact
// reverse for the inverse, so the spectrum is used in place.  Each thread
// holds E elements of one line; stages exchange through LDS.  Twiddles come
// from an FP64-accurate table exp(-2 pi i j/N) built on the host per index.
#pragma once

#include "gpe_kernels.h"

#include <cmath>

// Build-time tuning knobs (the defaults are the measured best on MI355X).
#ifndef GPE_CONTIG_THREADS
#define GPE_CONTIG_THREADS 256  // workgroup size for the contiguous axis
#endif
#ifndef GPE_TW_POWERS
#define GPE_TW_POWERS 1  // load w^(2^j), form the other twiddle powers by products
#endif
#ifndef GPE_WAVE_SYNC
#define GPE_WAVE_SYNC 1  // lines held inside one wavefront sync without s_barrier
#endif
#ifndef GPE_FP32_TW_HILO
#define GPE_FP32_TW_HILO 1  // FP32 twiddles applied as hi + lo pairs (else hi, powers by products)
#endif
#ifndef GPE_FP32_K_HILO
#define GPE_FP32_K_HILO 1  // FP32 per-frequency factors applied as hi + lo pairs
#endif
#ifndef GPE_FAST_SINCOS
#define GPE_FAST_SINCOS 1  // Cody-Waite reduction + Taylor series for the phase
#endif

namespace gpe {
namespace pass {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

// Non-temporal (streaming) element load and store: the cache policy of a
// pass that touches each element once; the values are unchanged.
template <typename S>
__device__ __forceinline__ cx<S> load_stream(const cx<S> *p) {
  typedef S v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return cx<S>{w.x, w.y};
}
template <typename S>
__device__ __forceinline__ void store_stream(cx<S> *p, cx<S> v) {
  typedef S v2 __attribute__((ext_vector_type(2)));
  const v2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<v2 *>(p));
}

// Table entries: FP64 tables hold the complex factor.  FP32 tables hold it as
// a hi + lo pair of FP32 complex numbers (x, y = hi; z, w = lo), and the
// product is formed by one chain of FMAs before a single rounding, so every
// twiddle and kinetic factor is unit-modulus to ~1e-14: a plainly rounded
// FP32 factor is off by up to 6e-8 in modulus, the same way every step, and
// the norm would drift linearly.
template <typename T> struct TabOf { using type = cx<T>; };
template <> struct TabOf<float> { using type = float4; };
template <typename T> using tab_t = typename TabOf<T>::type;

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

// u * w (or u * conj(w)) with w = (e.x + e.z) + i (e.y + e.w) given as an FP32
// hi + lo pair; the lo products are added first, then the hi products, each
// component rounded once at the end of its FMA chain.
template <bool CONJ>
__device__ __forceinline__ cx<float> cmul_hl(cx<float> u, const float4 &e) {
  if (CONJ) {
    const float re = fmaf(u.x, e.x, fmaf(u.y, e.y, fmaf(u.x, e.z, u.y * e.w)));
    const float im = fmaf(u.y, e.x, fmaf(-u.x, e.y, fmaf(u.y, e.z, -u.x * e.w)));
    return {re, im};
  }
  const float re = fmaf(u.x, e.x, fmaf(-u.y, e.y, fmaf(u.x, e.z, -u.y * e.w)));
  const float im = fmaf(u.x, e.y, fmaf(u.y, e.x, fmaf(u.x, e.w, u.y * e.z)));
  return {re, im};
}

// v * exp(SIGN * 2 pi i k / 16); k is a constant once loops are unrolled.  In
// FP32 the irrational constants are applied as hi + lo pairs, so the rotation
// has unit modulus to well below FP32 rounding (a plain FP32 sqrt(1/2) has
// 2 r^2 = 1 - 3.4e-8, a bias that would accumulate step after step).
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot16(cx<T> v, int k) {
  if constexpr (sizeof(T) == 8) {
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
  } else {
    const float rh = 0x1.6a09e6p-1f, rl = 1.2101617485882343e-08f;
    const float ch = 0x1.d906bcp-1f, cl = 2.830748968563057e-08f;
    const float sh = 0x1.87de2ap-2f, sl = 6.2233507236442165e-09f;
    auto cm2 = [](cx<float> a, float xh, float xl, float yh, float yl) {
      // a * ((xh + xl) + i (yh + yl))
      const float re = fmaf(a.x, xh, fmaf(a.x, xl, -fmaf(a.y, yh, a.y * yl)));
      const float im = fmaf(a.x, yh, fmaf(a.x, yl, fmaf(a.y, xh, a.y * xl)));
      return cx<float>{re, im};
    };
    switch (k) {
      case 0: return v;
      case 1: return cm2(v, ch, cl, SIGN * sh, SIGN * sl);
      case 2: {
        const float a = v.x - SIGN * v.y, b = v.y + SIGN * v.x;
        return {fmaf(rh, a, rl * a), fmaf(rh, b, rl * b)};
      }
      case 3: return cm2(v, sh, sl, SIGN * ch, SIGN * cl);
      case 4: return {-SIGN * v.y, SIGN * v.x};
      case 5: return cm2(v, -sh, -sl, SIGN * ch, SIGN * cl);
      case 6: {
        const float a = -(v.x + SIGN * v.y), b = SIGN * v.x - v.y;
        return {fmaf(rh, a, rl * a), fmaf(rh, b, rl * b)};
      }
      default: return cm2(v, -ch, -cl, SIGN * sh, SIGN * sl);
    }
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
// Alternative plans, chosen per axis at run time (plan 1): 1024 points as four
// stages of 8, 8, 8 and 2 with 8 points per thread -- half the registers of
// the default, at the cost of one more LDS exchange each way.
template <int N> struct PlanAlt { using type = typename PlanFor<N>::type; };
template <> struct PlanAlt<1024> { using type = Plan<1024, 8, 8, 8, 8, 2>; };

// LDS layout of a tile of W lines of N points (separate re and im planes).
// Strided tiles are rows of W columns with one padding row after every eight
// rows; contiguous lines get one padding slot per eight points.  For the
// radix-8 exchange patterns these spread a wavefront's accesses over all banks
// (no conflicts for strided tiles with 32 or 64 four-byte banks, FP64 or FP32).
template <int N, int W, bool STRIDED>
struct Lds {
  static constexpr int line = N + N / 8;
  static constexpr int size = STRIDED ? W * line : W * line;
  __device__ static __forceinline__ int idx(int p, int c) {
    return STRIDED ? W * (p + (p >> 3)) + c : c * line + p + (p >> 3);
  }
};

__host__ __device__ constexpr int high_bit(int d) {
  int h = 1;
  while (h * 2 <= d) h *= 2;
  return h;
}

// The leading (hi) part of a table entry.
template <typename T>
__device__ __forceinline__ cx<T> tab_hi(const tab_t<T> &e) {
  if constexpr (sizeof(T) == 4) return cx<T>{e.x, e.y};
  else return e;
}

// u[d] *= w^d (or conj(w^d)) for d = 1 .. R-1, w = exp(-2 pi i tb / N).  FP64:
// the powers w^(2^j) come from the FP64-accurate table and the others are
// products of at most log2(R) - 1 of them (a few ulp, not a long recurrence).
// FP32: every power is read from the hi + lo table.
template <int R, bool CONJ, typename T>
__device__ __forceinline__ void twiddle(cx<T> *u, const tab_t<T> *__restrict__ tw, int tb) {
  if constexpr (sizeof(T) == 4 && GPE_FP32_TW_HILO) {
#pragma unroll
    for (int d = 1; d < R; ++d) {
      u[d] = cmul_hl<CONJ>(u[d], tw[tb * d]);
    }
  } else {
#if GPE_TW_POWERS
    cx<T> w[R];
#pragma unroll
    for (int d = 1; d < R; d *= 2) w[d] = tab_hi<T>(tw[tb * d]);
#pragma unroll
    for (int d = 3; d < R; ++d)
      if (d & (d - 1)) w[d] = cmul(w[high_bit(d)], w[d - high_bit(d)]);
#pragma unroll
    for (int d = 1; d < R; ++d) u[d] = CONJ ? cmulc(u[d], w[d]) : cmul(u[d], w[d]);
#else
#pragma unroll
    for (int d = 1; d < R; ++d)
      u[d] = CONJ ? cmulc(u[d], tab_hi<T>(tw[tb * d])) : cmul(u[d], tab_hi<T>(tw[tb * d]));
#endif
  }
}

// Multiply by a per-frequency table entry.
template <typename T>
__device__ __forceinline__ cx<T> table_mul(cx<T> u, const tab_t<T> &e) {
  if constexpr (sizeof(T) == 4 && GPE_FP32_K_HILO) {
    return cmul_hl<false>(u, e);
  } else if constexpr (sizeof(T) == 4) {
    return cmul(u, cx<T>{e.x, e.y});
  } else {
    return cmul(u, e);
  }
}

// One forward (SIGN = -1: DFT then twiddle) or inverse (SIGN = +1: conjugate
// twiddle then DFT) stage S on the thread's E registers.
template <class PL, int S, int SIGN, typename T>
__device__ __forceinline__ void stage(cx<T> *v, int t, const tab_t<T> *__restrict__ tw) {
  constexpr int R = PL::rad(S), B = PL::E / R, ST = PL::stride(S), P = PL::P(S);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int q = t + PL::TPL * b;
    cx<T> *u = v + b * R;
    const int tb = P * (q % ST);
    if (SIGN < 0) {
      dft<R, -1>(u);
      if (ST > 1) twiddle<R, false>(u, tw, tb);
    } else {
      if (ST > 1) twiddle<R, true>(u, tw, tb);
      dft<R, +1>(u);
    }
  }
}

// Barrier between LDS writes and reads of an exchange.  When every line of the
// tile lives inside one wavefront (contiguous axis, N/E <= 64 threads per line)
// the wave's own in-order LDS queue suffices and only compiler ordering is
// needed; otherwise the whole workgroup waits.
template <class PL, int W, bool STRIDED>
__device__ __forceinline__ void lds_sync() {
  constexpr bool in_wave = GPE_WAVE_SYNC && (STRIDED ? PL::TPL * W <= 64 : PL::TPL <= 64);
  if constexpr (in_wave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS row of position p (one padding slot after every eight positions), and
// its split over the two parts of a stage position: pos(s, q, d) =
// qpart(q) + d * stride(s), with q from the thread and d a compile-time digit.
// row(qpart + d st) = row(qpart) + row(d st) whenever the two parts never
// carry into bit 3 together, which holds for every plan here (checked at
// compile time): a thread forms one base address per stage and reaches each
// element at a compile-time offset from it (few address registers, offsets
// folded into the LDS instructions).
__host__ __device__ constexpr int lds_row(int p) { return p + (p >> 3); }
template <class PL, int S>
__host__ __device__ constexpr int qpart(int q) {
  return (q % PL::stride(S)) + (q / PL::stride(S)) * PL::stride(S) * PL::rad(S);
}
template <class PL, int S>
constexpr bool rows_split() {
  for (int q = 0; q < PL::N / PL::rad(S); ++q)
    for (int d = 0; d < PL::rad(S); ++d)
      if (lds_row(qpart<PL, S>(q) + d * PL::stride(S)) !=
          lds_row(qpart<PL, S>(q)) + lds_row(d * PL::stride(S)))
        return false;
  return true;
}

// LDS index of the element at position qpart + d st of column / line c:
// base (from the thread) plus a compile-time offset (from the digit).
template <int N, int W, bool STRIDED>
__device__ __forceinline__ int lds_base(int qp, int c) {
  return STRIDED ? W * lds_row(qp) + c : c * Lds<N, W, STRIDED>::line + lds_row(qp);
}
template <int W, bool STRIDED>
__host__ __device__ constexpr int lds_off(int dp) {
  return STRIDED ? W * lds_row(dp) : lds_row(dp);
}

// Move the E registers from the stage-A layout to the stage-B layout.
template <class PL, int W, bool STRIDED, int A, int B, typename T>
__device__ __forceinline__ void exchange(cx<T> *v, int t, int c, T *lre, T *lim,
                                         bool first) {
  constexpr int RA = PL::rad(A), RB = PL::rad(B), SA = PL::stride(A), SB = PL::stride(B);
  static_assert(rows_split<PL, A>() && rows_split<PL, B>(),
                "LDS rows must split over the stage positions");
  if (!first) lds_sync<PL, W, STRIDED>();
#pragma unroll
  for (int b = 0; b < PL::E / RA; ++b) {
    const int i0 = lds_base<PL::N, W, STRIDED>(qpart<PL, A>(t + PL::TPL * b), c);
    T *__restrict__ r = lre + i0;
    T *__restrict__ m = lim + i0;
#pragma unroll
    for (int d = 0; d < RA; ++d) {
      r[lds_off<W, STRIDED>(d * SA)] = v[b * RA + d].x;
      m[lds_off<W, STRIDED>(d * SA)] = v[b * RA + d].y;
    }
  }
  lds_sync<PL, W, STRIDED>();
#pragma unroll
  for (int b = 0; b < PL::E / RB; ++b) {
    const int i0 = lds_base<PL::N, W, STRIDED>(qpart<PL, B>(t + PL::TPL * b), c);
    const T *__restrict__ r = lre + i0;
    const T *__restrict__ m = lim + i0;
#pragma unroll
    for (int d = 0; d < RB; ++d) {
      v[b * RB + d].x = r[lds_off<W, STRIDED>(d * SB)];
      v[b * RB + d].y = m[lds_off<W, STRIDED>(d * SB)];
    }
  }
}

template <class PL, int W, bool STRIDED, typename T>
__device__ __forceinline__ void forward_fft(cx<T> *v, int t, int c, T *lre, T *lim,
                                            const tab_t<T> *tw, bool first = true) {
  stage<PL, 0, -1>(v, t, tw);
  if constexpr (PL::M > 1) {
    exchange<PL, W, STRIDED, 0, 1>(v, t, c, lre, lim, first);
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
                                            const tab_t<T> *tw, bool first) {
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

// Analytic harmonic potential sum_j hv[j] x_j^2 at site (j0, j1, j2).
__device__ __forceinline__ double harmonic_potential(const double (&lo)[3], const double (&h)[3],
                                                     const double (&hv)[3], int j0, int j1,
                                                     int j2) {
  const double x0 = lo[0] + j0 * h[0], x1 = lo[1] + j1 * h[1], x2 = lo[2] + j2 * h[2];
  return hv[0] * x0 * x0 + hv[1] * x1 * x1 + hv[2] * x2 * x2;
}

__device__ __forceinline__ double site_potential(const PassArgs &a, int vkind, const double (&hv)[3],
                                                 int j0, int j1, int j2,
                                                 const double *__restrict__ vt) {
  if (vkind == V_NONE) return 0.0;
  if (vkind == V_ARRAY) return a.V[((long long)j0 * a.n[1] + j1) * a.n[2] + j2];
  if (vkind == V_TABLES) return vt[j0] + vt[a.n[0] + j1] + vt[a.n[0] + a.n[1] + j2];
  return harmonic_potential(a.lo, a.h, hv, j0, j1, j2);
}

// sin and cos of x in FP64: Cody-Waite reduction x = n pi/2 + r with pi/2 split
// in three parts (the first two with 33 significant bits, so n * part is exact
// for |n| < 2^20), then the Taylor series of sin and cos on |r| <= pi/4 up to
// degree 17 and 18 (truncation below 1e-19).  Arguments beyond 1e6 go to the
// library routine.  Small arguments (|x| < 2^-6: the phase of a step in a
// weakly interacting or untrapped region) need no reduction and only the
// series up to degree 7 and 6 (truncation below 1e-19 relative); the choice is
// per site, so a result never depends on its neighbours.
__device__ __forceinline__ void sincos_phase(double x, double *s, double *c) {
#if GPE_FAST_SINCOS
  if (fabs(x) < 0x1p-6) {
    const double r2 = x * x;
    double ps = fma(r2, -0.0001984126984126984, 0.008333333333333333);
    ps = fma(ps, r2, -0.16666666666666666);
    *s = fma(ps * r2, x, x);
    double pc = fma(r2, -0.001388888888888889, 0.041666666666666664);
    pc = fma(pc, r2, -0.5);
    *c = fma(pc, r2, 1.0);
    return;
  }
  if (!(fabs(x) < 1.0e6)) {
    sincos(x, s, c);
    return;
  }
  const double n = rint(x * 0.63661977236758134308);
  double r = fma(-n, 0x1.921fb54400000p+0, x);
  r = fma(-n, 0x1.0b4611a600000p-34, r);
  r = fma(-n, 0x1.3198a2e037073p-69, r);
  const double r2 = r * r;
  double ps = 2.8114572543455206e-15;
  ps = fma(ps, r2, -7.647163731819816e-13);
  ps = fma(ps, r2, 1.6059043836821613e-10);
  ps = fma(ps, r2, -2.505210838544172e-08);
  ps = fma(ps, r2, 2.7557319223985893e-06);
  ps = fma(ps, r2, -0.0001984126984126984);
  ps = fma(ps, r2, 0.008333333333333333);
  ps = fma(ps, r2, -0.16666666666666666);
  ps = fma(ps * r2, r, r);
  double pc = -1.5619206968586225e-16;
  pc = fma(pc, r2, 4.779477332387385e-14);
  pc = fma(pc, r2, -1.1470745597729725e-11);
  pc = fma(pc, r2, 2.08767569878681e-09);
  pc = fma(pc, r2, -2.755731922398589e-07);
  pc = fma(pc, r2, 2.48015873015873e-05);
  pc = fma(pc, r2, -0.001388888888888889);
  pc = fma(pc, r2, 0.041666666666666664);
  pc = fma(pc, r2, -0.5);
  pc = fma(pc, r2, 1.0);
  const int q = ((int)n) & 3;
  const double ss = (q & 1) ? pc : ps, cc = (q & 1) ? ps : pc;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
#else
  sincos(x, s, c);
#endif
}

// Nonlinear/potential phase in FP64 whatever the state precision.
template <typename T>
__device__ __forceinline__ cx<T> apply_phase(int op, cx<T> v, double V, double g,
                                             double tau) {
  const double re = (double)v.x, im = (double)v.y;
  const double th = (V + g * (re * re + im * im)) * tau;
  if (op == PH_REAL) {
    double s, c;
    sincos_phase(th, &s, &c);
    return {(T)(re * c + im * s), (T)(im * c - re * s)};
  }
  if (op == PH_IMAG_EXACT) {
    // rho = |psi|^2 obeys the Bernoulli equation d rho/d tau = -2 (V + g rho) rho
    const double E = V != 0.0 ? -expm1(-2.0 * V * tau) / V : 2.0 * tau;
    const double f = exp(-V * tau) / sqrt(1.0 + g * (re * re + im * im) * E);
    return {(T)(re * f), (T)(im * f)};
  }
  const double f = exp(-th);
  return {(T)(re * f), (T)(im * f)};
}

// Fixed-order block sums of NV values per thread; NT threads per block.
// Full wavefronts add across lanes with shuffles, then wave totals in order;
// a block smaller than a wavefront adds its threads' values in order (a
// shuffle would read lanes that do not exist).
template <int NV, int NT>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double *out,
                                                   int slot0) {
  if constexpr (NT >= 64) {
    __shared__ double red[16][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int nw = NT / 64;
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
  } else {
    __shared__ double red[NT][NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < NV) {
      double s = 0;
      for (int t = 0; t < NT; ++t) s += red[t][threadIdx.x];
      out[(long long)blockIdx.x * kRedSlots + slot0 + threadIdx.x] = s;
    }
  }
}

// Compile-time operation sets of the hot passes; MODE_GENERIC reads them from
// the arguments at run time.
enum PassMode : int {
  MODE_GENERIC = 0,
  MODE_PLAIN = 1,          // forward, table, inverse
  MODE_PRE_REAL = 2,       // real-time phase, forward, table, inverse
  MODE_PRE_IMAG = 3,       // scale, imaginary-time phase, forward, table, inverse
  MODE_POST_IMAG_RED = 4,  // forward, table, inverse, imaginary-time phase, norm sum
  MODE_SLOTS_REAL = 5,     // batched real-time class: operations from each block's slot
  MODE_SLOTS_IMAG = 6,     // batched imaginary-time class
  MODE_FWD = 7,            // forward only, spectrum stored in natural order
  MODE_DERIV = 8,          // forward, table, inverse, combine with the re-read
                           // state (PH_DERIV), forward again, store
  MODE_OBS = 9,            // forward only, kinetic sum, nothing stored
  MODE_OBS_REAL = 10,      // the same plus the real-space sums of the input
  MODE_PRE_IMAG_EXACT = 11,       // MODE_PRE_IMAG with the exact substep
  MODE_POST_IMAG_RED_EXACT = 12,  // MODE_POST_IMAG_RED with the exact substep
  MODE_POST_REAL = 13,     // forward, table, inverse, closing real-time phase
  MODE_FWD_REAL = 14,      // MODE_FWD plus the real-space sums of the input
};

// The step modes (MODE_PLAIN, MODE_PRE_REAL) also come with streaming
// (non-temporal) loads, stores or both: mode | STREAM_LOAD and/or
// | STREAM_STORE.
constexpr int STREAM_LOAD = 16, STREAM_STORE = 32;
// The batched slot modes also come with the role of the pass in the step
// fixed at compile time (first: the opening phase, and in imaginary time the
// pending scale; last: the closing phase and the norm sums; neither: plain):
// mode | SLOT_ROLE, plus SLOT_FIRST and/or SLOT_LAST.
constexpr int SLOT_FIRST = 64, SLOT_LAST = 128, SLOT_ROLE = 256;
__host__ __device__ constexpr int base_mode(int m) { return m & 15; }

// Storage type of the state in HBM, converted on load and store: the
// arithmetic type T, or FP32 storage with FP64 arithmetic (SX = float,
// T = double).
template <typename T, typename SX>
__device__ __forceinline__ cx<T> cvt(const cx<SX> &u) {
  return {(T)u.x, (T)u.y};
}

template <typename T, class PL, int W, bool STRIDED, int MODE_ARG, typename SX = T>
__global__ void __launch_bounds__(PL::TPL * W)
axis_pass_kernel(const PassArgs a) {
  constexpr int MODE = base_mode(MODE_ARG);
  constexpr bool SLOAD = (MODE_ARG & STREAM_LOAD) != 0, SSTORE = (MODE_ARG & STREAM_STORE) != 0;
  constexpr int N = PL::N, E = PL::E, TPL = PL::TPL;
  using L = Lds<N, W, STRIDED>;
  __shared__ T lre[PL::M > 1 ? L::size : 1], lim[PL::M > 1 ? L::size : 1];

  constexpr bool G = MODE == MODE_GENERIC;
  constexpr bool SLI = MODE == MODE_SLOTS_IMAG;
  constexpr bool SL = MODE == MODE_SLOTS_REAL || SLI;
  constexpr bool FWD = MODE == MODE_FWD || MODE == MODE_FWD_REAL, DER = MODE == MODE_DERIV;
  constexpr bool OBS = MODE == MODE_OBS || MODE == MODE_OBS_REAL;
  const int forward = G ? a.forward : 1;
  const int inverse = G ? a.inverse : (FWD || OBS ? 0 : 1);
  const int store = G ? a.store : (OBS ? 0 : 1);
  constexpr bool PRE_IM = MODE == MODE_PRE_IMAG || MODE == MODE_PRE_IMAG_EXACT;
  constexpr bool POST_IM = MODE == MODE_POST_IMAG_RED || MODE == MODE_POST_IMAG_RED_EXACT;
  constexpr bool EXACT = MODE == MODE_PRE_IMAG_EXACT || MODE == MODE_POST_IMAG_RED_EXACT;
  constexpr int IM_OP = EXACT ? PH_IMAG_EXACT : PH_IMAG;
  int pre = G ? a.pre : (MODE == MODE_PRE_REAL ? PH_REAL : PRE_IM ? IM_OP : PH_NONE);
  int post = G ? a.post
               : (POST_IM ? IM_OP : DER ? PH_DERIV : MODE == MODE_POST_REAL ? PH_REAL : PH_NONE);
  const int mid = G ? a.mid : (FWD || OBS ? MID_NONE : MID_TABLE);
  const bool refwd = G ? a.refwd != 0 : DER;
  int red = G ? a.red
              : (POST_IM                    ? RED_NORM_OUT
                 : MODE == MODE_OBS         ? RED_KIN
                 : MODE == MODE_OBS_REAL    ? (RED_KIN | RED_REAL)
                 : MODE == MODE_FWD_REAL    ? RED_REAL
                                            : RED_NONE);
  bool has_scale = G || OBS ? a.scale != nullptr : PRE_IM;
  // Per-block parameters: from the arguments, or (batched) from this block's slot.
  const void *psrc = a.src;
  void *pdst = a.dst;
  const void *ptab = a.mtab;
  const double *pscale = a.scale;
  // (copied by value: a pointer that may point into the kernel arguments
  // would force them into private memory)
  double hv[3] = {a.hv[0], a.hv[1], a.hv[2]};
  int vkind = a.vkind;
  double g = a.g, tau_pre = a.tau_pre, tau_post = a.tau_post;
  double *partial = a.partial;
  if constexpr (SL) {
    const int si = a.slot_map ? a.slot_map[blockIdx.y] : (int)blockIdx.y;
    const Slot &sl = a.slots[si];
    const int step = sl.steps_done + a.slot_step;
    if (sl.mode == SLOT_FREE || step >= sl.steps_total) return;
    constexpr bool im = SLI;
    constexpr bool ROLE = (MODE_ARG & SLOT_ROLE) != 0;
    const bool first = ROLE ? (MODE_ARG & SLOT_FIRST) != 0 : (a.slot_pass & SLOT_PASS_FIRST) != 0;
    const bool last = ROLE ? (MODE_ARG & SLOT_LAST) != 0 : (a.slot_pass & SLOT_PASS_LAST) != 0;
    psrc = sl.psi;
    pdst = sl.psi;
    ptab = im ? a.mtab_imag : a.mtab;
    g = sl.g;
    hv[0] = sl.hv[0];
    hv[1] = sl.hv[1];
    hv[2] = sl.hv[2];
    vkind = (hv[0] != 0 || hv[1] != 0 || hv[2] != 0) ? V_HARMONIC : V_NONE;
    pre = first ? (im ? PH_IMAG : PH_REAL) : PH_NONE;
    tau_pre = (im || step == 0) ? 0.5 * a.dt : a.dt;
    has_scale = first && im;
    pscale = &sl.scale;
    post = last ? ((im || step == sl.steps_total - 1) ? (im ? PH_IMAG : PH_REAL) : PH_NONE)
                : PH_NONE;
    tau_post = 0.5 * a.dt;
    red = (last && im) ? RED_NORM_OUT : RED_NONE;
    partial = a.partial + (long long)si * gridDim.x * kRedSlots;
  }

  const int tid = threadIdx.x;
  const int c = STRIDED ? (tid % W) : (tid / TPL);
  const int t = STRIDED ? (tid / W) : (tid % TPL);
  const int n1 = a.n[1], n2 = a.n[2];

  // Line geometry: element p of this thread's line is read at bin + p * Sin
  // and written at bout + p * Sout (the same place unless the pass rotates);
  // its site coordinates are (j0, j1, j2) with the axis coordinate replaced
  // by p.
  long long bin, Sin, bout, Sout;
  int j0 = 0, j1 = 0, j2 = 0;
  bool valid = true;
  if (!STRIDED) {
    const long long line = (long long)blockIdx.x * W + c;
    valid = (!G && !SL) || line < (long long)a.n[0] * n1;
    j0 = (int)(line / n1);
    j1 = (int)(line % n1);
    bin = bout = line * N;
    Sin = Sout = 1;
  } else {
    // Workgroups are dealt to the 8 XCDs round-robin; with xcd_remap each XCD
    // takes a contiguous run of tiles instead (same tiles, other order).
    int tile = blockIdx.x;
    if (a.xcd_remap && (gridDim.x & 7) == 0)
      tile = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (!SL && a.trans) {
      // Rotating pass: the W lines of the tile sit at consecutive positions
      // jb of axis b = axis + 1 (mod 3) and at position jc of the third axis;
      // each line is contiguous in the input [b][c][a], and the output
      // [c][a][b] puts the tile's W sites of each position p side by side.
      const int ax = a.axis, bx = ax == 2 ? 0 : ax + 1, cxs = 3 - ax - bx;
      const int nb = a.n[bx], nc = a.n[cxs];
      const int ct = nb / W;
      const int jc = tile / ct, jb = (tile % ct) * W + c;
      bin = ((long long)jb * nc + jc) * N;
      Sin = 1;
      bout = (long long)jc * N * nb + jb;
      Sout = nb;
      j0 = bx == 0 ? jb : cxs == 0 ? jc : 0;
      j1 = bx == 1 ? jb : cxs == 1 ? jc : 0;
      j2 = bx == 2 ? jb : cxs == 2 ? jc : 0;
    } else {
      const int ct = n2 / W;
      const int outer = tile / ct;
      j2 = (tile % ct) * W + c;
      if (a.axis == 1) {
        j0 = outer;
        bin = (long long)outer * n1 * n2 + j2;
        Sin = n2;
      } else {
        j1 = outer;
        bin = (long long)outer * n2 + j2;
        Sin = (long long)n1 * n2;
      }
      bout = bin;
      Sout = Sin;
    }
  }
  const int axis = STRIDED ? a.axis : 2;

  const cx<SX> *__restrict__ src = static_cast<const cx<SX> *>(psrc);
  cx<SX> *__restrict__ dst = static_cast<cx<SX> *>(pdst);
  const tab_t<T> *__restrict__ tw = static_cast<const tab_t<T> *>(a.tw);
  const tab_t<T> *__restrict__ mtab = static_cast<const tab_t<T> *>(ptab);
  constexpr int R0 = PL::rad(0), RL = PL::rad(PL::M - 1);

  double acc[kRedSlots];
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;

  cx<T> v[E];
  // The derivative pass combines its result with the state at the same
  // positions it loaded: it keeps the loaded values (in the storage type)
  // instead of reading them again.
  cx<SX> kept[DER ? E : 1];
  if (forward) {
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const int p = PL::pos(0, t + TPL * b, d);
        if constexpr (SLOAD) {
          v[b * R0 + d] = cvt<T>(load_stream(&src[bin + p * Sin]));
        } else if constexpr (DER) {
          kept[b * R0 + d] = valid ? src[bin + p * Sin] : cx<SX>{0, 0};
          v[b * R0 + d] = cvt<T>(kept[b * R0 + d]);
        } else {
          v[b * R0 + d] = valid ? cvt<T>(src[bin + p * Sin]) : cx<T>{0, 0};
        }
      }
    if (has_scale || pre != PH_NONE || (red & RED_REAL)) {
      const double sc = has_scale ? *pscale : 1.0;
      const double mus =
          (G || EXACT) && pre == PH_IMAG_EXACT && a.mu_shift ? *a.mu_shift : 0.0;
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          const int k0 = axis == 0 ? p : j0, k1 = axis == 1 ? p : j1, k2 = axis == 2 ? p : j2;
          cx<T> u = v[b * R0 + d];
          if (has_scale) u = {(T)(sc * (double)u.x), (T)(sc * (double)u.y)};
          const double V = (pre != PH_NONE || (red & RED_REAL)) && valid
                               ? site_potential(a, vkind, hv, k0, k1, k2, a.vtab) : 0.0;
          if (red & RED_REAL) {
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
          if (pre != PH_NONE) u = apply_phase(pre, u, V - mus, g, tau_pre);
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
        v[b * RL + d] = valid ? cvt<T>(src[bin + PL::freq(p) * Sin]) : cx<T>{0, 0};
      }
  }

  // Spectrum of this line: element (b, d) holds frequency freq(pos(M-1, q, d)).
  if ((red & RED_KIN) || mid == MID_TABLE || !inverse) {
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int d = 0; d < RL; ++d) {
        const int f = PL::freq(PL::pos(PL::M - 1, t + TPL * b, d));
        cx<T> u = v[b * RL + d];
        if (red & RED_KIN) acc[kSlotKin] += a.kw[f] * ((double)u.x * u.x + (double)u.y * u.y);
        if (mid == MID_TABLE) u = table_mul(u, mtab[f]);
        v[b * RL + d] = u;
        if (!inverse && store && valid) dst[bout + f * Sout] = cvt<SX>(u);
      }
  }

  if (inverse) {
    inverse_fft<PL, W, STRIDED>(v, t, c, lre, lim, tw, !forward);
    if (post != PH_NONE || (red & RED_NORM_OUT)) {
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          cx<T> u = v[b * R0 + d];
          if (post == PH_DERIV) {
            // combine the derivative with the state at this site (kept from
            // the load, or read again in the generic mode)
            cx<T> q;
            if constexpr (DER) q = cvt<T>(kept[b * R0 + d]);
            else q = valid ? cvt<T>(src[bin + p * Sin]) : cx<T>{0, 0};
            const double qr = q.x, qi = q.y, dr = u.x, di = u.y;
            const double mag = sqrt(qr * qr + qi * qi);
            const double zr = qr * dr + qi * di, zi = qr * di - qi * dr;  // conj(q) d
            const double inv = mag > 0 ? 1.0 / mag : 0.0;  // one division per site
            u = cx<T>{(T)(zi * inv), (T)(zr * inv)};
          } else if (post != PH_NONE) {
            const int k0 = axis == 0 ? p : j0, k1 = axis == 1 ? p : j1, k2 = axis == 2 ? p : j2;
            const double V =
                valid ? site_potential(a, vkind, hv, k0, k1, k2,
                                       a.vtab_post ? a.vtab_post : a.vtab)
                      : 0.0;
            const double mus =
                (G || EXACT) && post == PH_IMAG_EXACT && a.mu_shift ? *a.mu_shift : 0.0;
            u = apply_phase(post, u, V - mus, g, tau_post);
          }
          if (red & RED_NORM_OUT) acc[kSlotNormOut] += (double)u.x * u.x + (double)u.y * u.y;
          v[b * R0 + d] = u;
        }
    }
    if (refwd) {
      // transform the post-op result forward along this axis (the LDS was
      // last read by the inverse stages, so the first exchange waits)
      forward_fft<PL, W, STRIDED>(v, t, c, lre, lim, tw, false);
      if (store && valid) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
          for (int d = 0; d < RL; ++d) {
            const int f = PL::freq(PL::pos(PL::M - 1, t + TPL * b, d));
            dst[bout + f * Sout] = cvt<SX>(v[b * RL + d]);
          }
      }
    } else if (store && valid) {
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int d = 0; d < R0; ++d) {
          const int p = PL::pos(0, t + TPL * b, d);
          if constexpr (SSTORE) store_stream(&dst[bout + p * Sout], cvt<SX>(v[b * R0 + d]));
          else dst[bout + p * Sout] = cvt<SX>(v[b * R0 + d]);
        }
    }
  }

  if (red) {
    if (!valid) {
#pragma unroll
      for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;
    }
    block_reduce_store<kRedSlots, TPL * W>(acc, partial, 0);
  }
}

// The plain in-place step pass (forward, per-frequency table, inverse) of a
// strided axis over tiles of 2 W columns held as two W-column halves: both
// halves are loaded at once and go through the LDS tile one after the other,
// so the second half's loads and the first half's stores overlap the
// arithmetic of the other half, and each row of the tile is 2 W sites wide.
// For FP32 storage (the held half costs 8 x 2 FP32 registers per thread).
// The arithmetic of a line is that of axis_pass_kernel in MODE_PLAIN.
template <typename T, class PL, int W, int SM, typename SX>
__global__ void __launch_bounds__(PL::TPL * W) axis_pass_halves_kernel(const PassArgs a) {
  constexpr int N = PL::N, E = PL::E, TPL = PL::TPL;
  constexpr int R0 = PL::rad(0), RL = PL::rad(PL::M - 1);
  constexpr bool SLOAD = (SM & STREAM_LOAD) != 0, SSTORE = (SM & STREAM_STORE) != 0;
  using L = Lds<N, W, true>;
  __shared__ T lre[PL::M > 1 ? L::size : 1], lim[PL::M > 1 ? L::size : 1];
  const int tid = threadIdx.x, c = tid % W, t = tid / W;
  const int n1 = a.n[1], n2 = a.n[2];
  int tile = blockIdx.x;
  if (a.xcd_remap && (gridDim.x & 7) == 0)
    tile = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int ct = n2 / (2 * W);
  const int outer = tile / ct;
  const int j2 = (tile % ct) * 2 * W + c;
  long long base, S;
  if (a.axis == 1) {
    base = (long long)outer * n1 * n2 + j2;
    S = n2;
  } else {
    base = (long long)outer * n2 + j2;
    S = (long long)n1 * n2;
  }
  const cx<SX> *__restrict__ src = static_cast<const cx<SX> *>(a.src);
  cx<SX> *__restrict__ dst = static_cast<cx<SX> *>(a.dst);
  const tab_t<T> *__restrict__ tw = static_cast<const tab_t<T> *>(a.tw);
  const tab_t<T> *__restrict__ mtab = static_cast<const tab_t<T> *>(a.mtab);
  cx<SX> raw[2][E];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const long long i = base + h * W + PL::pos(0, t + TPL * b, d) * S;
        if constexpr (SLOAD) raw[h][b * R0 + d] = load_stream(&src[i]);
        else raw[h][b * R0 + d] = src[i];
      }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    cx<T> v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cvt<T>(raw[h][k]);
    // (the second half's first exchange waits for the first half's last reads)
    forward_fft<PL, W, true>(v, t, c, lre, lim, tw, h == 0);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int d = 0; d < RL; ++d) {
        const int f = PL::freq(PL::pos(PL::M - 1, t + TPL * b, d));
        v[b * RL + d] = table_mul(v[b * RL + d], mtab[f]);
      }
    inverse_fft<PL, W, true>(v, t, c, lre, lim, tw, false);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int d = 0; d < R0; ++d) {
        const long long i = base + h * W + PL::pos(0, t + TPL * b, d) * S;
        if constexpr (SSTORE) store_stream(&dst[i], cvt<SX>(v[b * R0 + d]));
        else dst[i] = cvt<SX>(v[b * R0 + d]);
      }
  }
}

template <typename T, class PL, typename SX>
void launch_halves(const PassArgs &a, int mode, dim3 grid, dim3 block, hipStream_t s) {
  switch (mode) {
    case MODE_PLAIN:
      hipLaunchKernelGGL((axis_pass_halves_kernel<T, PL, 16, 0, SX>), grid, block, 0, s, a);
      break;
    case MODE_PLAIN | STREAM_LOAD:
      hipLaunchKernelGGL((axis_pass_halves_kernel<T, PL, 16, STREAM_LOAD, SX>), grid, block, 0, s,
                         a);
      break;
    case MODE_PLAIN | STREAM_STORE:
      hipLaunchKernelGGL((axis_pass_halves_kernel<T, PL, 16, STREAM_STORE, SX>), grid, block, 0,
                         s, a);
      break;
    default:
      hipLaunchKernelGGL((axis_pass_halves_kernel<T, PL, 16, STREAM_LOAD | STREAM_STORE, SX>),
                         grid, block, 0, s, a);
  }
}

template <class PL>
constexpr int contig_lines() {
  return PL::TPL >= GPE_CONTIG_THREADS ? 1 : GPE_CONTIG_THREADS / PL::TPL;
}

// Columns per workgroup for a strided axis: the requested width, halved until
// the N x W tile (two planes plus padding) fits the 160 KiB of LDS and the
// workgroup (tpl threads per line) has at most 1024 threads.
__host__ __device__ constexpr int fit_w(int N, int esize, int W, int tpl) {
  while (W > 8 && (W * (N + N / 8) * esize > 160 * 1024 || tpl * W > 1024)) W /= 2;
  return W;
}

template <typename T, class PL, int W, bool STRIDED, typename SX>
void launch_mode(const PassArgs &a, int mode, dim3 grid, dim3 block, hipStream_t s) {
  switch (mode) {
    case MODE_PLAIN:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_PLAIN, SX>), grid, block, 0, s,
                         a);
      break;
    case MODE_PRE_REAL:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_PRE_REAL, SX>), grid, block, 0,
                         s, a);
      break;
    case MODE_PRE_IMAG:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_PRE_IMAG, SX>), grid, block, 0,
                         s, a);
      break;
    case MODE_POST_IMAG_RED:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_POST_IMAG_RED, SX>), grid,
                         block, 0, s, a);
      break;
#define GPE_SLOT_CASES(M)                                                                     \
  case M | SLOT_ROLE:                                                                           \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | SLOT_ROLE, SX>), grid, block, 0, \
                       s, a);                                                                   \
    break;                                                                                      \
  case M | SLOT_ROLE | SLOT_FIRST:                                                              \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | SLOT_ROLE | SLOT_FIRST, SX>),    \
                       grid, block, 0, s, a);                                                   \
    break;                                                                                      \
  case M | SLOT_ROLE | SLOT_LAST:                                                               \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | SLOT_ROLE | SLOT_LAST, SX>),     \
                       grid, block, 0, s, a);                                                   \
    break;                                                                                      \
  case M | SLOT_ROLE | SLOT_FIRST | SLOT_LAST:                                                  \
    hipLaunchKernelGGL(                                                                         \
        (axis_pass_kernel<T, PL, W, STRIDED, M | SLOT_ROLE | SLOT_FIRST | SLOT_LAST, SX>), grid,  \
        block, 0, s, a);                                                                        \
    break;
    GPE_SLOT_CASES(MODE_SLOTS_REAL)
    GPE_SLOT_CASES(MODE_SLOTS_IMAG)
#undef GPE_SLOT_CASES
    case MODE_FWD:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_FWD, SX>), grid, block, 0, s,
                         a);
      break;
    case MODE_DERIV:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_DERIV, SX>), grid, block, 0, s,
                         a);
      break;
    case MODE_OBS:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_OBS, SX>), grid, block, 0, s,
                         a);
      break;
    case MODE_PRE_IMAG_EXACT:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_PRE_IMAG_EXACT, SX>), grid,
                         block, 0, s, a);
      break;
    case MODE_POST_IMAG_RED_EXACT:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_POST_IMAG_RED_EXACT, SX>),
                         grid, block, 0, s, a);
      break;
#define GPE_STREAM_CASES(M)                                                                    \
  case M | STREAM_LOAD:                                                                        \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | STREAM_LOAD, SX>), grid, block, \
                       0, s, a);                                                               \
    break;                                                                                     \
  case M | STREAM_STORE:                                                                       \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | STREAM_STORE, SX>), grid,      \
                       block, 0, s, a);                                                        \
    break;                                                                                     \
  case M | STREAM_LOAD | STREAM_STORE:                                                         \
    hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, M | STREAM_LOAD | STREAM_STORE, SX>), \
                       grid, block, 0, s, a);                                                  \
    break;
    GPE_STREAM_CASES(MODE_PLAIN)
    GPE_STREAM_CASES(MODE_PRE_REAL)
#undef GPE_STREAM_CASES
    case MODE_POST_REAL:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_POST_REAL, SX>), grid, block,
                         0, s, a);
      break;
    case MODE_OBS_REAL:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_OBS_REAL, SX>), grid, block, 0,
                         s, a);
      break;
    case MODE_FWD_REAL:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_FWD_REAL, SX>), grid, block, 0,
                         s, a);
      break;
    default:
      hipLaunchKernelGGL((axis_pass_kernel<T, PL, W, STRIDED, MODE_GENERIC, SX>), grid, block, 0,
                         s, a);
  }
}

template <typename T, int N, typename SX, class PL>
hipError_t launch_np(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  const dim3 grid((unsigned)sh.blocks, (unsigned)(a.slots ? a.nslots : 1)), block((unsigned)sh.threads);
  constexpr int W16 = fit_w(N, (int)(2 * sizeof(T)), 16, PL::TPL);
  if (!sh.strided) {
    launch_mode<T, PL, contig_lines<PL>(), false, SX>(a, mode, grid, block, s);
  } else if (sh.W == 32) {
    // two 16-column halves: the plain step pass with FP32 storage only
    if constexpr (sizeof(SX) == 4 && N >= 256 && W16 == 16) {
      if (base_mode(mode) != MODE_PLAIN || a.trans) return hipErrorInvalidValue;
      launch_halves<T, PL, SX>(a, mode, grid, block, s);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (sh.W == 4) {
    // 4-line tiles: rotating passes only (rows of 4 sites)
    if constexpr (N >= 128) {
      if (!a.trans) return hipErrorInvalidValue;
      launch_mode<T, PL, 4, true, SX>(a, mode, grid, block, s);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (sh.W == 8) {
    launch_mode<T, PL, 8, true, SX>(a, mode, grid, block, s);
  } else if (sh.W == 16 && W16 == 16) {
    launch_mode<T, PL, (W16 == 16 ? 16 : 8), true, SX>(a, mode, grid, block, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N, typename SX>
hipError_t launch_n(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  if constexpr (N == 1024) {
    if (a.plan == 1) return launch_np<T, N, SX, typename PlanAlt<N>::type>(a, sh, mode, s);
  }
  return launch_np<T, N, SX, typename PlanFor<N>::type>(a, sh, mode, s);
}

template <typename T, typename SX = T>
hipError_t launch_t(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  switch (sh.N) {
    case 8: return launch_n<T, 8, SX>(a, sh, mode, s);
    case 16: return launch_n<T, 16, SX>(a, sh, mode, s);
    case 32: return launch_n<T, 32, SX>(a, sh, mode, s);
    case 64: return launch_n<T, 64, SX>(a, sh, mode, s);
    case 128: return launch_n<T, 128, SX>(a, sh, mode, s);
    case 256: return launch_n<T, 256, SX>(a, sh, mode, s);
    case 512: return launch_n<T, 512, SX>(a, sh, mode, s);
    case 1024: return launch_n<T, 1024, SX>(a, sh, mode, s);
    default: return hipErrorInvalidValue;
  }
}

int tpl_of(int N, int plan);

}  // namespace pass
}  // namespace gpe
