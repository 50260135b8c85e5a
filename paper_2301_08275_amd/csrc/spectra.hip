// |k|-shell spectra (feature list: particle-number, compressible and
// incompressible kinetic-energy spectra).
//
// The spectra of Z_j = u_j + i w_j (two real fields packed in one complex FFT)
// are unpacked per wavenumber from Z_j(k) and Z_j(-k):
//   U_j(k) = (Z_j(k) + conj(Z_j(-k))) / 2,  W_j(k) = (Z_j(k) - conj(Z_j(-k))) / (2i),
// U is split into k (k.U)/|k|^2 (compressible) and the rest (incompressible;
// k = 0 belongs there), and |.|^2 is summed per shell round(|k|/dk).  Each
// workgroup keeps its histogram in LDS (FP64 atomics) and writes it out; a
// second kernel adds the workgroup histograms in a fixed order.
#include "gpe_kernels.h"

namespace gpe {
namespace {

constexpr int kShellThreads = 256;
constexpr int kShellMaxBlocks = 1024;

template <typename T>
struct alignas(2 * sizeof(T)) cxs {
  T x, y;
};

__device__ __forceinline__ long mode_of(int i, int n) { return i < n / 2 ? i : i - n; }

template <typename T>
__global__ void __launch_bounds__(kShellThreads) shell_kernel(const ShellArgs a) {
  extern __shared__ double hist[];  // 4 * nbins
  const int nb = a.nbins;
  for (int i = threadIdx.x; i < 4 * nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const long long sites = (long long)n0 * n1 * n2;
  const cxs<T> *f0 = static_cast<const cxs<T> *>(a.f[0]);
  const cxs<T> *f1 = static_cast<const cxs<T> *>(a.f[1]);
  const cxs<T> *f2 = static_cast<const cxs<T> *>(a.f[2]);
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < sites;
       s += (long long)gridDim.x * blockDim.x) {
    const int i2 = (int)(s % n2);
    const long long r = s / n2;
    const int i1 = (int)(r % n1), i0 = (int)(r / n1);
    const long m0 = mode_of(i0, n0), m1 = mode_of(i1, n1), m2 = mode_of(i2, n2);
    const double k0 = a.kscale[0] * m0, k1 = a.kscale[1] * m1, k2 = a.kscale[2] * m2;
    const double kk = k0 * k0 + k1 * k1 + k2 * k2;
    int bin;
    if (a.integer_shells) {
      const long M = m0 * m0 + m1 * m1 + m2 * m2;
      long q = (long)sqrt((double)M);
      while ((2 * q + 1) * (2 * q + 1) <= 4 * M) ++q;
      while (q > 0 && 4 * M < (2 * q - 1) * (2 * q - 1)) --q;
      bin = (int)q;
    } else {
      bin = (int)floor(sqrt(kk) / a.dk + 0.5);
    }
    if (bin >= nb) bin = nb - 1;  // unreachable for the shell count used
    if (a.kind == 0) {
      const cxs<T> v = f0[s];
      atomicAdd(&hist[bin], a.w * ((double)v.x * v.x + (double)v.y * v.y));
    } else {
      const long long ms = (((long long)((n0 - i0) % n0) * n1 + (n1 - i1) % n1) * n2 + (n2 - i2) % n2);
      const double kv[3] = {k0, k1, k2};
      const cxs<T> *fs[3] = {f0, f1, f2};
      double ur[3] = {0, 0, 0}, ui[3] = {0, 0, 0}, qsum = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (!fs[j]) continue;
        const cxs<T> zp = fs[j][s], zm = fs[j][ms];
        ur[j] = 0.5 * ((double)zp.x + (double)zm.x);
        ui[j] = 0.5 * ((double)zp.y - (double)zm.y);
        const double wr = 0.5 * ((double)zp.y + (double)zm.y);
        const double wi = -0.5 * ((double)zp.x - (double)zm.x);
        qsum += wr * wr + wi * wi;
      }
      double csum = 0, isum = 0;
      if (kk > 0) {
        const double pr = (kv[0] * ur[0] + kv[1] * ur[1] + kv[2] * ur[2]) / kk;
        const double pi = (kv[0] * ui[0] + kv[1] * ui[1] + kv[2] * ui[2]) / kk;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double cr = kv[j] * pr, ci = kv[j] * pi;
          csum += cr * cr + ci * ci;
          isum += (ur[j] - cr) * (ur[j] - cr) + (ui[j] - ci) * (ui[j] - ci);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) isum += ur[j] * ur[j] + ui[j] * ui[j];
      }
      atomicAdd(&hist[nb + bin], 0.5 * a.w * csum);
      atomicAdd(&hist[2 * nb + bin], 0.5 * a.w * isum);
      atomicAdd(&hist[3 * nb + bin], 0.5 * a.w * qsum);
    }
  }
  __syncthreads();
  double *out = a.partial + (long long)blockIdx.x * 4 * nb;
  for (int i = threadIdx.x; i < 4 * nb; i += blockDim.x) out[i] = hist[i];
}

__global__ void sum_columns_kernel(const double *__restrict__ partial, long long count, int len,
                                   double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0;
  for (long long b = 0; b < count; ++b) s += partial[b * len + i];
  out[i] = s;
}

}  // namespace

int shell_blocks(long long sites) {
  long long b = (sites + kShellThreads - 1) / kShellThreads;
  return (int)(b < kShellMaxBlocks ? (b < 1 ? 1 : b) : kShellMaxBlocks);
}

hipError_t launch_shells(int precision, const ShellArgs &a, hipStream_t s) {
  const long long sites = (long long)a.n[0] * a.n[1] * a.n[2];
  const int blocks = shell_blocks(sites);
  const size_t lds = 4 * (size_t)a.nbins * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (state_f32(precision))  // the packed fields are stored like the state
    hipLaunchKernelGGL(shell_kernel<float>, dim3(blocks), dim3(kShellThreads), lds, s, a);
  else
    hipLaunchKernelGGL(shell_kernel<double>, dim3(blocks), dim3(kShellThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_sum_columns(const double *partial, long long count, int len, double *out,
                              hipStream_t s) {
  hipLaunchKernelGGL(sum_columns_kernel, dim3((len + 255) / 256), dim3(256), 0, s, partial, count,
                     len, out);
  return hipGetLastError();
}

}  // namespace gpe
